"""Pins of the MLP oracle: finite differences, complex step, closed forms."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_1807_09807_amd import meshgen

RNG = np.random.default_rng(7)


def _layers():
    return [(RNG.standard_normal((k, n)) / math.sqrt(k), 0.1 * RNG.standard_normal(n)) for k, n in M.LAYERS]


def test_parameter_count():
    assert M.N_PARAMS == 10706


def test_gelu_closed_forms_and_derivative():
    assert M.gelu(0.0) == 0.0
    assert M.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-15)     # Phi(1)
    z = np.linspace(-4, 4, 17)
    np.testing.assert_allclose(M.gelu(z) - M.gelu(-z), z, atol=1e-15)      # Phi(z) + Phi(-z) = 1
    h = 1e-30
    cs = np.imag(M.gelu(z + 1j * h)) / h
    np.testing.assert_allclose(M.gelu_prime(z), cs, rtol=1e-14, atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, math.pi, -2.0 ** -130, 65504.0], np.float32)
    exp = np.array([1.0, 1.0, 1.0 + 2 ** -6, 3.140625, -2.0 ** -130, 65536.0])
    np.testing.assert_array_equal(M.bf16_round(vals), exp)


def test_backward_matches_finite_differences():
    layers = _layers()
    X = RNG.standard_normal((7, 18))
    dY = RNG.standard_normal((7, 18))
    Y, cache = M.forward_layers(layers, X)
    grads, dX = M.backward_layers(layers, cache, dY)
    f = lambda L, Xi: float(np.sum(dY * M.forward_layers(L, Xi)[0]))
    eps = 1e-6
    for li in range(4):
        for which in (0, 1):
            arr = layers[li][which]
            idx = [tuple(RNG.integers(0, s) for s in arr.shape) for _ in range(5)]
            for ix in idx:
                Lp = [(W.copy(), b.copy()) for W, b in layers]
                Lm = [(W.copy(), b.copy()) for W, b in layers]
                Lp[li][which][ix] += eps
                Lm[li][which][ix] -= eps
                fd = (f(Lp, X) - f(Lm, X)) / (2 * eps)
                assert grads[li][which][ix] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    for _ in range(5):
        i, j = RNG.integers(0, 7), RNG.integers(0, 18)
        Xp, Xm = X.copy(), X.copy()
        Xp[i, j] += eps
        Xm[i, j] -= eps
        assert dX[i, j] == pytest.approx((f(layers, Xp) - f(layers, Xm)) / (2 * eps), rel=1e-6, abs=1e-8)


def test_mse_gradient():
    Y, L = RNG.standard_normal((5, 18)), RNG.standard_normal((5, 18))
    loss, dY = M.mse_grad(Y, L)
    assert loss == pytest.approx(np.mean((Y - L) ** 2), rel=1e-14)
    eps = 1e-7
    Yp = Y.copy()
    Yp[2, 3] += eps
    assert dY[2, 3] == pytest.approx((M.mse_grad(Yp, L)[0] - loss) / eps, rel=1e-5)


def test_adam_first_step_is_signed_lr():
    th, g = RNG.standard_normal(50), RNG.standard_normal(50)
    new, m, v = M.adam_step(th, np.zeros(50), np.zeros(50), g, 1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(new, th - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_features_and_labels_closed_forms():
    mesh = meshgen.box_mesh(2, 3, 2)
    X = M.features(mesh.x_grid, mesh.elem_node, mesh.h)
    ref = np.concatenate([np.tile([-0.5, 0.0, 0.5], 3), np.repeat([-0.5, 0.0, 0.5], 3)])
    np.testing.assert_allclose(X, np.broadcast_to(ref, X.shape), atol=1e-14)
    L = M.labels(mesh.x_grid, mesh.x_grid + np.array([[0.3], [-0.2]]), mesh.elem_node, mesh.h)
    assert np.max(np.abs(L)) < 1e-14                       # a translation is unobservable


def test_proposal_closed_forms():
    mesh = meshgen.box_mesh(2, 4, 2)
    x = mesh.x_grid
    # affine displacement fields are invisible to the per-element proposal
    A = np.array([[0.02, 0.01], [-0.03, 0.015]])
    xs = x + A @ x + 0.1
    out = M.propose(x, M.labels(x, xs, mesh.elem_node, mesh.h), mesh.elem_node, mesh.h, mesh.fixed)
    np.testing.assert_allclose(out, x, atol=1e-15)
    # one element-interior node moved by delta: it gets 8/9 of it back, the
    # element's free vertices -delta/36 (4 elements each), edge nodes -delta/18
    m = mesh.n * 2 + 1
    e = 1 + 4 * 1                          # element (1, 1)
    center = mesh.elem_node[e, 4]
    delta = np.array([0.01, -0.02])
    xs = x.copy()
    xs[:, center] += delta
    out = M.propose(x, M.labels(x, xs, mesh.elem_node, mesh.h), mesh.elem_node, mesh.h, mesh.fixed)
    np.testing.assert_allclose(out[:, center] - x[:, center], 8 / 9 * delta, atol=1e-15)
    v = mesh.elem_node[e, 0]
    np.testing.assert_allclose(out[:, v] - x[:, v], -delta / 36, atol=1e-15)
    ed = mesh.elem_node[e, 1]
    np.testing.assert_allclose(out[:, ed] - x[:, ed], -delta / 18, atol=1e-15)
