"""The learned initial guess: MLP kernels against the numpy oracle (same
BF16-valued weights, FP32 arithmetic on the GPU), the gather / merge
kernels, and what a trained network gains over plain Newton."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen
from tests._helpers import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _params(seed=3):
    from paper_1807_09807_amd import mlp as ML
    p = ML.init_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 10)
    layers = M.unpack(p)
    p = M.pack([(W * (10.0 if li == 3 else 1.0), 0.1 * rng.standard_normal(b.size)) for li, (W, b) in enumerate(layers)])
    return p.astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [1, 37, 1000])
def test_forward_matches_oracle(n):
    from paper_1807_09807_amd import mlp as ML
    p = _params()
    X = np.random.default_rng(n).uniform(-0.7, 0.7, (n, 18)).astype(np.float32)
    net = ML.MLP(p)
    Y = net.forward(_dev(X)).cpu().numpy()
    Yo, _ = M.forward(p, X)
    e = _rel(Y, Yo)
    say(f"[mlp] forward n={n}: rel err {e:.2e}")
    assert e <= 1e-5


def test_backward_matches_oracle():
    from paper_1807_09807_amd import mlp as ML
    p = _params(4)
    rng = np.random.default_rng(5)
    n = 517
    X = rng.uniform(-0.7, 0.7, (n, 18)).astype(np.float32)
    dY = rng.standard_normal((n, 18)).astype(np.float32)
    net = ML.MLP(p)
    dp, dX = net.backward(_dev(X), _dev(dY), want_dX=True)
    _, cache = M.forward(p, X)
    dpo, dXo = M.backward(p, cache, dY.astype(np.float64))
    dp = dp.cpu().numpy()
    o = 0
    for li, (k, m) in enumerate(M.LAYERS):
        for name, size in (("W", k * m), ("b", m)):
            e = _rel(dp[o:o + size], dpo[o:o + size])
            say(f"[mlp] backward d{name}{li + 1}: rel err {e:.2e}")
            assert e <= 1e-5
            o += size
    assert _rel(dX.cpu().numpy(), dXo) <= 1e-5


def test_train_step_matches_oracle_adam():
    """One step: loss value, then the Adam update of the oracle applied to
    the oracle gradient (first step: -lr sign(g) where g is not tiny)."""
    from paper_1807_09807_amd import mlp as ML
    p = _params(6)
    rng = np.random.default_rng(7)
    n = 256
    X = rng.uniform(-0.7, 0.7, (n, 18)).astype(np.float32)
    L = 0.05 * rng.standard_normal((n, 18)).astype(np.float32)
    net = ML.MLP(p)
    lr = 1e-3
    loss = net.train_step(_dev(X), _dev(L), lr, want_loss=True)
    Y, cache = M.forward(p, X)
    loss_o, dYo = M.mse_grad(Y, L.astype(np.float64))
    g, _ = M.backward(p, cache, dYo)
    assert loss == pytest.approx(loss_o, rel=1e-5)
    new_o, _, _ = M.adam_step(p.astype(np.float64), np.zeros_like(g), np.zeros_like(g), g, 1, lr)
    new = net.params()
    big = np.abs(g) > 1e-3 * np.max(np.abs(g))
    np.testing.assert_allclose(new[big], new_o[big], rtol=0, atol=1e-5 * lr + 1e-7)


def test_features_labels_propose_match_oracle():
    from paper_1807_09807_amd import mlp as ML
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(2, 16, 2)
    W = mesh.h * np.eye(2)
    prob = O.Problem(2, 2, 4, mesh.elem_node, 2, W)
    tm = meshgen.training_mesh(16, 1234, bad_elements=prob.bad_elements)
    x = tm.x
    xs = mesh.x_grid + 0.01 * np.random.default_rng(1).standard_normal(x.shape) * mesh.h
    ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 2, W, fixed=mesh.fixed)
    xd = torch.from_numpy(x).cuda()
    Xg = ML.features(ctx, xd).cpu().numpy()
    Xo = M.features(x, mesh.elem_node, mesh.h)
    assert np.max(np.abs(Xg - Xo)) <= 1e-6 * np.max(np.abs(Xo))
    Lg = ML.labels(ctx, xd, torch.from_numpy(xs).cuda()).cpu().numpy()
    Lo = M.labels(x, xs, mesh.elem_node, mesh.h)
    assert np.max(np.abs(Lg - Lo)) <= 1e-6 * np.max(np.abs(Lo))
    p = _params(8)
    net = ML.MLP(p)
    xp = ML.propose(ctx, net, xd).cpu().numpy()
    Yo, _ = M.forward(p, Xo)
    xpo = M.propose(x, Yo, mesh.elem_node, mesh.h, mesh.fixed)
    assert np.max(np.abs(xp - xpo)) <= 1e-5 * mesh.h
    fx = mesh.fixed.astype(bool)
    np.testing.assert_array_equal(xp[fx], x[fx])


def test_trained_network_gains_over_plain_newton():
    """Train on the method's own Newton solutions of 96 seeded 32^2 meshes,
    then on two unseen 64^2 meshes: the proposal lowers F below F(x0),
    Newton from it reaches the plain-Newton F_tol without the fallback, and
    it takes no more Newton iterations than plain Newton on either mesh and
    fewer in total (the gain claimed; the inner CG iterations and the wall
    time are printed, not asserted: one of the two meshes needs more CG
    iterations from the proposal).  A network whose output layer is zero
    proposes x0 itself and is never used (the fallback)."""
    from paper_1807_09807_amd import mlp as ML
    logs = []
    data = ML.generate_training_data(n_mesh=96, n=32, seed0=1000, log=say)
    say(f"[mlp] data: {data.info}")
    net, tinfo = ML.train(data, epochs=6, batch_meshes=2, lr=2e-3, seed=0, log=say)
    hist = tinfo["loss_history"]
    assert hist[-1] < hist[0]
    rows = ML.evaluate(net, n=64, seeds=(10000, 10001), log=say)
    for r in rows:
        assert r["F_proposal"] < r["F0"], "the trained proposal must lower the objective"
        assert r["used_proposal"] and not r["learned"]["fell_back_after_solve"]
        assert r["learned"]["F"] <= r["F_tol"] and r["plain"]["F"] <= r["F_tol"]
        assert r["learned"]["iters"] <= r["plain"]["iters"]
        say(f"[mlp] seed {r['seed']}: Newton {r['plain']['iters']} -> {r['learned']['iters']}, CG "
            f"{r['plain']['cg']} -> {r['learned']['cg']}, wall {r['plain']['wall_s']:.4f} -> "
            f"{r['learned']['wall_s']:.4f} s")
    gain_it = np.mean([r["plain"]["iters"] - r["learned"]["iters"] for r in rows])
    say(f"[mlp] mean Newton iterations saved: {gain_it:.2f}")
    assert gain_it > 0
    # zero-output control
    p0 = ML.init_params(0)
    p0[-64 * 18 - 18:] = 0.0
    zero = ML.MLP(p0)
    for r in ML.evaluate(zero, n=64, seeds=(10000,), log=say):
        assert not r["used_proposal"] and r["F_proposal"] == pytest.approx(r["F0"], rel=1e-12)
