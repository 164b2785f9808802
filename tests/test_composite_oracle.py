"""Pins of the oracle's Section 4 objectives to references outside them:

* restricted movement, first algorithm (eq. 4.2): closed forms for a rigid
  translation and for a linear displacement field (the exact integral of a
  quadratic over the box), complex-step derivatives, the diagonal against
  unit-vector actions, and the monotone effect of delta on Newton's
  displacement;
* the two-term composite metric (eq. 4.1): linearity against two plain
  problems, per-point weights against their pointwise contributions,
  complex-step derivatives;
* the replication composite (Section 4.3.2): gamma = 1 is the plain problem,
  gamma = 0 makes the initial mesh a stationary point with F = 0, and for a
  linear map M of the initial mesh the mu_98 part is the closed form
  (1 - gamma) vol |M - I|^2 / det M.
"""
import math

import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen

EPS_CS = 1e-30


def _mesh(dim, n, p, Q, metric, noise=0.12, seed=11):
    mesh = meshgen.box_mesh(dim, n, p)
    W = mesh.h * np.eye(dim)
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, W)
    x0 = meshgen.perturb(mesh, noise, seed, bad_elements=prob.bad_elements)
    return mesh, W, prob, x0


def _fresh(mesh, p, Q, metric, W):
    return O.Problem(mesh.dim, p, Q, mesh.elem_node, metric, W)


def _cs_checks(prob, x, seed):
    """g . v and H v by complex step through the objective and gradient."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1, 1, x.shape)
    g = prob.gradient(x)
    Fc, _ = prob.energy(x + 1j * EPS_CS * v)
    gv = float(np.sum(g * v))
    assert abs(Fc.imag / EPS_CS - gv) <= 1e-12 * max(abs(gv), np.sum(np.abs(g * v)))
    Hv = prob.hessian_apply(x, v)
    Hv_cs = prob.gradient(x + 1j * EPS_CS * v).imag / EPS_CS
    assert np.max(np.abs(Hv - Hv_cs)) <= 1e-12 * np.max(np.abs(Hv_cs))


def _diag_by_unit_vectors(prob, x):
    ref = np.empty(x.size)
    for k in range(x.size):
        e = np.zeros(x.size)
        e[k] = 1.0
        ref[k] = prob.hessian_apply(x, e.reshape(x.shape)).ravel()[k]
    return ref


# ----------------------------------------------------------------- eq. 4.2

@pytest.mark.parametrize("dim,n,p,Q,metric", [(2, 3, 2, 4, 2), (2, 2, 3, 5, 9), (3, 2, 2, 3, 303)])
def test_restriction_translation_closed_form(dim, n, p, Q, metric):
    """x = x_init + t: A is unchanged and x(q) - x_init(q) = t at every
    point (the basis is a partition of unity), so the penalty is
    delta |t|^2 sum_E sum_q w_q det W = delta |t|^2 n_elem h^d."""
    mesh, W, prob, x0 = _mesh(dim, n, p, Q, metric)
    plain = _fresh(mesh, p, Q, metric, W)
    delta = 3.7
    prob.set_restriction(delta, x0)
    t = np.array([0.3, -0.45, 0.2][:dim])
    x = x0 + t[:, None]
    F, _ = prob.energy(x)
    F0, _ = plain.energy(x0)
    expect = delta * float(t @ t) * mesh.n_elem * mesh.h ** dim
    assert F - F0 == pytest.approx(expect, rel=1e-12)
    assert prob.energy(x0)[0] == F0          # no displacement, no penalty


@pytest.mark.parametrize("dim,n,p,Q", [(2, 3, 2, 3), (2, 2, 3, 4), (3, 2, 2, 2)])
def test_restriction_linear_field_closed_form(dim, n, p, Q):
    """u = x - x_init = L x_grid is linear, so with W = h I the penalty is
    delta * integral over the unit box of |L y|^2, exact for Q >= 2:
    sum_c (sum_k L_ck^2 / 3 + sum_{k != l} L_ck L_cl / 4)."""
    mesh, W, prob, x0 = _mesh(dim, n, p, Q, 2 if dim == 2 else 303)
    plain = _fresh(mesh, p, Q, prob.metric, W)
    L = np.random.default_rng(3).uniform(-0.2, 0.2, (dim, dim))
    x = x0 + L @ mesh.x_grid
    delta = 0.9
    prob.set_restriction(delta, x0)
    exact = sum(sum(L[c, k] ** 2 / 3.0 for k in range(dim))
                + sum(L[c, k] * L[c, l] / 4.0 for k in range(dim) for l in range(dim) if k != l)
                for c in range(dim))
    Fr, _ = prob.energy(x)
    Fp, _ = plain.energy(x)
    assert Fr - Fp == pytest.approx(delta * exact, rel=1e-11)


@pytest.mark.parametrize("dim,n,p,Q,metric", [(2, 2, 2, 3, 2), (3, 1, 2, 3, 302)])
def test_restriction_derivatives(dim, n, p, Q, metric):
    mesh, W, prob, x0 = _mesh(dim, n, p, Q, metric)
    x = meshgen.perturb(mesh, 0.05, 12, base=x0, bad_elements=prob.bad_elements)
    prob.set_restriction(25.0, x0)
    _cs_checks(prob, x, 4)
    D = prob.hessian_diagonal(x).ravel()
    ref = _diag_by_unit_vectors(prob, x)
    assert np.max(np.abs(D - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("dim,n,p,Q", [(2, 3, 2, 4), (3, 2, 3, 4)])
def test_field_at_points_is_the_position(dim, n, p, Q):
    """On the unperturbed grid the field x(q) of eq. 2.1 is the physical
    point (e_c + s_(q_c)) / n of element e, with the point index
    q = q0 + Q q1 (+ Q^2 q2) and the lexicographic element index."""
    mesh, W, prob, _ = _mesh(dim, n, p, Q, 2 if dim == 2 else 303)
    xq = prob._field_at_points(mesh.x_grid, 0, mesh.n_elem)
    s, _ = O.gauss_legendre(Q)
    e = np.arange(mesh.n_elem)
    q = np.arange(Q ** dim)
    for c in range(dim):
        ec = (e // n ** c) % n
        qc = (q // Q ** c) % Q
        np.testing.assert_allclose(xq[:, :, c], (ec[:, None] + s[qc][None, :]) / n, rtol=0, atol=4e-15)


def test_restriction_mass_is_symmetric_and_sums_to_volume():
    """H of the penalty alone is 2 delta M per component: symmetric, and
    1^T M 1 = sum_E sum_q w_q det W (the target volume)."""
    mesh, W, prob, x0 = _mesh(2, 3, 2, 4, 2)
    plain = _fresh(mesh, 2, 4, 2, W)
    delta = 0.5
    prob.set_restriction(delta, x0)
    rng = np.random.default_rng(9)
    a, b = rng.uniform(-1, 1, x0.shape), rng.uniform(-1, 1, x0.shape)
    Ma = (prob.hessian_apply(x0, a) - plain.hessian_apply(x0, a)) / (2 * delta)
    Mb = (prob.hessian_apply(x0, b) - plain.hessian_apply(x0, b)) / (2 * delta)
    assert float(np.sum(Ma * b)) == pytest.approx(float(np.sum(Mb * a)), rel=1e-12)
    one = np.zeros_like(x0)
    one[0] = 1.0
    M1 = (prob.hessian_apply(x0, one) - plain.hessian_apply(x0, one)) / (2 * delta)
    assert float(np.sum(M1[0])) == pytest.approx(mesh.n_elem * mesh.h ** 2, rel=1e-12)
    assert np.max(np.abs(M1[1])) <= 1e-14


def _displacement(mesh, W, x, x0):
    """integral over the target elements of |x - x_init|^2 (eq. 4.2 with
    delta = 1), from the difference of a restricted and a plain problem"""
    r = _fresh(mesh, 2, 4, 2, W)
    r.set_restriction(1.0, x0)
    return r.energy(x)[0] - _fresh(mesh, 2, 4, 2, W).energy(x)[0]


def test_restriction_limits_displacement():
    """Section 4.3.1: the movement away from the initial mesh (measured as
    the penalty's integral) shrinks as delta grows; delta = 0 is the plain
    problem."""
    mesh, W, prob0, x0 = _mesh(2, 5, 2, 4, 2, noise=0.15, seed=21)
    disp, Fs = [], []
    for delta in (0.0, 10.0, 1000.0):
        prob = _fresh(mesh, 2, 4, 2, W)
        prob.set_restriction(delta, x0)
        x, rep = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=40, cg_rtol=1e-10))
        assert rep.stop == O.STOP_CONVERGED
        disp.append(_displacement(mesh, W, x, x0))
        Fs.append(rep.F)
    plain_x, plain_rep = O.newton_solve(prob0, x0, mesh.fixed, O.NewtonOptions(max_it=40, cg_rtol=1e-10))
    assert Fs[0] == pytest.approx(plain_rep.F, rel=1e-9, abs=1e-18)
    assert disp[0] > disp[1] > disp[2]
    assert disp[2] < 0.2 * disp[0]


# ----------------------------------------------------------------- eq. 4.1

@pytest.mark.parametrize("dim,n,p,Q,m1,m2", [(2, 3, 2, 4, 1, 77), (2, 2, 3, 5, 2, 9), (3, 2, 2, 3, 303, 302)])
def test_combo_is_linear_in_the_terms(dim, n, p, Q, m1, m2):
    """eta_1 mu_1(A W^-1) + eta_2 mu_2(A W_2^-1) with constant weights equals
    eta_1 F_1 + eta_2 F_2 of two plain problems, and so do g and Hv."""
    mesh, W, prob, x0 = _mesh(dim, n, p, Q, m1)
    W2 = 0.8 * mesh.h * np.eye(dim)
    W2[0, 1] = 0.1 * mesh.h
    P1 = _fresh(mesh, p, Q, m1, W)
    P2 = _fresh(mesh, p, Q, m2, W2)
    eta1, eta2 = 0.7, 2.5
    prob.set_combo(m2, W2, eta1, eta2)
    v = np.random.default_rng(5).uniform(-1, 1, x0.shape)
    F = prob.energy(x0)[0]
    assert F == pytest.approx(eta1 * P1.energy(x0)[0] + eta2 * P2.energy(x0)[0], rel=1e-13)
    for op in (lambda P: P.gradient(x0), lambda P: P.hessian_apply(x0, v), lambda P: P.hessian_diagonal(x0)):
        ref = eta1 * op(P1) + eta2 * op(P2)
        assert np.max(np.abs(op(prob) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_combo_per_point_weights():
    """A per-point eta_2 weighs the second metric's pointwise contributions
    (the space-dependent weight of Section 5.2.4)."""
    mesh, W, prob, x0 = _mesh(2, 3, 3, 4, 1)
    W2 = 0.5 * mesh.h * np.eye(2)
    eta2 = np.random.default_rng(6).uniform(0.2, 1.2, (mesh.n_elem, 16))
    prob.set_combo(77, W2, 1.0, eta2)
    c1, _ = _fresh(mesh, 3, 4, 1, W).pointwise(x0)
    c2, _ = _fresh(mesh, 3, 4, 77, W2).pointwise(x0)
    assert prob.energy(x0)[0] == pytest.approx(math.fsum((c1 + eta2 * c2).ravel()), rel=1e-13)
    _cs_checks(prob, x0, 7)


def test_combo_validation():
    mesh, W, prob, x0 = _mesh(2, 2, 2, 3, 2)
    with pytest.raises(ValueError):
        prob.set_combo(303, np.eye(2))
    with pytest.raises(ValueError):
        prob.set_combo(77, np.diag([1.0, -1.0]))


# ----------------------------------------------------------- Section 4.3.2

def test_replication_gamma_one_is_the_plain_problem():
    mesh, W, prob, x0 = _mesh(2, 3, 2, 4, 2)
    plain = _fresh(mesh, 2, 4, 2, W)
    x = meshgen.perturb(mesh, 0.05, 3, base=x0, bad_elements=prob.bad_elements)
    prob.set_replication(1.0, x0)
    assert prob.energy(x)[0] == pytest.approx(plain.energy(x)[0], rel=1e-14)
    assert np.max(np.abs(prob.gradient(x) - plain.gradient(x))) <= 1e-14 * np.max(np.abs(plain.gradient(x)))


def test_replication_gamma_zero_keeps_the_initial_mesh():
    """gamma = 0: mu' = mu_98(A A_init^-1) is 0 at x_init, which is a
    stationary point (dmu_98 = 0 at T = I); Newton does not move."""
    mesh, W, prob, x0 = _mesh(2, 4, 2, 4, 2)
    prob.set_replication(0.0, x0)
    F, _ = prob.energy(x0)
    g = prob.gradient(x0)
    assert abs(F) <= 1e-28
    assert np.max(np.abs(g)) <= 1e-13
    x, rep = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=5, atol=1e-12))
    assert rep.iters == 0 and np.array_equal(x, x0)


@pytest.mark.parametrize("dim,metric,gamma", [(2, 9, 0.0), (2, 9, 0.3), (2, 9, 0.8), (3, 303, 0.0), (3, 302, 0.6)])
def test_replication_linear_map_closed_form(dim, metric, gamma):
    """x = M x_init: T_0 = M at every point, so the mu_98 part is
    (1 - gamma) |M - I|^2 / det M times the target volume n_elem h^d."""
    mesh, W, prob, x0 = _mesh(dim, 3 if dim == 2 else 2, 2, 4 if dim == 2 else 3, metric)
    plain = _fresh(mesh, 2, 4 if dim == 2 else 3, metric, W)
    M = np.array([[1.1, 0.15, 0.05], [-0.05, 0.95, 0.1], [0.02, -0.1, 1.05]])[:dim, :dim]
    x = M @ x0
    prob.set_replication(gamma, x0)
    F = prob.energy(x)[0]
    part98 = (1 - gamma) * float(np.sum((M - np.eye(dim)) ** 2)) / np.linalg.det(M) * mesh.n_elem * mesh.h ** dim
    assert F == pytest.approx(gamma * plain.energy(x)[0] + part98, rel=1e-12)


def test_replication_3d_gamma_zero_is_stationary():
    mesh, W, prob, x0 = _mesh(3, 2, 2, 3, 303)
    prob.set_replication(0.0, x0)
    assert abs(prob.energy(x0)[0]) <= 1e-28
    assert np.max(np.abs(prob.gradient(x0))) <= 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_replication_derivatives(dim):
    mesh, W, prob, x0 = _mesh(dim, 2 if dim == 2 else 1, 2, 3, 2 if dim == 2 else 302)
    x = meshgen.perturb(mesh, 0.05, 13, base=x0, bad_elements=prob.bad_elements)
    prob.set_replication(0.4, x0)
    _cs_checks(prob, x, 8)
    D = prob.hessian_diagonal(x).ravel()
    ref = _diag_by_unit_vectors(prob, x)
    assert np.max(np.abs(D - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_replication_limits_displacement():
    """Intermediate gamma mixes the fully restricted (gamma = 0) and the
    unrestricted (gamma = 1) problems: the displacement grows with gamma."""
    mesh, W, prob0, x0 = _mesh(2, 5, 2, 4, 2, noise=0.15, seed=21)
    disp = []
    for gamma in (0.2, 0.6, 1.0):
        prob = _fresh(mesh, 2, 4, 2, W)
        prob.set_replication(gamma, x0)
        x, rep = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=40, cg_rtol=1e-10))
        assert rep.stop == O.STOP_CONVERGED
        disp.append(_displacement(mesh, W, x, x0))
    assert disp[0] < disp[1] < disp[2]
