"""Pins of the oracle's Hessian diagonal and inner solvers to references
outside the oracle: the diagonal against the (pinned) Hessian action on
unit vectors, MINRES against scipy's implementation and against a direct
solve, preconditioned truncated CG against a direct solve and its
unpreconditioned special case, and the Newton variants against the known
minimizer of the 8x8 workload (Sections 3.4 and 5)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen


def _tiny(dim, n, p, Q, metric, W0=None, noise=0.15, seed=5):
    mesh = meshgen.box_mesh(dim, n, p)
    W = mesh.h * (np.eye(dim) if W0 is None else np.asarray(W0))
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, W)
    x = meshgen.perturb(mesh, noise, seed, bad_elements=prob.bad_elements)
    return mesh, prob, x


@pytest.mark.parametrize("dim,n,p,Q,metric,W0", [
    (2, 2, 2, 3, 2, None),
    (2, 2, 3, 4, 7, ((1.0, 0.3), (-0.2, 1.2))),
    (3, 1, 2, 3, 303, None),
    (3, 2, 1, 2, 302, ((1.0, 0.2, 0.0), (0.0, 1.1, 0.3), (0.1, 0.0, 0.9))),
])
def test_hessian_diagonal_is_unit_vector_action(dim, n, p, Q, metric, W0):
    """diag(H)_k = (H e_k)_k for every DOF, boundary included."""
    mesh, prob, x = _tiny(dim, n, p, Q, metric, W0)
    D = prob.hessian_diagonal(x).ravel()
    ref = np.empty(x.size)
    for k in range(x.size):
        e = np.zeros(x.size)
        e[k] = 1.0
        ref[k] = prob.hessian_apply(x, e.reshape(x.shape)).ravel()[k]
    assert np.max(np.abs(D - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_hessian_diagonal_at_grid_closed_form():
    """On the unperturbed 1-element Q1 square with mu_2 and W = I, the
    second variation at T = I is 2 |dev sym E|^2 (deviatoric elasticity):
    for a unit move of one corner along x, E = e_0 (grad w)^T with
    grad w = (+-(1 - s1), +-(1 - s0)) (bilinear basis), so
    dev sym E has entries (+-g0/2, g1/2; g1/2, -+g0/2) and the integrand is
    2 (g0^2/2 + g1^2/2) = g0^2 + g1^2, whose integral over [0,1]^2 is 2/3."""
    mesh = meshgen.box_mesh(2, 1, 1)
    prob = O.Problem(2, 1, 2, mesh.elem_node, 2, np.eye(2))
    D = prob.hessian_diagonal(mesh.x_grid * 1.0)
    # mesh of one element of size 1: W = I gives T = I at the grid
    np.testing.assert_allclose(D, np.full(D.shape, 2.0 / 3.0), rtol=1e-14)


def _sym_indefinite(n, n_neg, seed):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.concatenate([rng.uniform(-3.0, -0.5, n_neg), rng.uniform(0.5, 5.0, n - n_neg)])
    return (Qm * ev) @ Qm.T, rng.standard_normal(n)


@pytest.mark.parametrize("precond", [False, True])
def test_minres_matches_scipy_iterates(precond):
    """Every MINRES iterate (k = 1..12) equals scipy.sparse.linalg.minres
    stopped after k iterations, on a symmetric indefinite matrix, with and
    without an SPD diagonal preconditioner (scipy's M applies M^{-1})."""
    A, b = _sym_indefinite(30, 8, 1)
    minv = 1.0 / np.abs(np.diag(A)) if precond else None
    M = np.diag(minv) if precond else None
    for k in range(1, 13):
        d, it = O.minres(lambda v: A @ v, b, 0.0, k, minv)
        ref, _ = spla.minres(A, b, maxiter=k, rtol=0.0, M=M)
        assert it == k
        assert np.max(np.abs(d - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("precond", [False, True])
def test_minres_converges_to_solution(precond):
    A, b = _sym_indefinite(40, 10, 2)
    minv = 1.0 / np.abs(np.diag(A)) if precond else None
    d, it = O.minres(lambda v: A @ v, b, 1e-13, 500, minv)
    x = np.linalg.solve(A, b)
    assert it < 500
    assert np.max(np.abs(d - x)) <= 1e-10 * np.max(np.abs(x))


def test_minres_residual_estimate_is_residual():
    """Unpreconditioned, |phibar_k| is the 2-norm of b - A d_k: stopping at
    rtol leaves |b - A d| <= rtol |b| (to rounding)."""
    A, b = _sym_indefinite(40, 10, 3)
    for rtol in (1e-1, 1e-3, 1e-6):
        d, it = O.minres(lambda v: A @ v, b, rtol, 500)
        r = np.linalg.norm(b - A @ d)
        assert r <= rtol * np.linalg.norm(b) * (1 + 1e-8)
        d1, _ = O.minres(lambda v: A @ v, b, 0.0, it - 1)
        assert np.linalg.norm(b - A @ d1) > rtol * np.linalg.norm(b)


def test_preconditioned_cg_solves_spd():
    rng = np.random.default_rng(4)
    Qm, _ = np.linalg.qr(rng.standard_normal((50, 50)))
    A = (Qm * rng.uniform(0.1, 10.0, 50)) @ Qm.T + np.diag(rng.uniform(0.0, 50.0, 50))
    g = rng.standard_normal(50)
    minv = 1.0 / np.diag(A)
    d, it, neg = O.truncated_cg(lambda v: A @ v, g, 1e-13, 500, minv)
    x = np.linalg.solve(A, -g)
    assert not neg and it < 500
    assert np.max(np.abs(d - x)) <= 1e-10 * np.max(np.abs(x))
    # a unit preconditioner is plain CG, iterate by iterate
    for k in (1, 3, 7):
        a, _, _ = O.truncated_cg(lambda v: A @ v, g, 0.0, k, np.ones(50))
        b, _, _ = O.truncated_cg(lambda v: A @ v, g, 0.0, k)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.max(np.abs(b)))


def test_preconditioned_cg_first_step_negative_curvature():
    """Non-positive curvature at the first step returns -M^{-1} g."""
    A = -np.eye(4)
    g = np.array([1.0, -2.0, 3.0, 0.5])
    minv = np.array([0.5, 2.0, 1.0, 4.0])
    d, it, neg = O.truncated_cg(lambda v: A @ v, g, 1e-10, 10, minv)
    assert neg and it == 1
    np.testing.assert_array_equal(d, -minv * g)


def test_shifted_cg_positive_definite_is_cg():
    """With H positive definite and a positive diagonal no shift is made:
    the direction is CG's solution of H d = -g (numpy.linalg.solve)."""
    rng = np.random.default_rng(6)
    Qm, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    A = (Qm * rng.uniform(0.5, 20.0, 40)) @ Qm.T
    g = rng.standard_normal(40)
    d, it, nshift, tau = O.shifted_cg(lambda v: A @ v, g, 1e-13, 400, np.diag(A))
    assert nshift == 0 and tau == 0.0
    x = np.linalg.solve(A, -g)
    assert np.max(np.abs(d - x)) <= 1e-10 * np.max(np.abs(x))


@pytest.mark.parametrize("neg_diag", [False, True])
def test_shifted_cg_indefinite(neg_diag):
    """An indefinite H (smallest eigenvalue -3): tau follows Nocedal and
    Wright's Algorithm 3.3 -- tau_0 = 0 for a positive diagonal, else
    beta - min diag; then tau <- max(2 tau, beta) -- until H + tau I is
    positive definite, and the direction solves (H + tau I) d = -g, so
    g . d < 0."""
    rng = np.random.default_rng(7)
    Qm, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    ev = np.concatenate([[-3.0, -0.5], rng.uniform(1.0, 8.0, 28)])
    A = (Qm * ev) @ Qm.T
    if neg_diag:
        A[4, 4] = -2.0                     # a negative diagonal entry sets tau_0 = beta - min diag
    g = rng.standard_normal(30)
    diag = np.diag(A)
    beta = 1e-3 * np.mean(np.abs(diag))
    d, it, nshift, tau = O.shifted_cg(lambda v: A @ v, g, 1e-13, 400, diag)
    lam_min = np.linalg.eigvalsh(A)[0]
    # the sequence of shifts tried, by the rule
    seq = [0.0 if diag.min() > 0 else -diag.min() + beta]
    while len(seq) <= nshift:
        seq.append(max(2.0 * seq[-1], beta))
    assert tau == seq[-1]
    assert tau > -lam_min                  # H + tau I is positive definite ...
    assert nshift == 0 or seq[-2] < -lam_min + 1e-12   # ... and the shift before was not (up to CG's test)
    x = np.linalg.solve(A + tau * np.eye(30), -g)
    assert np.max(np.abs(d - x)) <= 1e-9 * np.max(np.abs(x))
    assert float(np.dot(g, d)) < 0.0


def test_jacobi_inverse():
    m = np.array([1.0, 1.0, 0.0, 1.0])
    D = np.array([-4.0, 2.0, 7.0, 0.0])
    np.testing.assert_array_equal(O.jacobi_inverse(D, m), [0.25, 0.5, 1.0, 1.0])


@pytest.mark.parametrize("inner,precond", [("minres", "none"), ("minres", "jacobi"), ("cg", "jacobi"),
                                          ("shifted_cg", "none"), ("shifted_cg", "jacobi")])
def test_newton_variants_reach_grid(inner, precond):
    """The Q2 mu_2 workload on 5x5 elements: with each inner solver and
    preconditioner Newton returns to the unperturbed grid, the known
    minimizer F* = 0.  (MINRES directions on the indefinite early Hessians
    need not descend; the 1.2-growth line search lets F rise for a while,
    so these runs take more Newton steps than truncated CG.)"""
    w = meshgen.WORKLOADS["q2_square_8"]
    mesh = meshgen.box_mesh(2, 5, w["p"])
    prob = O.Problem(2, w["p"], w["Q"], mesh.elem_node, w["metric"], mesh.h * np.eye(2))
    x0 = meshgen.perturb(mesh, w["noise"], w["seed"], bad_elements=prob.bad_elements)
    opts = O.NewtonOptions(max_it=60, cg_rtol=1e-10, inner=inner, precond=precond)
    x, rep = O.newton_solve(prob, x0, mesh.fixed, opts)
    assert rep.stop == O.STOP_CONVERGED
    assert np.max(np.abs(x - mesh.x_grid)) < 1e-9 * mesh.h
    assert rep.F < 1e-14 * rep.F0


def test_newton_rejects_unknown_solver():
    mesh, prob, x = _tiny(2, 2, 2, 3, 2)
    with pytest.raises(ValueError):
        O.newton_solve(prob, x, mesh.fixed, O.NewtonOptions(inner="gmres"))
    with pytest.raises(ValueError):
        O.newton_solve(prob, x, mesh.fixed, O.NewtonOptions(precond="ilu"))


def test_w3_sizes_affine_mesh():
    """On x = M x_grid every point has A = M h-scaled: det A = det M h^d, so
    the W_3 sizes are (det M)^(1/d) h exactly."""
    for dim, M in ((2, np.array([[1.2, 0.3], [-0.1, 0.9]])),
                   (3, np.array([[1.1, 0.2, 0.0], [0.0, 0.9, 0.1], [0.2, 0.0, 1.3]]))):
        mesh = meshgen.box_mesh(dim, 2, 2)
        prob = O.Problem(dim, 2, 3, mesh.elem_node, 303 if dim == 3 else 2, mesh.h * np.eye(dim))
        s = prob.point_sizes(M @ mesh.x_grid)
        np.testing.assert_allclose(s, np.linalg.det(M) ** (1.0 / dim) * mesh.h, rtol=1e-14)


@pytest.mark.parametrize("dim,metric", [(2, 77), (2, 9)])
def test_w3_target_reproduces_initial_sizes(dim, metric):
    """With the W_3 target of the initial mesh, det T = 1 at every point of
    that mesh: the size metric mu_77 = (tau - 1/tau)^2 / 2 and its gradient
    vanish there; for mu_9 the targets make F equal to the sum of
    w_q det A(x0) mu_9(A / s_q)."""
    mesh = meshgen.box_mesh(dim, 3, 2)
    prob0 = O.Problem(dim, 2, 4, mesh.elem_node, metric, mesh.h * np.eye(dim))
    x0 = meshgen.perturb(mesh, 0.15, 3, bad_elements=prob0.bad_elements)
    s = prob0.point_sizes(x0)
    W = s[:, :, None, None] * np.eye(dim)
    prob = O.Problem(dim, 2, 4, mesh.elem_node, metric, W)
    F, _ = prob.energy(x0)
    if metric == 77:
        assert abs(F) < 1e-28
        assert np.max(np.abs(prob.gradient(x0))) < 1e-14
    else:
        A = np.concatenate([prob._jac(x0, e0, e1) for e0, e1 in prob._chunks()])
        detA = np.linalg.det(A)
        ref = math.fsum((prob.wq[None, :] * detA * O.mu(9, A / s[:, :, None, None])).ravel())
        assert F == pytest.approx(ref, rel=1e-13)


def test_newton_sliding_boundary_returns_to_grid():
    """Boundary nodes moved along their (axis-parallel) face slide back:
    Newton with only the normal components fixed returns to the grid, and no
    node leaves its face (Section 4.1)."""
    mesh = meshgen.box_mesh(2, 4, 2, slide=True)
    prob = O.Problem(2, 2, 4, mesh.elem_node, 2, mesh.h * np.eye(2))
    x0 = meshgen.perturb(mesh, 0.1, 8, bad_elements=prob.bad_elements)
    rng = np.random.default_rng(9)
    for c in range(2):   # tangential moves of the nodes on the faces with normal 1 - c
        on = mesh.fixed[1 - c].astype(bool) & ~mesh.fixed[c].astype(bool)
        x0[c, on] += rng.uniform(-0.15, 0.15, on.sum()) * mesh.h
    assert prob.element_min_det(x0).min() > 0
    x, rep = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=40, cg_rtol=1e-10))
    assert rep.stop == O.STOP_CONVERGED
    assert np.max(np.abs(x - mesh.x_grid)) < 1e-9 * mesh.h
    fx = mesh.fixed.astype(bool)
    np.testing.assert_array_equal(x[fx], x0[fx])
