"""Pins of the oracle's derivative-free solver (Section 3.4, eq. 3.3) to
references outside it: its Nelder-Mead against scipy's implementation of
the same method and against known minimizers, the node colouring against a
brute-force check, the patch quality against the (pinned) objective, a
single free node that returns to its known optimal position, monotone
sweeps, and the converged mesh against Newton's minimizer."""
import math

import numpy as np
import pytest
import scipy.optimize as so

from oracle import tmop_dfo as D
from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen


def _mesh(dim, n, p, Q, metric, noise, seed):
    mesh = meshgen.box_mesh(dim, n, p)
    W = mesh.h * np.eye(dim)
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, W)
    x0 = meshgen.perturb(mesh, noise, seed, bad_elements=prob.bad_elements) if noise else mesh.x_grid.copy()
    return mesh, prob, x0


@pytest.mark.parametrize("n", [1, 2, 3])
def test_nelder_mead_finds_quadratic_minimum(n):
    rng = np.random.default_rng(n)
    G = rng.uniform(-1, 1, (n, n))
    M = G @ G.T + n * np.eye(n)
    c = rng.uniform(-1, 1, n)
    best, fb, evals = D.nelder_mead(lambda y: float((y - c) @ M @ (y - c)), np.zeros(n), 0.3, 1e-10, 10000)
    assert np.max(np.abs(best - c)) < 1e-8 and fb < 1e-15 and evals < 10000


def test_nelder_mead_matches_scipy():
    """Same method, same initial simplex: scipy's non-adaptive Nelder-Mead
    (with its f-criterion switched off) ends at the same point of the
    Rosenbrock function."""
    rosen = lambda y: 100.0 * (y[1] - y[0] ** 2) ** 2 + (1.0 - y[0]) ** 2
    x0 = np.array([-1.2, 1.0])
    best, fb, _ = D.nelder_mead(rosen, x0, 0.1, 1e-10, 100000)
    sim = np.array([x0, x0 + [0.1, 0.0], x0 + [0.0, 0.1]])
    r = so.minimize(rosen, x0, method="Nelder-Mead",
                    options=dict(initial_simplex=sim, xatol=1e-10, fatol=np.inf, maxfev=100000, adaptive=False))
    assert np.max(np.abs(best - r.x)) < 1e-8
    assert np.max(np.abs(best - 1.0)) < 1e-8


@pytest.mark.parametrize("dim,n,p", [(2, 4, 2), (2, 3, 3), (3, 2, 2), (2, 5, 1)])
def test_node_colouring_is_valid(dim, n, p):
    mesh = meshgen.box_mesh(dim, n, p)
    colours = D.node_colouring(mesh.elem_node, mesh.n_node)
    seen = np.concatenate(colours)
    assert np.array_equal(np.sort(seen), np.arange(mesh.n_node))
    col = np.empty(mesh.n_node, dtype=np.int64)
    for c, nodes in enumerate(colours):
        col[nodes] = c
    for nodes in mesh.elem_node:                      # no two nodes of an element share a colour
        assert len(set(col[nodes])) == len(nodes)
    assert len(colours) == (p + 1) ** dim or p == 1 and len(colours) == 2 ** dim


def test_patch_quality_is_the_patch_part_of_F():
    mesh, prob, x0 = _mesh(2, 4, 2, 4, 2, 0.1, 3)
    pat = D.Patches(prob, mesh.n_node)
    c, _ = prob.pointwise(x0)
    for i in (0, 7, 40, mesh.n_node - 1):
        assert pat.quality(x0, i) == pytest.approx(math.fsum(c[pat.elems[i]].ravel()), rel=1e-14)
    # moving node i changes F by exactly the change of Q(x_i)
    i = 40
    x1 = x0.copy()
    x1[:, i] += 0.03 * mesh.h
    dF = prob.energy(x1)[0] - prob.energy(x0)[0]
    assert dF == pytest.approx(pat.quality(x1, i) - pat.quality(x0, i), rel=1e-9)
    # an inverting move gives +inf
    x2 = x0.copy()
    x2[:, i] = x0[:, i + 2]
    assert pat.quality(x2, i) == math.inf


@pytest.mark.parametrize("dim,n,p,Q,metric", [(2, 4, 2, 4, 2), (3, 2, 2, 3, 303)])
def test_single_free_node_returns_to_grid(dim, n, p, Q, metric):
    """On the uniform grid (F = 0, the minimizer of a shape metric with
    W = h I) one interior node displaced by 0.2 h, all others fixed: one
    sweep puts it back."""
    mesh, prob, _ = _mesh(dim, n, p, Q, metric, 0.0, 0)
    m = n * p + 1
    i = (m // 2) * (1 + m + (m * m if dim == 3 else 0))      # the centre node
    x = mesh.x_grid.copy()
    x[:, i] += 0.2 * mesh.h * np.array([1.0, -0.6, 0.3][:dim])
    free = np.zeros((dim, mesh.n_node), dtype=np.int64)
    free[:, i] = 1
    colours = D.node_colouring(mesh.elem_node, mesh.n_node)
    move = D.dfo_sweep(prob, D.Patches(prob, mesh.n_node), x, free, colours,
                       D.DfoOptions(xtol=1e-9, max_evals=2000))
    assert np.max(np.abs(x - mesh.x_grid)) < 1e-7 * mesh.h
    assert move == pytest.approx(0.2 * mesh.h, rel=1e-5)


def test_sweeps_decrease_F_and_reach_the_newton_minimizer():
    """Each node keeps its position unless Nelder-Mead found a lower Q, so F
    never increases over a sweep; swept to t = 1e-9 the mesh is Newton's
    minimizer (the grid) to within the Nelder-Mead tolerance."""
    mesh, prob, x0 = _mesh(2, 3, 1, 2, 2, 0.2, 5)
    opts = D.DfoOptions(t=1e-9, max_sweeps=400, xtol=1e-11, max_evals=1000)
    x = x0.copy()
    free = 1 - mesh.fixed.astype(np.int64)
    colours = D.node_colouring(mesh.elem_node, mesh.n_node)
    pat = D.Patches(prob, mesh.n_node)
    F = [prob.energy(x)[0]]
    for _ in range(opts.max_sweeps):
        m = D.dfo_sweep(prob, pat, x, free, colours, opts)
        F.append(prob.energy(x)[0])
        if m < opts.t:
            break
    # (F reaches the rounding floor of mu_2 = |T|^2 / (2 tau) - 1 near T = sI)
    assert all(b <= a + 1e-14 * abs(a) + 1e-16 for a, b in zip(F, F[1:]))
    xn, rep = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=40, cg_rtol=1e-12, atol=1e-10))
    assert rep.stop == O.STOP_CONVERGED
    assert np.max(np.abs(xn - mesh.x_grid)) < 1e-9 * mesh.h
    assert np.max(np.abs(x - xn)) < 1e-6 * mesh.h
    assert F[-1] < 1e-10 * F[0]


def test_dfo_solve_report():
    mesh, prob, x0 = _mesh(2, 4, 2, 3, 2, 0.1, 8)
    x, rep = D.dfo_solve(prob, x0, mesh.fixed, mesh.n_node, D.DfoOptions(t=1e-4, max_sweeps=30))
    assert rep.converged and rep.sweeps == len(rep.max_move) and rep.max_move[-1] < 1e-4
    assert rep.F < 0.2 * rep.F0
    np.testing.assert_array_equal(x[mesh.fixed.astype(bool)], x0[mesh.fixed.astype(bool)])
