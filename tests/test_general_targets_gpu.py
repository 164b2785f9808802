"""General target matrices per element and per quadrature point (Section
3.1: W may be chosen at every point, det W > 0) in the HIP library, against
the oracle with the same targets: energy, gradient, Hessian action, diagonal
and energy + gradient element by element (FP64 within 1e-12 relative, mixed
FP32 within each result's first-order rounding bound), with the displacement penalty of eq. 4.2
(whose weight det W then varies per point), Newton with non-isotropic
per-point targets against the oracle's Newton, and the set-up checks."""
import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen
from tests._helpers import mixed_tol, rel_max_err, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [  # dim, n, p, Q, metric, noise, seed, kind
    (2, 5, 2, 4, 2, 0.10, 70, "elem"),
    (2, 5, 2, 4, 2, 0.10, 70, "qp"),
    (2, 4, 3, 5, 7, 0.06, 71, "qp"),
    (2, 6, 1, 2, 9, 0.10, 72, "elem"),
    (3, 3, 2, 4, 303, 0.10, 73, "elem"),
    (3, 3, 2, 4, 303, 0.10, 73, "qp"),
    (3, 2, 3, 4, 302, 0.05, 74, "qp"),
]


def targets(mesh, Q, kind, seed):
    """h (I + 0.25 M) with M uniform in [-1, 1]: |0.25 M|_2 <= 0.75 < 1, so
    det W > 0; one per element or one per point."""
    d = mesh.dim
    shape = (mesh.n_elem,) if kind == "elem" else (mesh.n_elem, Q ** d)
    M = np.random.default_rng(seed).uniform(-1.0, 1.0, shape + (d, d))
    return mesh.h * (np.eye(d) + 0.25 * M)


def _case(dim, n, p, Q, metric, noise, seed, kind):
    mesh = meshgen.box_mesh(dim, n, p)
    prob0 = O.Problem(dim, p, Q, mesh.elem_node, metric, mesh.h * np.eye(dim))
    x = meshgen.perturb(mesh, noise, seed, bad_elements=prob0.bad_elements)
    W = targets(mesh, Q, kind, seed + 1)
    return mesh, O.Problem(dim, p, Q, mesh.elem_node, metric, W), x, W


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}d_p{c[2]}_q{c[3]}_mu{c[4]}_{c[7]}")
def setup(request):
    say(f"[general targets] case {request.param}")
    mesh, prob, x, W = _case(*request.param)
    v = np.random.default_rng(request.param[6] + 2).uniform(-1, 1, x.shape)
    F, md = prob.energy(x)
    ref = dict(F=F, md=md, g=prob.gradient(x), Hv=prob.hessian_apply(x, v), D=prob.hessian_diagonal(x),
               mtol=mixed_tol(prob, x, v, diag=True))
    return request.param, mesh, prob, x, v, W, ref


def _ctx(case, mesh, W, precision):
    from paper_1807_09807_amd import tmop as T
    dim, n, p, Q, metric = case[:5]
    return T.Context(dim, p, mesh.elem_node, mesh.n_node, Q, metric, W, fixed=mesh.fixed, precision=precision)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_general_targets(setup, precision):
    case, mesh, prob, x, v, W, ref = setup
    ctx = _ctx(case, mesh, W, precision)
    xd, vd = to_dev(x), to_dev(v)
    tol = dict(F=1e-12, min_detA=1e-12, g=1e-12, Hv=1e-12, diag=1e-12) if precision == 0 else ref["mtol"]
    F, md, st = ctx.energy(xd)
    eF = abs(F - ref["F"]) / abs(ref["F"])
    eg = rel_max_err(ctx.gradient(xd).cpu().numpy(), ref["g"])
    eh = rel_max_err(ctx.hessian_apply(xd, vd).cpu().numpy(), ref["Hv"])
    ed = rel_max_err(ctx.hessian_diagonal(xd).cpu().numpy(), ref["D"])
    Fe, mde, _, ge = ctx.energy_gradient(xd)
    say(f"  prec={precision}: F rel {eF:.2e} g {eg:.2e} Hv {eh:.2e} diag {ed:.2e} "
        f"(bars g {tol['g']:.1e} Hv {tol['Hv']:.1e})")
    assert st == 0
    assert eF <= tol["F"] and abs(Fe - ref["F"]) <= tol["F"] * abs(ref["F"])
    assert abs(md - ref["md"]) <= tol["min_detA"] * abs(ref["md"]) and md == mde
    assert eg <= tol["g"] and eh <= tol["Hv"] and ed <= tol["diag"]
    assert rel_max_err(ge.cpu().numpy(), ref["g"]) <= tol["g"]


def test_general_targets_with_penalty(setup):
    """eq. 4.2 over the target elements: the weight det W_q differs per point."""
    case, mesh, prob, x, v, W, ref = setup
    x_init = mesh.x_grid
    delta = 7.0
    prob.set_restriction(delta, x_init)
    try:
        F_o, _ = prob.energy(x)
        g_o, Hv_o, D_o = prob.gradient(x), prob.hessian_apply(x, v), prob.hessian_diagonal(x)
    finally:
        prob.set_restriction(0.0)
    ctx = _ctx(case, mesh, W, 0)
    ctx.set_restriction(delta, to_dev(x_init))
    xd, vd = to_dev(x), to_dev(v)
    F, _, st = ctx.energy(xd)
    assert st == 0 and abs(F - F_o) <= 1e-12 * abs(F_o)
    assert rel_max_err(ctx.gradient(xd).cpu().numpy(), g_o) <= 1e-12
    assert rel_max_err(ctx.hessian_apply(xd, vd).cpu().numpy(), Hv_o) <= 1e-12
    assert rel_max_err(ctx.hessian_diagonal(xd).cpu().numpy(), D_o) <= 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_newton_general_per_point_targets(dim):
    """Newton with non-isotropic per-point targets matches the oracle's
    Newton (same rules): same first step, same end state."""
    n, p, Q, metric = (4, 2, 4, 2) if dim == 2 else (2, 2, 3, 303)
    mesh = meshgen.box_mesh(dim, n, p)
    prob0 = O.Problem(dim, p, Q, mesh.elem_node, metric, mesh.h * np.eye(dim))
    x0 = meshgen.perturb(mesh, 0.1, 80 + dim, bad_elements=prob0.bad_elements)
    W = targets(mesh, Q, "qp", 90 + dim)
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, W)
    opts = O.NewtonOptions(max_it=40, rtol=1e-10, cg_rtol=1e-10)
    xo, rep_o = O.newton_solve(prob, x0, mesh.fixed, opts)
    ctx = T_ctx(dim, p, Q, metric, mesh, W)
    xd = to_dev(x0)
    st, rep = ctx.newton_solve(xd, max_it=40, rtol=1e-10, cg_rtol=1e-10)
    say(f"  oracle: stop {rep_o.stop} iters {rep_o.iters} F {rep_o.F0:.6e} -> {rep_o.F:.6e}; "
        f"gpu: status {st} iters {rep['iters']} F {rep['F']:.6e}")
    assert rep_o.stop == O.STOP_CONVERGED and st == 0
    assert abs(rep["history_F"][1] - rep_o.history[1][0]) <= 1e-8 * rep_o.history[1][0]
    assert abs(rep["F"] - rep_o.F) <= 1e-10 * rep_o.F0
    x = xd.cpu().numpy()
    assert np.max(np.abs(x - xo)) <= 1e-7 * mesh.h
    fixed = mesh.fixed.astype(bool)
    np.testing.assert_array_equal(x[fixed], x0[fixed])


def T_ctx(dim, p, Q, metric, mesh, W, precision=0):
    from paper_1807_09807_amd import tmop as T
    return T.Context(dim, p, mesh.elem_node, mesh.n_node, Q, metric, W, fixed=mesh.fixed, precision=precision)


def test_general_target_setup_checks():
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(2, 3, 2)
    for kind in ("elem", "qp"):
        W = targets(mesh, 4, kind, 5)
        bad = W.copy()
        bad.reshape(-1, 2, 2)[3] = [[1.0, 0.0], [0.0, -1.0]]     # det W < 0 at one element / point
        with pytest.raises(T.TMOPError) as ei:
            T_ctx(2, 2, 4, 2, mesh, bad)
        assert ei.value.status == T.TMOP_E_TARGET
        bad = W.copy()
        bad.reshape(-1)[7] = np.nan
        with pytest.raises(T.TMOPError) as ei:
            T_ctx(2, 2, 4, 2, mesh, bad)
        assert ei.value.status == T.TMOP_E_TARGET
        ctx = T_ctx(2, 2, 4, 2, mesh, W)
        x = to_dev(mesh.x_grid)
        for call in (lambda: ctx.set_combo(2, np.eye(2)), lambda: ctx.set_replication(0.5, x),
                     lambda: ctx.dfo_sweep(x.clone())):
            with pytest.raises(T.TMOPError) as ei:
                call()
            assert ei.value.status == T.TMOP_E_UNSUPPORTED
