"""The Hessian diagonal and the Newton inner solvers of the HIP library:
the diagonal against the oracle element by element (FP64 within 1e-12
relative, mixed FP32 within its first-order rounding bound), and Newton
with each inner solver (the shifted CG, truncated CG, MINRES of Section 5)
and with the Jacobi preconditioner against the oracle's implementation of
the same rules on the 8x8 Q2 workload."""
import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen
from tests._helpers import build, context, mixed_tol, rel_max_err, say, small_cases, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = small_cases()


@pytest.fixture(scope="module", params=CASES, ids=str)
def setup(request):
    case = request.param
    say(f"[diag] case {case.name}")
    mesh, prob, W = build(case)
    return case, mesh, W, prob.hessian_diagonal(mesh.x), mixed_tol(prob, mesh.x, diag=True)["diag"]


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_hessian_diagonal(setup, precision):
    case, mesh, W, ref, mtol = setup
    ctx = context(case, mesh, W, precision)
    x = to_dev(mesh.x)
    D = ctx.hessian_diagonal(x)
    err = rel_max_err(D.cpu().numpy(), ref)
    say(f"  {case.name} prec={precision} diag rel err {err:.2e} (bar {mtol:.1e})")
    assert err <= (1e-12 if precision == 0 else mtol)
    assert torch.equal(D, ctx.hessian_diagonal(x))          # bitwise reproducible


def _c1(n=None):
    w = meshgen.WORKLOADS["q2_square_8"]
    mesh = meshgen.box_mesh(2, n or w["n"], w["p"])
    W = mesh.h * np.eye(2)
    prob = O.Problem(2, w["p"], w["Q"], mesh.elem_node, w["metric"], W)
    x0 = meshgen.perturb(mesh, w["noise"], w["seed"], bad_elements=prob.bad_elements)
    return w, mesh, W, prob, x0


INNER = {"cg": 0, "minres": 1, "shifted_cg": 2}


@pytest.mark.parametrize("inner,precond", [("minres", "none"), ("minres", "jacobi"), ("cg", "jacobi"),
                                          ("shifted_cg", "none"), ("shifted_cg", "jacobi")])
def test_newton_inner_solvers_match_oracle(inner, precond):
    """Same rules on both sides, compared where the result is unique: the
    end state (the grid) and the early F history.  Truncated CG: F within
    1e-6 relative while F > 1e-2 F0 and the same Newton and inner
    iteration counts to within one (rounding decides the inner iterates,
    so the trajectories separate slowly: with the preconditioner the
    relative F difference grows about tenfold every two Newton steps, from
    1e-14 at the first step to 2e-6 at F = 4e-3 F0).  MINRES: its
    directions on the indefinite early Hessians need not descend, the 1.2
    growth rule then accepts steps that raise F, and a rounding-level
    difference in a direction can change the step length the line search
    picks, after which the trajectories differ; so the first two steps are
    compared, and the iteration counts within 25%."""
    from paper_1807_09807_amd import tmop as T
    say(f"[newton] q2_square_8 inner={inner} precond={precond}")
    w, mesh, W, prob, x0 = _c1()
    opts = O.NewtonOptions(max_it=60, cg_rtol=1e-10, inner=inner, precond=precond)
    xo, rep_o = O.newton_solve(prob, x0, mesh.fixed, opts)
    ctx = T.Context(2, w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
    xd = to_dev(x0)
    st, rep = ctx.newton_solve(xd, max_it=60, cg_rtol=1e-10, inner=INNER[inner],
                               precond=T.TMOP_PREC_JACOBI if precond == "jacobi" else T.TMOP_PREC_NONE)
    F_o = [h[0] for h in rep_o.history]
    F_g = rep["history_F"]
    say(f"  oracle iters {rep_o.iters} inner {rep_o.cg_iters}; gpu iters {rep['iters']} inner {rep['cg_iters']}")
    worst = 0.0
    n_cmp = min(len(F_o), len(F_g)) if inner != "minres" else 3
    for k in range(max(len(F_o), len(F_g))):
        a = F_o[k] if k < len(F_o) else float("nan")
        b = F_g[k] if k < len(F_g) else float("nan")
        say(f"  it {k}: F oracle {a:.16e} gpu {b:.16e}")
        if k < n_cmp and a > 1e-2 * F_o[0]:
            worst = max(worst, abs(b - a) / a)
    say(f"  worst relative F difference over the compared iterations: {worst:.2e}")
    assert st == T.TMOP_OK and rep_o.stop == O.STOP_CONVERGED
    assert worst <= 1e-6
    if inner == "minres":
        assert abs(rep["iters"] - rep_o.iters) <= max(2, 0.25 * rep_o.iters)
    else:
        assert abs(rep["iters"] - rep_o.iters) <= 1
    x = xd.cpu().numpy()
    assert np.max(np.abs(x - mesh.x_grid)) < 1e-9 * mesh.h
    np.testing.assert_array_equal(x[mesh.fixed.astype(bool)], x0[mesh.fixed.astype(bool)])


@pytest.mark.parametrize("inner", ["cg", "minres", "shifted_cg"])
def test_newton_3d_jacobi_returns_to_grid(inner):
    """Q2 hex mu_303 (6^3 elements) with the Jacobi preconditioner."""
    from paper_1807_09807_amd import tmop as T
    say(f"[newton] q2_cube_64@6 jacobi inner={inner}")
    w = meshgen.WORKLOADS["q2_cube_64"]
    mesh = meshgen.box_mesh(3, 6, 2)
    W = mesh.h * np.eye(3)
    prob = O.Problem(3, 2, 4, mesh.elem_node, 303, W)
    x0 = meshgen.perturb(mesh, w["noise"], w["seed"], bad_elements=prob.bad_elements)
    ctx = T.Context(3, 2, mesh.elem_node, mesh.n_node, 4, 303, W, fixed=mesh.fixed)
    xd = to_dev(x0)
    st, rep = ctx.newton_solve(xd, max_it=60, rtol=1e-10, precond=T.TMOP_PREC_JACOBI, inner=INNER[inner])
    say(f"  status {st} iters {rep['iters']} inner {rep['cg_iters']} F {rep['F0']:.3e} -> {rep['F']:.3e}")
    assert st == T.TMOP_OK
    assert np.max(np.abs(xd.cpu().numpy() - mesh.x_grid)) / mesh.h < 1e-8


def test_newton_rejects_unknown_solver():
    from paper_1807_09807_amd import tmop as T
    w, mesh, W, prob, x0 = _c1(4)
    ctx = T.Context(2, w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
    xd = to_dev(x0)
    for bad in (dict(inner=7), dict(precond=-1), dict(shift_beta=0.0), dict(shift_beta=float("nan"))):
        with pytest.raises(T.TMOPError):
            ctx.newton_solve(xd, **bad)
    assert torch.equal(xd, to_dev(x0))
