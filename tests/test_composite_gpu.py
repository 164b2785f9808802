"""The Section 4 objectives in the HIP library against the oracle, element
by element (FP64 within 1e-12 relative, mixed FP32 within the mixed
tolerance of the worse-conditioned term): the displacement penalty of
eq. 4.2, the two-term composite metric of eq. 4.1 with per-point weights
and the replication composite of Section 4.3.2 (each in 2D and 3D, the
penalty also with per-point targets), all of them together, argument checks, and Newton on each
against the oracle's Newton."""
import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen
from tests._helpers import mixed_tol, rel_max_err, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _base(dim, n, p, Q, metric, seed, per_point=False):
    mesh = meshgen.box_mesh(dim, n, p)
    W = mesh.h * np.eye(dim)
    prob0 = O.Problem(dim, p, Q, mesh.elem_node, metric, W)
    x0 = meshgen.perturb(mesh, 0.10, seed, bad_elements=prob0.bad_elements)
    x = meshgen.perturb(mesh, 0.04, seed + 1, base=x0, bad_elements=prob0.bad_elements)
    sizes = None
    if per_point:
        sizes = mesh.h * np.random.default_rng(seed + 2).uniform(0.8, 1.2, (mesh.n_elem, Q ** dim))
        W = sizes[:, :, None, None] * np.eye(dim)
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, W)
    return mesh, prob, x0, x, sizes


def _ctx(mesh, p, Q, metric, sizes, precision):
    from paper_1807_09807_amd import tmop as T
    W = None if sizes is not None else mesh.h * np.eye(mesh.dim)
    return T.Context(mesh.dim, p, mesh.elem_node, mesh.n_node, Q, metric, W, fixed=mesh.fixed,
                     precision=precision, target_sizes=sizes)


def _compare(ctx, prob, x, v, precision, label):
    """Every operation against the oracle: FP64 within 1e-12, mixed FP32
    within each result's first-order rounding bound (all terms included)."""
    xd, vd = to_dev(x), to_dev(v)
    F_ref, md_ref = prob.energy(x)
    F, md, st = ctx.energy(xd)
    Fe, mde, _, ge = ctx.energy_gradient(xd)
    g_ref = prob.gradient(x)
    errs = dict(F=abs(F - F_ref) / abs(F_ref), Fe=abs(Fe - F_ref) / abs(F_ref),
                g=rel_max_err(ctx.gradient(xd).cpu().numpy(), g_ref),
                ge=rel_max_err(ge.cpu().numpy(), g_ref),
                Hv=rel_max_err(ctx.hessian_apply(xd, vd).cpu().numpy(), prob.hessian_apply(x, v)),
                diag=rel_max_err(ctx.hessian_diagonal(xd).cpu().numpy(), prob.hessian_diagonal(x)))
    if precision == 0:
        tol = dict(F=1e-12, Fe=1e-12, g=1e-12, ge=1e-12, Hv=1e-12, diag=1e-12, min_detA=1e-12)
    else:
        b = mixed_tol(prob, x, v, diag=True)
        tol = dict(b, Fe=b["F"], ge=b["g"])
    say(f"  {label}: " + " ".join(f"{k} {e:.2e} (bar {tol[k]:.1e})" for k, e in errs.items()))
    assert st == 0 and md == mde
    assert abs(md - md_ref) <= tol["min_detA"] * abs(md_ref)
    for k, e in errs.items():
        assert e <= tol[k], k


def _newton_compare(F_o, F_g, rep_o, rep, xo, xg, h):
    """Same Newton rules on both sides, compared where the result is
    unique: the start (to rounding), the first step (every direction comes
    from up to hundreds of truncated-CG iterations whose iterates depend on
    rounding, 1e-6), and the end state (the Newton tolerance).  In between,
    a negative curvature exit, the CG stopping test or the 1.2-growth
    acceptance of a step length can flip, after which the paths separate
    (with the replication composite the F after the third step differs by 3%
    while both converge to the same mesh)."""
    from paper_1807_09807_amd import tmop as T
    cg_o, cg_g = [hh[3] for hh in rep_o.history[1:]], list(rep["history_cg"][1:])
    say(f"  oracle {rep_o.iters} it F {F_o[0]:.6e} -> {F_o[-1]:.6e}, CG {cg_o}, alpha "
        f"{[hh[2] for hh in rep_o.history[1:]]}; gpu {rep['iters']} it -> {F_g[-1]:.6e}, CG {cg_g}")
    assert rep["status"] == T.TMOP_OK and rep_o.stop == O.STOP_CONVERGED
    assert abs(F_g[0] - F_o[0]) <= 1e-12 * abs(F_o[0])
    assert abs(F_g[1] - F_o[1]) <= 1e-6 * abs(F_o[1])
    assert abs(F_g[-1] - F_o[-1]) <= 1e-10 * abs(F_o[-1])
    assert abs(rep["iters"] - rep_o.iters) <= 2
    assert np.max(np.abs(xg - xo)) < 1e-7 * h


# ----------------------------------------------------------------- eq. 4.2

RESTRICT = [  # dim, n, p, Q, metric, seed, per-point targets
    (2, 6, 2, 4, 2, 80, False),
    (2, 5, 3, 5, 9, 81, False),
    (2, 7, 1, 2, 7, 82, False),
    (3, 3, 2, 4, 303, 83, False),
    (3, 3, 1, 2, 302, 84, False),
    (2, 5, 2, 4, 2, 85, True),
    (3, 2, 3, 4, 303, 86, True),
]


@pytest.mark.parametrize("case", RESTRICT, ids=lambda c: f"{c[0]}d_p{c[2]}_q{c[3]}_mu{c[4]}{'_qps' if c[6] else ''}")
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_restriction_parity(case, precision):
    dim, n, p, Q, metric, seed, per_point = case
    say(f"[restrict] case {case} precision {precision}")
    mesh, prob, x0, x, sizes = _base(*case)
    delta = 40.0
    prob.set_restriction(delta, x0)
    ctx = _ctx(mesh, p, Q, metric, sizes, precision)
    ctx.set_restriction(delta, to_dev(x0))
    v = np.random.default_rng(seed + 3).uniform(-1, 1, x.shape)
    _compare(ctx, prob, x, v, precision, "restricted")


def test_restriction_removal_and_timing():
    from paper_1807_09807_amd import tmop as T
    mesh, prob, x0, x, _ = _base(2, 6, 2, 4, 2, 90)
    ctx = _ctx(mesh, 2, 4, 2, None, 0)
    xd = to_dev(x)
    F0 = ctx.energy(xd)[0]
    with pytest.raises(T.TMOPError) as ei:
        ctx.set_restriction(-1.0, to_dev(x0))
    assert ei.value.status == T.TMOP_E_ARG
    with pytest.raises(T.TMOPError):
        ctx.set_restriction(float("inf"), to_dev(x0))
    ctx.set_restriction(5.0, to_dev(x0))
    ctx.timing_enable(True)
    F1 = ctx.energy(xd)[0]
    ctx.hessian_apply(xd, xd)
    ms, launches = ctx.timing_read(T.TIMING_PENALTY)
    assert launches >= 2 and ms > 0.0
    ctx.timing_enable(False)
    ctx.set_restriction(0.0)
    assert F1 > F0 and ctx.energy(xd)[0] == F0


def test_newton_restricted_matches_oracle():
    """Section 4.3.1 on the 8x8 Q2 mu_2 workload with delta = 10: F history
    and the optimized mesh against the oracle's Newton."""
    from paper_1807_09807_amd import tmop as T
    say("[restrict] newton 8x8 delta 10")
    w = meshgen.WORKLOADS["q2_square_8"]
    mesh = meshgen.box_mesh(2, w["n"], w["p"])
    W = mesh.h * np.eye(2)
    prob = O.Problem(2, w["p"], w["Q"], mesh.elem_node, w["metric"], W)
    x0 = meshgen.perturb(mesh, w["noise"], w["seed"], bad_elements=prob.bad_elements)
    prob.set_restriction(10.0, x0)
    xo, rep_o = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=40, cg_rtol=1e-10))
    ctx = T.Context(2, w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
    ctx.set_restriction(10.0, to_dev(x0))
    xd = to_dev(x0)
    st, rep = ctx.newton_solve(xd, max_it=40, cg_rtol=1e-10)
    _newton_compare([h[0] for h in rep_o.history], rep["history_F"], rep_o, rep, xo, xd.cpu().numpy(), mesh.h)


# ----------------------------------------------------------------- eq. 4.1

COMBO = [  # dim, n, p, Q, metric, metric2, W2 / h, eta1, eta2, per-point eta2, seed
    (2, 6, 2, 4, 1, 77, ((0.7, 0.0), (0.0, 0.7)), 1.0, 0.5, True, 100),
    (2, 5, 3, 5, 2, 9, ((1.0, 0.3), (-0.2, 1.1)), 0.7, 2.0, False, 101),
    (2, 7, 1, 2, 7, 14, ((1.2, 0.0), (0.1, 0.9)), 1.3, 0.4, True, 102),
    (2, 4, 4, 5, 98, 2, ((0.9, 0.0), (0.0, 1.1)), 0.5, 1.0, True, 103),
    (3, 3, 2, 4, 303, 302, ((0.8, 0.1, 0.0), (0.0, 1.1, 0.2), (0.1, 0.0, 0.9)), 1.0, 0.6, True, 104),
    (3, 2, 3, 4, 302, 303, ((0.7, 0.0, 0.0), (0.0, 0.7, 0.0), (0.0, 0.0, 0.7)), 0.8, 1.5, False, 105),
]


def _combo(case):
    dim, n, p, Q, m1, m2, W2s, eta1, eta2, pp, seed = case
    mesh, prob, x0, x, _ = _base(dim, n, p, Q, m1, seed)
    W2 = mesh.h * np.asarray(W2s)
    eq = np.random.default_rng(seed + 5).uniform(0.2, 1.5, (mesh.n_elem, Q ** dim)) if pp else None
    prob.set_combo(m2, W2, eta1, eta2 * (eq if pp else 1.0))
    return mesh, prob, x0, x, W2, eq


@pytest.mark.parametrize("case", COMBO, ids=lambda c: f"{c[0]}d_p{c[2]}_q{c[3]}_mu{c[4]}+mu{c[5]}")
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_combo_parity(case, precision):
    dim, n, p, Q, m1, m2, W2s, eta1, eta2, pp, seed = case
    say(f"[combo] case {case} precision {precision}")
    mesh, prob, x0, x, W2, eq = _combo(case)
    ctx = _ctx(mesh, p, Q, m1, None, precision)
    ctx.set_combo(m2, W2, eta1, eta2, eq)
    v = np.random.default_rng(seed + 6).uniform(-1, 1, x.shape)
    _compare(ctx, prob, x, v, precision, "combo")


def test_combo_arguments():
    from paper_1807_09807_amd import tmop as T
    mesh, prob, x0, x, _ = _base(2, 4, 2, 3, 2, 110)
    ctx = _ctx(mesh, 2, 3, 2, None, 0)
    xd = to_dev(x)
    F0 = ctx.energy(xd)[0]
    for bad, code in [(dict(metric2=303, W2=np.eye(2)), T.TMOP_E_ARG),
                      (dict(metric2=77, W2=np.diag([1.0, -1.0])), T.TMOP_E_TARGET),
                      (dict(metric2=77, W2=np.eye(2), eta2=-1.0), T.TMOP_E_ARG),
                      (dict(metric2=77, W2=np.eye(2), eta2_q=-np.ones((mesh.n_elem, 9))), T.TMOP_E_ARG)]:
        with pytest.raises(T.TMOPError) as ei:
            ctx.set_combo(**bad)
        assert ei.value.status == code
    assert ctx.energy(xd)[0] == F0
    ctx.set_combo(0, eta1=2.0)                       # eta_1 alone scales F
    assert ctx.energy(xd)[0] == pytest.approx(2.0 * F0, rel=1e-14)
    qps = _ctx(mesh, 2, 3, 2, np.full((mesh.n_elem, 9), mesh.h), 0)
    with pytest.raises(T.TMOPError) as ei:
        qps.set_combo(77, np.eye(2))
    assert ei.value.status == T.TMOP_E_UNSUPPORTED
    m3 = meshgen.box_mesh(3, 2, 2)
    c3 = T.Context(3, 2, m3.elem_node, m3.n_node, 3, 303, m3.h * np.eye(3))
    with pytest.raises(T.TMOPError) as ei:
        c3.set_combo(77, np.eye(3))                    # a 2D metric
    assert ei.value.status == T.TMOP_E_ARG
    with pytest.raises(ValueError):
        c3.set_combo(302, np.eye(2))                   # a 2x2 target


def test_newton_combo_matches_oracle():
    """mu_1 + eta(x) mu_77 with a smaller size target (the form of Section
    5.2.4 on a synthetic mesh): F history and result against the oracle."""
    from paper_1807_09807_amd import tmop as T
    say("[combo] newton mu_1 + eta mu_77")
    mesh = meshgen.box_mesh(2, 6, 2)
    W = mesh.h * np.eye(2)
    prob = O.Problem(2, 2, 4, mesh.elem_node, 1, W)
    x0 = meshgen.perturb(mesh, 0.15, 120, bad_elements=prob.bad_elements)
    W2 = np.sqrt(0.5) * mesh.h * np.eye(2)
    eq = np.random.default_rng(121).uniform(0.2, 1.2, (mesh.n_elem, 16))
    prob.set_combo(77, W2, 1.0, eq)
    xo, rep_o = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=40, cg_rtol=1e-10))
    ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 1, W, fixed=mesh.fixed)
    ctx.set_combo(77, W2, 1.0, 1.0, eq)
    xd = to_dev(x0)
    st, rep = ctx.newton_solve(xd, max_it=40, cg_rtol=1e-10)
    _newton_compare([h[0] for h in rep_o.history], rep["history_F"], rep_o, rep, xo, xd.cpu().numpy(), mesh.h)


# ----------------------------------------------------------- Section 4.3.2

REPL = [  # dim, n, p, Q, metric, gamma, seed
    (2, 6, 2, 4, 2, 0.4, 130),
    (2, 5, 3, 5, 9, 0.7, 131),
    (2, 4, 4, 5, 1, 0.0, 132),
    (2, 7, 1, 2, 77, 1.0, 133),
    (3, 3, 2, 4, 303, 0.5, 134),
    (3, 2, 3, 4, 302, 0.3, 135),
    (3, 3, 1, 2, 303, 0.0, 136),
]


@pytest.mark.parametrize("case", REPL, ids=lambda c: f"{c[0]}d_p{c[2]}_q{c[3]}_mu{c[4]}_g{c[5]}")
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_replication_parity(case, precision):
    dim, n, p, Q, metric, gamma, seed = case
    say(f"[replication] case {case} precision {precision}")
    mesh, prob, x0, x, _ = _base(dim, n, p, Q, metric, seed)
    prob.set_replication(gamma, x0)
    A0 = prob._jac(x0, 0, mesh.n_elem)
    ctx = _ctx(mesh, p, Q, metric, None, precision)
    ctx.set_replication(gamma, to_dev(x0))
    v = np.random.default_rng(seed + 7).uniform(-1, 1, x.shape)
    _compare(ctx, prob, x, v, precision, "replication")


def test_replication_3d_keeps_initial_mesh():
    from paper_1807_09807_amd import tmop as T
    mesh, prob, x0, x, _ = _base(3, 3, 2, 3, 303, 141)
    ctx = _ctx(mesh, 2, 3, 303, None, 0)
    x0d = to_dev(x0)
    ctx.set_replication(0.0, x0d)
    F, md, st = ctx.energy(x0d)
    assert st == 0 and abs(F) <= 1e-26 and float(ctx.gradient(x0d).abs().max()) <= 1e-13


def test_replication_keeps_initial_mesh_and_rejects_inverted():
    from paper_1807_09807_amd import tmop as T
    mesh, prob, x0, x, _ = _base(2, 6, 2, 4, 2, 140)
    ctx = _ctx(mesh, 2, 4, 2, None, 0)
    x0d = to_dev(x0)
    ctx.set_replication(0.0, x0d)
    F, md, st = ctx.energy(x0d)
    g = ctx.gradient(x0d).cpu().numpy()
    assert st == 0 and abs(F) <= 1e-26 and np.max(np.abs(g)) <= 1e-13
    xd = x0d.clone()
    st, rep = ctx.newton_solve(xd, max_it=5, atol=1e-12)
    assert st == T.TMOP_OK and rep["iters"] == 0 and torch.equal(xd, x0d)
    # an inverted x_init is refused and leaves the context as it was
    bad = x0.copy()
    a = (mesh.n * 2 + 1) + 1
    bad[:, [a, a + 1]] = bad[:, [a + 1, a]]
    with pytest.raises(T.TMOPError) as ei:
        ctx.set_replication(0.5, to_dev(bad))
    assert ei.value.status == T.TMOP_E_TARGET
    assert ctx.energy(x0d)[0] == F
    with pytest.raises(T.TMOPError) as ei:
        ctx.set_replication(1.5, x0d)
    assert ei.value.status == T.TMOP_E_ARG


def test_newton_replication_matches_oracle():
    from paper_1807_09807_amd import tmop as T
    say("[replication] newton gamma 0.5")
    mesh = meshgen.box_mesh(2, 6, 2)
    W = mesh.h * np.eye(2)
    prob = O.Problem(2, 2, 4, mesh.elem_node, 2, W)
    x0 = meshgen.perturb(mesh, 0.15, 150, bad_elements=prob.bad_elements)
    prob.set_replication(0.5, x0)
    xo, rep_o = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=40, cg_rtol=1e-10))
    ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 2, W, fixed=mesh.fixed)
    xd = to_dev(x0)
    ctx.set_replication(0.5, xd)
    st, rep = ctx.newton_solve(xd, max_it=40, cg_rtol=1e-10)
    _newton_compare([h[0] for h in rep_o.history], rep["history_F"], rep_o, rep, xo, xd.cpu().numpy(), mesh.h)


# ------------------------------------------------------------- all together

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_all_terms_together(dim, precision):
    """Replication composite and displacement penalty at once (2D Q3, 3D Q2)."""
    n, p, Q, metric = (5, 3, 5, 9) if dim == 2 else (3, 2, 3, 303)
    mesh, prob, x0, x, _ = _base(dim, n, p, Q, metric, 160)
    prob.set_replication(0.6, x0)
    prob.set_restriction(20.0, x0)
    ctx = _ctx(mesh, p, Q, metric, None, precision)
    ctx.set_replication(0.6, to_dev(x0))
    ctx.set_restriction(20.0, to_dev(x0))
    v = np.random.default_rng(161).uniform(-1, 1, x.shape)
    _compare(ctx, prob, x, v, precision, "all")


def test_restriction_general_target_3d():
    """The penalty with a general constant target W in 3D (det W weights the
    mass matrix; the FP64 Hessian action fuses it into the element kernel)."""
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(3, 3, 2)
    W = mesh.h * np.array([[1.0, 0.2, 0.0], [0.0, 1.1, 0.3], [0.1, 0.0, 0.9]])
    prob = O.Problem(3, 2, 4, mesh.elem_node, 302, W)
    x0 = meshgen.perturb(mesh, 0.08, 170, bad_elements=prob.bad_elements)
    x = meshgen.perturb(mesh, 0.03, 171, base=x0, bad_elements=prob.bad_elements)
    v = np.random.default_rng(172).uniform(-1, 1, x.shape)
    prob.set_restriction(60.0, x0)
    ctx = T.Context(3, 2, mesh.elem_node, mesh.n_node, 4, 302, W, fixed=mesh.fixed)
    ctx.set_restriction(60.0, to_dev(x0))
    _compare(ctx, prob, x, v, 0, "3D general W + penalty")


def test_fused_penalty_bitwise_deterministic():
    """The FP64 3D Hessian action with the penalty fused into the element
    kernel keeps the coloured scatter's bitwise reproducibility, and so do
    the separate penalty kernels of the other operations."""
    from paper_1807_09807_amd import tmop as T
    mesh, prob, x0, x, _ = _base(3, 3, 2, 4, 303, 180)
    ctx = _ctx(mesh, 2, 4, 303, None, T.TMOP_FP64)
    ctx.set_restriction(40.0, to_dev(x0))
    xd, vd = to_dev(x), to_dev(np.random.default_rng(181).uniform(-1, 1, x.shape))
    assert torch.equal(ctx.hessian_apply(xd, vd), ctx.hessian_apply(xd, vd))
    assert torch.equal(ctx.gradient(xd), ctx.gradient(xd))
    assert torch.equal(ctx.hessian_diagonal(xd), ctx.hessian_diagonal(xd))
    assert ctx.energy(xd) == ctx.energy(xd)


@pytest.mark.parametrize("dim", [2, 3])
def test_second_term_switches(dim):
    """One context through combo -> replication -> combo -> none: the
    combo keeps its weight per point (W2 constant), the replication
    W_0^{-1} and its weight, so the library re-sizes its per-point data at
    each switch; every state matches the oracle's."""
    case = COMBO[0] if dim == 2 else COMBO[4]
    d, n, p, Q, m1, m2, W2s, eta1, eta2, pp, seed = case
    say(f"[combo] switches {dim}D")
    mesh, prob, x0, x, W2, eq = _combo(case)
    ctx = _ctx(mesh, p, Q, m1, None, 0)
    v = np.random.default_rng(seed + 7).uniform(-1, 1, x.shape)
    ctx.set_combo(m2, W2, eta1, eta2, eq)
    _compare(ctx, prob, x, v, 0, "combo")
    rep = O.Problem(dim, p, Q, mesh.elem_node, m1, mesh.h * np.eye(dim))
    rep.set_replication(0.4, x0)
    ctx.set_replication(0.4, to_dev(x0))
    _compare(ctx, rep, x, v, 0, "then replication")
    ctx.set_combo(m2, W2, eta1, eta2, eq)
    _compare(ctx, prob, x, v, 0, "combo again")
    ctx.set_combo(0, eta1=1.0)
    plain = O.Problem(dim, p, Q, mesh.elem_node, m1, mesh.h * np.eye(dim))
    _compare(ctx, plain, x, v, 1e-12, "none")
