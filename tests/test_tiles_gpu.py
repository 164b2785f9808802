"""The owner-computes tile scatter of 2D meshes (TMOP_SCATTER_TILES, on
request): the gradient, energy + gradient and Hessian action in one tile
launch plus the halo sums, against the FP64 oracle element by element (FP64 within 1e-12
relative, mixed FP32 within each result's first-order rounding bound),
against the colour launches (to rounding: the two add the same element
contributions in different orders), bitwise repeatable, with per-point and
general targets, with the Section 4 terms added after the tile pass, inside
Newton, and at the full 2D workload sizes."""
import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen
from tests._helpers import build, context, mixed_tol, rel_max_err, say, small_cases, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP64_TOL = 1e-12
CASES = [c for c in small_cases() if c.dim == 2]


def _tiles(ctx):
    from paper_1807_09807_amd import tmop as T
    ctx.set_scatter(T.TMOP_SCATTER_TILES)
    return ctx


def _colours(ctx):
    from paper_1807_09807_amd import tmop as T
    ctx.set_scatter(T.TMOP_SCATTER_COLOURS)
    return ctx


@pytest.fixture(scope="module", params=CASES, ids=str)
def setup(request):
    case = request.param
    say(f"[tiles] case {case.name}")
    mesh, prob, W = build(case)
    v = np.random.default_rng(case.seed + 100).uniform(-1, 1, mesh.x.shape)
    F, md = prob.energy(mesh.x)
    ref = dict(F=F, mindet=md, g=prob.gradient(mesh.x), Hv=prob.hessian_apply(mesh.x, v),
               mixed=mixed_tol(prob, mesh.x, v))
    return case, mesh, W, v, ref


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_tiles_against_oracle_and_colours(setup, precision):
    case, mesh, W, v, ref = setup
    col = _colours(context(case, mesh, W, precision))
    til = _tiles(context(case, mesh, W, precision))
    x, vd = to_dev(mesh.x), to_dev(v)
    tol = dict(F=FP64_TOL, min_detA=1e-12, g=FP64_TOL, Hv=FP64_TOL) if precision == 0 else ref["mixed"]
    g = til.gradient(x)
    Hv = til.hessian_apply(x, vd)
    F, md, st, ge = til.energy_gradient(x)
    eg, eh = rel_max_err(g.cpu().numpy(), ref["g"]), rel_max_err(Hv.cpu().numpy(), ref["Hv"])
    say(f"  {case.name} prec={precision}: tiles g {eg:.2e} Hv {eh:.2e} F {abs(F - ref['F']) / abs(ref['F']):.2e} "
        f"(bars {tol['g']:.1e} {tol['Hv']:.1e})")
    assert st == 0
    assert eg <= tol["g"] and eh <= tol["Hv"]
    assert rel_max_err(ge.cpu().numpy(), ref["g"]) <= tol["g"]
    assert abs(F - ref["F"]) <= tol["F"] * abs(ref["F"])
    assert abs(md - ref["mindet"]) <= tol["min_detA"] * abs(ref["mindet"])
    # the colour launches: same element contributions, other summation order
    gc, Hc = col.gradient(x), col.hessian_apply(x, vd)
    Fc, mdc, _, _ = col.energy_gradient(x)
    dg, dh = rel_max_err(g.cpu().numpy(), gc.cpu().numpy()), rel_max_err(Hv.cpu().numpy(), Hc.cpu().numpy())
    say(f"  {case.name} prec={precision}: tiles vs colours g {dg:.1e} Hv {dh:.1e}")
    # FP64: rounding of the summation order; mixed: the FP32 element results may
    # round differently where the two instantiations contract other products into FMAs
    same = 1e-14 if precision == 0 else 2 * max(tol["g"], tol["Hv"])
    assert dg <= same and dh <= same
    assert abs(F - Fc) <= (1e-13 if precision == 0 else tol["F"]) * abs(Fc)
    assert abs(md - mdc) <= (0.0 if precision == 0 else tol["min_detA"]) * abs(mdc)
    col.close()
    til.close()


def test_tiles_bitwise_repeatable(setup):
    case, mesh, W, v, ref = setup
    ctx = _tiles(context(case, mesh, W, 0))
    x, vd = to_dev(mesh.x), to_dev(v)
    assert torch.equal(ctx.gradient(x), ctx.gradient(x))
    assert torch.equal(ctx.hessian_apply(x, vd), ctx.hessian_apply(x, vd))
    a, b = ctx.energy_gradient(x), ctx.energy_gradient(x)
    assert a[:3] == b[:3] and torch.equal(a[3], b[3])
    ctx.close()


def test_split_passes_match_bitwise(setup, monkeypatch):
    """The FP64 gradient tile kernels' split passes (one component at a time
    through the LDS area, forced on with TMOP_TILE_SPLIT=1) give the same
    gradient and energy + gradient bit for bit as the passes over both
    components (forced off), and match the oracle."""
    case, mesh, W, v, ref = setup
    x = to_dev(mesh.x)
    out = {}
    for force in ("0", "1"):
        monkeypatch.setenv("TMOP_TILE_SPLIT", force)
        ctx = _tiles(context(case, mesh, W, 0))
        out[force] = (ctx.gradient(x), ctx.energy_gradient(x))
        ctx.close()
    (g0, eg0), (g1, eg1) = out["0"], out["1"]
    assert torch.equal(g0, g1) and torch.equal(eg0[3], eg1[3]) and eg0[:3] == eg1[:3]
    assert rel_max_err(g1.cpu().numpy(), ref["g"]) <= FP64_TOL
    assert abs(eg1[0] - ref["F"]) <= FP64_TOL * abs(ref["F"])


def test_switching_modes(setup):
    """The mode is a per-call choice: tiles, colours, tiles again (bit for
    bit as the first time)."""
    from paper_1807_09807_amd import tmop as T
    case, mesh, W, v, ref = setup
    ctx = _tiles(context(case, mesh, W, 0))
    x = to_dev(mesh.x)
    g0 = ctx.gradient(x).clone()
    ctx.set_scatter(T.TMOP_SCATTER_COLOURS)
    g1 = ctx.gradient(x)
    ctx.set_scatter(T.TMOP_SCATTER_TILES)
    assert torch.equal(ctx.gradient(x), g0)
    assert rel_max_err(g1.cpu().numpy(), ref["g"]) <= FP64_TOL
    ctx.close()


def _general_targets(mesh, Q, kind, seed):
    d = mesh.dim
    shape = (mesh.n_elem,) if kind == "elem" else (mesh.n_elem, Q ** d)
    M = np.random.default_rng(seed).uniform(-1.0, 1.0, shape + (d, d))
    return mesh.h * (np.eye(d) + 0.25 * M)


@pytest.mark.parametrize("kind", ["sizes", "elem", "qp"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_tiles_with_point_targets(kind, precision):
    """Per-point sizes and general targets per element or per point: the
    tile kernels read them in element order."""
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(2, 7, 2)
    prob0 = O.Problem(2, 2, 4, mesh.elem_node, 2, mesh.h * np.eye(2))
    x = meshgen.perturb(mesh, 0.1, 80, bad_elements=prob0.bad_elements)
    v = np.random.default_rng(81).uniform(-1, 1, x.shape)
    if kind == "sizes":
        sizes = mesh.h * np.random.default_rng(82).uniform(0.7, 1.3, (mesh.n_elem, 16))
        prob = O.Problem(2, 2, 4, mesh.elem_node, 2, sizes[:, :, None, None] * np.eye(2))
        ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 2, None, fixed=mesh.fixed, precision=precision,
                        target_sizes=sizes)
    else:
        W = _general_targets(mesh, 4, kind, 83)
        prob = O.Problem(2, 2, 4, mesh.elem_node, 2, W)
        ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 2, W, fixed=mesh.fixed, precision=precision)
    _tiles(ctx)
    tol = dict(g=FP64_TOL, Hv=FP64_TOL) if precision == 0 else mixed_tol(prob, x, v)
    xd, vd = to_dev(x), to_dev(v)
    eg = rel_max_err(ctx.gradient(xd).cpu().numpy(), prob.gradient(x))
    eh = rel_max_err(ctx.hessian_apply(xd, vd).cpu().numpy(), prob.hessian_apply(x, v))
    F, md, st, ge = ctx.energy_gradient(xd)
    say(f"  targets {kind} prec={precision}: g {eg:.2e} Hv {eh:.2e}")
    assert st == 0 and eg <= tol["g"] and eh <= tol["Hv"]
    assert rel_max_err(ge.cpu().numpy(), prob.gradient(x)) <= tol["g"]
    ctx.close()


def test_tiles_with_section4_terms():
    """The second metric term (eq. 4.1) and the displacement penalty (eq.
    4.2) run as colour launches after the tile pass and add to its output."""
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(2, 6, 2)
    W = mesh.h * np.eye(2)
    prob0 = O.Problem(2, 2, 4, mesh.elem_node, 2, W)
    x = meshgen.perturb(mesh, 0.1, 84, bad_elements=prob0.bad_elements)
    x_init = meshgen.perturb(mesh, 0.05, 85, bad_elements=prob0.bad_elements)
    v = np.random.default_rng(86).uniform(-1, 1, x.shape)
    out = []
    for mode in (T.TMOP_SCATTER_COLOURS, T.TMOP_SCATTER_TILES):
        ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 2, W, fixed=mesh.fixed)
        ctx.set_combo(7, mesh.h * np.array([[1.2, 0.1], [0.0, 0.8]]), 1.0, 0.5)
        ctx.set_restriction(0.3, to_dev(x_init))
        ctx.set_scatter(mode)
        xd, vd = to_dev(x), to_dev(v)
        F, md, st, g = ctx.energy_gradient(xd)
        out.append((F, g.cpu().numpy(), ctx.hessian_apply(xd, vd).cpu().numpy()))
        ctx.close()
    (Fc, gc, hc), (Ft, gt, ht) = out
    assert abs(Ft - Fc) <= 1e-13 * abs(Fc)
    assert rel_max_err(gt, gc) <= 1e-14 and rel_max_err(ht, hc) <= 1e-14


def test_newton_with_tiles():
    """Newton on the 8 x 8 Q2 workload with each scatter.  The inner CG
    iterates are not unique in floating point (the two scatters sum the
    Hessian action in different orders), so the trajectories may separate
    slowly, as against the oracle's Newton: the same bar as there, F within
    1e-6 relative while F > 1e-8 F0, and the same iteration count."""
    from paper_1807_09807_amd import tmop as T
    w = meshgen.WORKLOADS["q2_square_8"]
    mesh = meshgen.box_mesh(2, w["n"], w["p"])
    W = mesh.h * np.eye(2)
    prob = O.Problem(2, w["p"], w["Q"], mesh.elem_node, w["metric"], W)
    mesh = meshgen.make_workload("q2_square_8", bad_elements=lambda x, e: prob.bad_elements(x, e, w["tau_min"]))
    res = []
    for mode in (T.TMOP_SCATTER_COLOURS, T.TMOP_SCATTER_TILES):
        ctx = T.Context(2, w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
        ctx.set_scatter(mode)
        x = to_dev(mesh.x)
        st, rep = ctx.newton_solve(x, max_it=10)
        res.append((st, rep))
        ctx.close()
    (sc, rc), (stt, rt) = res
    Fc, Ft = rc["history_F"], rt["history_F"]
    worst = max(abs(b - a) / a for a, b in zip(Fc, Ft) if a > 1e-8 * Fc[0])
    say(f"  newton colours: it {rc['iters']} F {rc['F']:.6e}; tiles: it {rt['iters']} F {rt['F']:.6e}; "
        f"worst relative F difference {worst:.2e}")
    assert sc == stt and rt["iters"] == rc["iters"] and len(Fc) == len(Ft)
    assert worst <= 1e-6
    assert all(b < a for a, b in zip(Ft, Ft[1:]))


def test_tiles_refused_in_3d():
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(3, 2, 1)
    ctx = T.Context(3, 1, mesh.elem_node, mesh.n_node, 2, 303, mesh.h * np.eye(3))
    with pytest.raises(T.TMOPError) as ei:
        ctx.set_scatter(T.TMOP_SCATTER_TILES)
    assert ei.value.status == T.TMOP_E_UNSUPPORTED
    with pytest.raises(T.TMOPError) as ei:
        ctx.set_scatter(7)
    assert ei.value.status == T.TMOP_E_ARG
    ctx.close()


@pytest.mark.parametrize("name", ["q2_square_512", "q3_square_256"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_tiles_full_size(name, precision):
    """The full 2D workloads: tiles against colours over every DOF (to
    rounding) and against the oracle at 64 seeded nodes."""
    from paper_1807_09807_amd import tmop as T
    w = meshgen.WORKLOADS[name]
    mesh = meshgen.box_mesh(2, w["n"], w["p"])
    W = mesh.h * np.eye(2)
    prob = O.Problem(2, w["p"], w["Q"], mesh.elem_node, w["metric"], W)
    say(f"[tiles full] {name} prec={precision}: building")
    mesh = meshgen.make_workload(name, bad_elements=lambda x, e: prob.bad_elements(x, e, w["tau_min"]))
    x = mesh.x
    v = meshgen.random_direction(mesh, w["seed"] + 100)
    nodes = np.random.default_rng(w["seed"] + 200).choice(mesh.n_node, 64, replace=False)
    ctx = T.Context(2, w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed,
                    precision=precision)
    xd, vd = to_dev(x), to_dev(v)
    ctx.set_scatter(T.TMOP_SCATTER_COLOURS)
    gc, hc = ctx.gradient(xd), ctx.hessian_apply(xd, vd)
    ctx.set_scatter(T.TMOP_SCATTER_TILES)
    gt, ht = ctx.gradient(xd), ctx.hessian_apply(xd, vd)
    ctx.close()
    idx = torch.from_numpy(nodes).cuda()
    g_ref, h_ref = prob.gradient_at(x, nodes), prob.hessian_apply_at(x, v, nodes)
    eg = np.max(np.abs(gt[:, idx].cpu().numpy() - g_ref)) / np.max(np.abs(g_ref))
    eh = np.max(np.abs(ht[:, idx].cpu().numpy() - h_ref)) / np.max(np.abs(h_ref))
    if precision == 0:   # every DOF against the colour launches, the sampled ones against the oracle
        dg = rel_max_err(gt.cpu().numpy(), gc.cpu().numpy())
        dh = rel_max_err(ht.cpu().numpy(), hc.cpu().numpy())
        bars = dict(g=FP64_TOL, Hv=FP64_TOL, same=1e-14)
    else:                # the FP32 element results may round differently: the sampled DOFs, to the bound
        from oracle import fp32_bound
        bs = fp32_bound.dof_bounds(prob, x, v, elems=prob._elements_touching(nodes))
        bars = dict(g=np.max(bs["g"][:, nodes]) / np.max(np.abs(g_ref)),
                    Hv=np.max(bs["Hv"][:, nodes]) / np.max(np.abs(h_ref)))
        bars["same"] = 2 * max(bars["g"], bars["Hv"])
        dg = np.max(np.abs((gt - gc)[:, idx].cpu().numpy())) / np.max(np.abs(g_ref))
        dh = np.max(np.abs((ht - hc)[:, idx].cpu().numpy())) / np.max(np.abs(h_ref))
    say(f"  {name} prec={precision}: tiles vs colours g {dg:.1e} Hv {dh:.1e}; vs oracle at 64 nodes g {eg:.1e} "
        f"Hv {eh:.1e}")
    assert dg <= bars["same"] and dh <= bars["same"]
    assert eg <= bars["g"] and eh <= bars["Hv"]
