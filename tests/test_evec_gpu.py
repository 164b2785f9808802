"""The element-vector scatter (TMOP_SCATTER_ELEMENTS, 2D and 3D): one
launch over every element writing each element's gradient / Hessian-action
share, then a pass summing each node's entries in ascending element order.
Against the FP64 oracle element by element (FP64 within 1e-12 relative,
mixed FP32 within each result's first-order rounding bound), against the
colour launches (FP64 to rounding: the same element contributions summed in
another order), bitwise repeatable, with per-point targets, with the fused
displacement penalty and the second metric term, inside Newton, and at full
size."""
import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen
from tests._helpers import build, context, mixed_tol, rel_max_err, say, small_cases, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP64_TOL = 1e-12
CASES = small_cases()


def _mode(ctx, name):
    from paper_1807_09807_amd import tmop as T
    ctx.set_scatter(getattr(T, f"TMOP_SCATTER_{name}"))
    return ctx


@pytest.fixture(scope="module", params=CASES, ids=str)
def setup(request):
    case = request.param
    say(f"[evec] case {case.name}")
    mesh, prob, W = build(case)
    v = np.random.default_rng(case.seed + 100).uniform(-1, 1, mesh.x.shape)
    F, md = prob.energy(mesh.x)
    ref = dict(F=F, mindet=md, g=prob.gradient(mesh.x), Hv=prob.hessian_apply(mesh.x, v),
               mixed=mixed_tol(prob, mesh.x, v))
    return case, mesh, W, v, ref


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_evec_against_oracle_and_colours(setup, precision):
    case, mesh, W, v, ref = setup
    ev = _mode(context(case, mesh, W, precision), "ELEMENTS")
    col = _mode(context(case, mesh, W, precision), "COLOURS")
    x, vd = to_dev(mesh.x), to_dev(v)
    tol = dict(F=FP64_TOL, min_detA=1e-12, g=FP64_TOL, Hv=FP64_TOL) if precision == 0 else ref["mixed"]
    g, Hv = ev.gradient(x), ev.hessian_apply(x, vd)
    F, md, st, ge = ev.energy_gradient(x)
    eg, eh = rel_max_err(g.cpu().numpy(), ref["g"]), rel_max_err(Hv.cpu().numpy(), ref["Hv"])
    say(f"  {case.name} prec={precision}: g {eg:.2e} Hv {eh:.2e} (bars {tol['g']:.1e} {tol['Hv']:.1e})")
    assert st == 0 and eg <= tol["g"] and eh <= tol["Hv"]
    assert rel_max_err(ge.cpu().numpy(), ref["g"]) <= tol["g"]
    assert abs(F - ref["F"]) <= tol["F"] * abs(ref["F"])
    assert abs(md - ref["mindet"]) <= tol["min_detA"] * abs(ref["mindet"])
    gc, hc = col.gradient(x), col.hessian_apply(x, vd)
    dg, dh = rel_max_err(g.cpu().numpy(), gc.cpu().numpy()), rel_max_err(Hv.cpu().numpy(), hc.cpu().numpy())
    say(f"  {case.name} prec={precision}: elements vs colours g {dg:.1e} Hv {dh:.1e}")
    same = 1e-14 if precision == 0 else 2 * max(tol["g"], tol["Hv"])
    assert dg <= same and dh <= same
    ev.close()
    col.close()


def test_evec_bitwise_repeatable(setup):
    case, mesh, W, v, ref = setup
    ctx = _mode(context(case, mesh, W, 0), "ELEMENTS")
    x, vd = to_dev(mesh.x), to_dev(v)
    assert torch.equal(ctx.gradient(x), ctx.gradient(x))
    assert torch.equal(ctx.hessian_apply(x, vd), ctx.hessian_apply(x, vd))
    a, b = ctx.energy_gradient(x), ctx.energy_gradient(x)
    assert a[:3] == b[:3] and torch.equal(a[3], b[3])
    ctx.close()


@pytest.mark.parametrize("term", ["sizes", "penalty", "combo"])
def test_evec_with_targets_and_section4(term):
    """Per-point sizes (the kernels read them in element order), the
    displacement penalty fused into the FP64 Hessian action (its share joins
    the element vector) and the second metric term (colour launches adding
    after the gather): against the colour launches."""
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(3, 3, 2)
    W = mesh.h * np.eye(3)
    prob0 = O.Problem(3, 2, 4, mesh.elem_node, 303, W)
    x = meshgen.perturb(mesh, 0.1, 90, bad_elements=prob0.bad_elements)
    x_init = meshgen.perturb(mesh, 0.05, 91, bad_elements=prob0.bad_elements)
    v = np.random.default_rng(92).uniform(-1, 1, x.shape)
    sizes = mesh.h * np.random.default_rng(93).uniform(0.8, 1.2, (mesh.n_elem, 64))
    out = []
    for mode in ("COLOURS", "ELEMENTS"):
        if term == "sizes":
            ctx = T.Context(3, 2, mesh.elem_node, mesh.n_node, 4, 303, None, fixed=mesh.fixed, target_sizes=sizes)
        else:
            ctx = T.Context(3, 2, mesh.elem_node, mesh.n_node, 4, 303, W, fixed=mesh.fixed)
        if term == "penalty":
            ctx.set_restriction(50.0, to_dev(x_init))
        if term == "combo":
            ctx.set_combo(302, mesh.h * np.array([[1.1, 0.1, 0.0], [0.0, 0.9, 0.1], [0.0, 0.0, 1.0]]), 1.0, 0.5)
        _mode(ctx, mode)
        xd, vd = to_dev(x), to_dev(v)
        F, md, st, g = ctx.energy_gradient(xd)
        out.append((F, g.cpu().numpy(), ctx.hessian_apply(xd, vd).cpu().numpy()))
        ctx.close()
    (Fc, gc, hc), (Fe, ge, he) = out
    assert abs(Fe - Fc) <= 1e-13 * abs(Fc)
    assert rel_max_err(ge, gc) <= 1e-14 and rel_max_err(he, hc) <= 1e-14


def test_newton_with_evec():
    """Newton on an 8^3 Q2 hex with each scatter: the same trajectory bar as
    against the oracle's Newton (F within 1e-6 relative while F > 1e-8 F0,
    same iteration count), both back on the grid."""
    from paper_1807_09807_amd import tmop as T
    w = meshgen.WORKLOADS["q2_cube_64"]
    mesh = meshgen.box_mesh(3, 8, 2)
    W = mesh.h * np.eye(3)
    prob = O.Problem(3, 2, 4, mesh.elem_node, 303, W)
    x0 = meshgen.perturb(mesh, w["noise"], w["seed"], bad_elements=prob.bad_elements)
    res = []
    for mode in ("COLOURS", "ELEMENTS"):
        ctx = _mode(T.Context(3, 2, mesh.elem_node, mesh.n_node, 4, 303, W, fixed=mesh.fixed), mode)
        xd = to_dev(x0)
        st, rep = ctx.newton_solve(xd, max_it=30, rtol=1e-10)
        res.append((st, rep, xd.cpu().numpy()))
        ctx.close()
    (sc, rc, xc), (se, re_, xe) = res
    Fc, Fe = rc["history_F"], re_["history_F"]
    worst = max(abs(b - a) / a for a, b in zip(Fc, Fe) if a > 1e-8 * Fc[0])
    say(f"  newton colours {rc['iters']} it, elements {re_['iters']} it, worst relative F difference {worst:.2e}")
    assert sc == se == 0 and rc["iters"] == re_["iters"] and worst <= 1e-6
    assert np.max(np.abs(xe - mesh.x_grid)) < 1e-8 * mesh.h


@pytest.mark.parametrize("dim,n,precision,expect", [(3, 8, 0, "ELEMENTS"), (3, 72, 0, "ELEMENTS"),
                                                      (3, 74, 0, "COLOURS"), (3, 74, 1, "ELEMENTS"),
                                                      (3, 101, 1, "ELEMENTS"), (3, 102, 1, "COLOURS"),
                                                      (2, 16, 0, "ELEMENTS"), (2, 512, 1, "ELEMENTS")])
def test_default_scatter(dim, n, precision, expect):
    """The default mode follows the mesh: in 2D the element vector; in 3D the
    element vector while the 2^3 colours average at most 49,152 elements
    (72^3 Q2: 46,656; 131,072 in the mixed path, 101^3 Q2: 128,788), the
    colour launches above (74^3: 50,653; mixed, 102^3: 132,651).
    tmop_get_scatter reports it, and then what tmop_set_scatter selects."""
    from paper_1807_09807_amd import tmop as T
    say(f"[evec] default scatter dim={dim} n={n} precision={precision}")
    mesh = meshgen.box_mesh(dim, n, 2)
    ctx = T.Context(dim, 2, mesh.elem_node, mesh.n_node, 4, 303 if dim == 3 else 2, mesh.h * np.eye(dim),
                    precision=precision)
    assert ctx.scatter == getattr(T, f"TMOP_SCATTER_{expect}")
    ctx.set_scatter(T.TMOP_SCATTER_COLOURS)
    assert ctx.scatter == T.TMOP_SCATTER_COLOURS
    ctx.close()


def test_modes_switch_back_and_forth_2d():
    """2D: the element vector (default), tiles (built on first selection),
    colours, then the element vector again, bit for bit as the first time;
    tiles refused in 3D."""
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(2, 6, 2)
    x = to_dev(meshgen.perturb(mesh, 0.05, 1))
    ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 2, mesh.h * np.eye(2), fixed=mesh.fixed)
    assert ctx.scatter == T.TMOP_SCATTER_ELEMENTS
    g0 = ctx.gradient(x).clone()
    out = {}
    for mode in (T.TMOP_SCATTER_TILES, T.TMOP_SCATTER_COLOURS, T.TMOP_SCATTER_ELEMENTS):
        ctx.set_scatter(mode)
        assert ctx.scatter == mode
        out[mode] = ctx.gradient(x).clone()
    assert torch.equal(out[T.TMOP_SCATTER_ELEMENTS], g0)
    for mode in (T.TMOP_SCATTER_TILES, T.TMOP_SCATTER_COLOURS):
        assert rel_max_err(out[mode].cpu().numpy(), g0.cpu().numpy()) <= 1e-14
    ctx.close()
    m3 = meshgen.box_mesh(3, 2, 2)
    c3 = T.Context(3, 2, m3.elem_node, m3.n_node, 4, 303, m3.h * np.eye(3))
    with pytest.raises(T.TMOPError) as ei:
        c3.set_scatter(T.TMOP_SCATTER_TILES)
    assert ei.value.status == T.TMOP_E_UNSUPPORTED
    c3.close()


@pytest.mark.parametrize("name", ["q2_cube_32", "q2_cube_64", "q2_square_512", "q3_square_256"])
def test_evec_full_size(name):
    """Full workloads, FP64: every DOF against the colour launches (selected
    explicitly: the element vector is these meshes' default), 64 seeded
    nodes against the oracle."""
    from paper_1807_09807_amd import tmop as T
    w = meshgen.WORKLOADS[name]
    d = w["dim"]
    mesh = meshgen.box_mesh(d, w["n"], w["p"])
    W = mesh.h * np.eye(d)
    prob = O.Problem(d, w["p"], w["Q"], mesh.elem_node, w["metric"], W)
    say(f"[evec full] {name}: building")
    mesh = meshgen.make_workload(name, bad_elements=lambda x, e: prob.bad_elements(x, e, w["tau_min"]))
    x = mesh.x
    v = meshgen.random_direction(mesh, w["seed"] + 100)
    nodes = np.random.default_rng(w["seed"] + 200).choice(mesh.n_node, 64, replace=False)
    ctx = T.Context(d, w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W, fixed=mesh.fixed)
    assert ctx.scatter == T.TMOP_SCATTER_ELEMENTS
    xd, vd = to_dev(x), to_dev(v)
    ge, he = ctx.gradient(xd), ctx.hessian_apply(xd, vd)
    ctx.set_scatter(T.TMOP_SCATTER_COLOURS)
    gc, hc = ctx.gradient(xd), ctx.hessian_apply(xd, vd)
    ctx.close()
    dg = rel_max_err(ge.cpu().numpy(), gc.cpu().numpy())
    dh = rel_max_err(he.cpu().numpy(), hc.cpu().numpy())
    idx = torch.from_numpy(nodes).cuda()
    g_ref, h_ref = prob.gradient_at(x, nodes), prob.hessian_apply_at(x, v, nodes)
    eg = np.max(np.abs(ge[:, idx].cpu().numpy() - g_ref)) / np.max(np.abs(g_ref))
    eh = np.max(np.abs(he[:, idx].cpu().numpy() - h_ref)) / np.max(np.abs(h_ref))
    say(f"  {name}: elements vs colours g {dg:.1e} Hv {dh:.1e}; vs oracle at 64 nodes g {eg:.1e} Hv {eh:.1e}")
    assert dg <= 1e-14 and dh <= 1e-14 and eg <= FP64_TOL and eh <= FP64_TOL


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_evec_runs_of_any_length(precision):
    """The sum over a node's entries for runs outside a structured quad
    mesh's 1 to 4: five Q2 quadrilaterals around one vertex (a run of 5,
    past the unrolled loads) and one node that no element uses (a run of 0,
    whose gradient, Hessian action and diagonal are zero).  Against the
    oracle at the FP64 bar, or the mixed path's rounding bound."""
    from tests.test_dfo_gpu import _pentagon
    from paper_1807_09807_amd import tmop as T
    x, en, _ = _pentagon()
    x = np.concatenate([x, [[2.0], [2.0]]], axis=1)          # the unused node
    n = x.shape[1]
    W = 0.8 * np.eye(2)
    prob = O.Problem(2, 2, 4, en, 2, W)
    v = np.random.default_rng(7).uniform(-1, 1, x.shape)
    ref = dict(g=prob.gradient(x), Hv=prob.hessian_apply(x, v), D=prob.hessian_diagonal(x))
    assert np.all(ref["g"][:, -1] == 0) and np.all(ref["D"][:, -1] == 0)
    tol = dict(g=FP64_TOL, Hv=FP64_TOL, diag=FP64_TOL) if precision == 0 else mixed_tol(prob, x, v, diag=True)
    ctx = T.Context(2, 2, en, n, 4, 2, W, precision=precision)
    assert ctx.scatter == T.TMOP_SCATTER_ELEMENTS
    xd, vd = to_dev(x), to_dev(v)
    g, Hv, D = ctx.gradient(xd).cpu().numpy(), ctx.hessian_apply(xd, vd).cpu().numpy(), \
        ctx.hessian_diagonal(xd).cpu().numpy()
    eg, eh, ed = rel_max_err(g, ref["g"]), rel_max_err(Hv, ref["Hv"]), rel_max_err(D, ref["D"])
    say(f"  pentagon prec={precision}: g {eg:.2e} Hv {eh:.2e} diag {ed:.2e}")
    assert eg <= tol["g"] and eh <= tol["Hv"] and ed <= tol["diag"]
    assert np.all(g[:, -1] == 0) and np.all(Hv[:, -1] == 0) and np.all(D[:, -1] == 0)
    ctx.close()


@pytest.mark.parametrize("dim,copies", [(2, 8), (3, 4)], ids=["2d_x8", "3d_x4"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_evec_long_runs(precision, dim, copies):
    """Every element of a Q2 block (4x4, or 3x3x3) given several times (8 in
    2D, 4 in 3D): runs of up to 32 entries per node, beyond the unrolled
    loads, and more entries in a block of 256 nodes than the FP32 gather
    stages (1,024 in 2D, 2,048 in 3D), so its per-lane fallback runs (in 3D
    the second block of nodes is staged).  Against the oracle on the same
    connectivity."""
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(dim, 4 if dim == 2 else 3, 2)
    x = meshgen.perturb(mesh, 0.1, seed=5)
    en = np.tile(np.asarray(mesh.elem_node), (copies, 1))
    W = mesh.h * np.eye(dim)
    metric = 2 if dim == 2 else 303
    prob = O.Problem(dim, 2, 4, en, metric, W)
    v = np.random.default_rng(8).uniform(-1, 1, x.shape)
    ref = dict(g=prob.gradient(x), Hv=prob.hessian_apply(x, v), D=prob.hessian_diagonal(x))
    tol = dict(g=FP64_TOL, Hv=FP64_TOL, diag=FP64_TOL) if precision == 0 else mixed_tol(prob, x, v, diag=True)
    ctx = T.Context(dim, 2, en, mesh.n_node, 4, metric, W, precision=precision)
    assert ctx.scatter == T.TMOP_SCATTER_ELEMENTS
    xd, vd = to_dev(x), to_dev(v)
    g, Hv, D = ctx.gradient(xd).cpu().numpy(), ctx.hessian_apply(xd, vd).cpu().numpy(), \
        ctx.hessian_diagonal(xd).cpu().numpy()
    eg, eh, ed = rel_max_err(g, ref["g"]), rel_max_err(Hv, ref["Hv"]), rel_max_err(D, ref["D"])
    say(f"  {dim}D x{copies} prec={precision}: g {eg:.2e} Hv {eh:.2e} diag {ed:.2e}")
    assert eg <= tol["g"] and eh <= tol["Hv"] and ed <= tol["diag"]
    ctx.close()
