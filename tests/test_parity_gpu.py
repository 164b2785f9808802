"""Parity of the HIP path with the FP64 oracle (energy, gradient, Hessian
action), element by element, on seeded meshes: FP64 within 1e-12
relative, the mixed FP32 path within the first-order rounding bound of each
result (tests/_helpers.mixed_tol)."""
import numpy as np
import pytest

from tests._helpers import build, context, mixed_tol, rel_max_err, say, small_cases, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP64_TOL = 1e-12
CASES = small_cases()


@pytest.fixture(scope="module", params=CASES, ids=str)
def setup(request):
    case = request.param
    say(f"[parity] case {case.name}")
    mesh, prob, W = build(case)
    v = np.random.default_rng(case.seed + 100).uniform(-1, 1, mesh.x.shape)
    F, md = prob.energy(mesh.x)
    ref = dict(F=F, mindet=md, g=prob.gradient(mesh.x), Hv=prob.hessian_apply(mesh.x, v),
               mixed=mixed_tol(prob, mesh.x, v))
    return case, mesh, W, v, ref


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_energy(setup, precision):
    case, mesh, W, v, ref = setup
    ctx = context(case, mesh, W, precision)
    F, md, st = ctx.energy(to_dev(mesh.x))
    tol = FP64_TOL if precision == 0 else ref["mixed"]["F"]
    say(f"  {case.name} prec={precision} F={F!r} ref={ref['F']!r} rel={abs(F - ref['F']) / ref['F']:.2e} "
        f"(bar {tol:.1e})")
    assert st == 0
    assert abs(F - ref["F"]) <= tol * abs(ref["F"])
    # det A is always evaluated in FP64 from the contracted A
    assert abs(md - ref["mindet"]) <= (1e-12 if precision == 0 else ref["mixed"]["min_detA"]) * abs(ref["mindet"])


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_gradient(setup, precision):
    case, mesh, W, v, ref = setup
    ctx = context(case, mesh, W, precision)
    g = ctx.gradient(to_dev(mesh.x)).cpu().numpy()
    err = rel_max_err(g, ref["g"])
    tol = FP64_TOL if precision == 0 else ref["mixed"]["g"]
    say(f"  {case.name} prec={precision} grad rel err {err:.2e} (bar {tol:.1e})")
    assert err <= tol


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_hessian_apply(setup, precision):
    case, mesh, W, v, ref = setup
    ctx = context(case, mesh, W, precision)
    Hv = ctx.hessian_apply(to_dev(mesh.x), to_dev(v)).cpu().numpy()
    err = rel_max_err(Hv, ref["Hv"])
    tol = FP64_TOL if precision == 0 else ref["mixed"]["Hv"]
    say(f"  {case.name} prec={precision} Hv rel err {err:.2e} (bar {tol:.1e})")
    assert err <= tol


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_energy_gradient_one_pass(setup, precision):
    """The fused pass gives the oracle's F, min det A and g, and the separate
    calls' g to rounding: the same arithmetic in another kernel
    instantiation, where the compiler may fuse a different set of products
    and sums into FMAs (often bit for bit, not always: FP64 within 1e-14;
    mixed, two FP32 evaluations each within the first-order rounding bound
    of the oracle's g, so within twice that bound of each other); F differs
    from the energy call only in its summation order."""
    case, mesh, W, v, ref = setup
    ctx = context(case, mesh, W, precision)
    x = to_dev(mesh.x)
    F, md, st, g = ctx.energy_gradient(x)
    tol = dict(F=FP64_TOL, min_detA=1e-12, g=FP64_TOL) if precision == 0 else ref["mixed"]
    assert st == 0
    assert abs(F - ref["F"]) <= tol["F"] * abs(ref["F"])
    assert abs(md - ref["mindet"]) <= tol["min_detA"] * abs(ref["mindet"])
    assert rel_max_err(g.cpu().numpy(), ref["g"]) <= tol["g"]
    F1, md1, _ = ctx.energy(x)
    assert abs(F - F1) <= 1e-13 * abs(F1) and md == md1
    g1 = ctx.gradient(x)
    d = rel_max_err(g.cpu().numpy(), g1.cpu().numpy())
    if d > 0.0:
        say(f"  {case.name} prec={precision}: fused and separate gradients differ by {d:.2e} (relative)")
    assert d <= (1e-14 if precision == 0 else 2 * tol["g"])


def test_bitwise_deterministic(setup):
    case, mesh, W, v, ref = setup
    ctx = context(case, mesh, W, 0)
    x, vd = to_dev(mesh.x), to_dev(v)
    g1, g2 = ctx.gradient(x), ctx.gradient(x)
    h1, h2 = ctx.hessian_apply(x, vd), ctx.hessian_apply(x, vd)
    e1, e2 = ctx.energy(x), ctx.energy(x)
    assert torch.equal(g1, g2) and torch.equal(h1, h2) and e1 == e2
