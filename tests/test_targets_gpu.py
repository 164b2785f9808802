"""Per-quadrature-point isotropic targets W_q = s_q I (Section 3.1: W may be
given at every point; W_3 = (det A(x_0))^(1/d) I and space-scaled W_2 are
of this form) in the HIP library, against the oracle with the same
per-point W: energy, gradient, Hessian action and diagonal element by
element (FP64 within 1e-12 relative, mixed FP32 within the mixed
tolerance), the W_3 sizes of a mesh, size validation, and Newton with
mu_9 and the W_3 target (the shape + initial size optimization of
Section 5.2.2)."""
import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen
from tests._helpers import mixed_tol, rel_max_err, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [  # dim, n, p, Q, metric, noise, seed
    (2, 6, 2, 4, 2, 0.10, 50),
    (2, 5, 3, 5, 9, 0.08, 51),
    (2, 7, 1, 2, 77, 0.12, 52),
    (3, 3, 2, 4, 303, 0.10, 53),
    (3, 2, 3, 4, 302, 0.05, 54),
]


def _case(dim, n, p, Q, metric, noise, seed):
    mesh = meshgen.box_mesh(dim, n, p)
    prob0 = O.Problem(dim, p, Q, mesh.elem_node, metric, mesh.h * np.eye(dim))
    x = meshgen.perturb(mesh, noise, seed, bad_elements=prob0.bad_elements)
    sizes = mesh.h * np.random.default_rng(seed + 1).uniform(0.7, 1.3, (mesh.n_elem, Q ** dim))
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, sizes[:, :, None, None] * np.eye(dim))
    return mesh, prob, x, sizes


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}d_p{c[2]}_q{c[3]}_mu{c[4]}")
def setup(request):
    dim, n, p, Q, metric, noise, seed = request.param
    say(f"[targets] case {request.param}")
    mesh, prob, x, sizes = _case(*request.param)
    v = np.random.default_rng(seed + 2).uniform(-1, 1, x.shape)
    F, md = prob.energy(x)
    ref = dict(F=F, md=md, g=prob.gradient(x), Hv=prob.hessian_apply(x, v), D=prob.hessian_diagonal(x),
               mtol=mixed_tol(prob, x, v, diag=True))
    return request.param, mesh, x, v, sizes, ref


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_per_point_targets(setup, precision):
    from paper_1807_09807_amd import tmop as T
    (dim, n, p, Q, metric, _, _), mesh, x, v, sizes, ref = setup
    ctx = T.Context(dim, p, mesh.elem_node, mesh.n_node, Q, metric, None, fixed=mesh.fixed, precision=precision,
                    target_sizes=sizes)
    xd, vd = to_dev(x), to_dev(v)
    tol = dict(F=1e-12, min_detA=1e-12, g=1e-12, Hv=1e-12, diag=1e-12) if precision == 0 else ref["mtol"]
    F, md, st = ctx.energy(xd)
    eg = rel_max_err(ctx.gradient(xd).cpu().numpy(), ref["g"])
    eh = rel_max_err(ctx.hessian_apply(xd, vd).cpu().numpy(), ref["Hv"])
    ed = rel_max_err(ctx.hessian_diagonal(xd).cpu().numpy(), ref["D"])
    Fe, mde, _, ge = ctx.energy_gradient(xd)
    say(f"  prec={precision}: F rel {abs(F - ref['F']) / abs(ref['F']):.2e} g {eg:.2e} Hv {eh:.2e} diag {ed:.2e} "
        f"(bars g {tol['g']:.1e} Hv {tol['Hv']:.1e})")
    assert st == 0
    assert abs(F - ref["F"]) <= tol["F"] * abs(ref["F"]) and abs(Fe - ref["F"]) <= tol["F"] * abs(ref["F"])
    assert abs(md - ref["md"]) <= tol["min_detA"] * abs(ref["md"]) and md == mde
    assert eg <= tol["g"] and eh <= tol["Hv"] and ed <= tol["diag"]
    assert rel_max_err(ge.cpu().numpy(), ref["g"]) <= tol["g"]


@pytest.mark.parametrize("dim,p,Q", [(2, 2, 4), (3, 2, 3), (2, 3, 5)])
def test_w3_sizes(dim, p, Q):
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(dim, 4, p)
    metric = 2 if dim == 2 else 303
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, mesh.h * np.eye(dim))
    x0 = meshgen.perturb(mesh, 0.1, 60 + dim, bad_elements=prob.bad_elements)
    ctx = T.Context(dim, p, mesh.elem_node, mesh.n_node, Q, metric, mesh.h * np.eye(dim), fixed=mesh.fixed)
    s, st = ctx.target_sizes_w3(to_dev(x0))
    ref = prob.point_sizes(x0)
    assert st == T.TMOP_OK
    assert rel_max_err(s.cpu().numpy(), ref) <= 1e-13
    # an inverted element is reported
    x = x0.copy()
    a = (mesh.n * p + 1) + 1          # an interior node next to node a + 1
    x[:, [a, a + 1]] = x[:, [a + 1, a]]
    _, st = ctx.target_sizes_w3(to_dev(x))
    assert st == T.TMOP_W_INVERTED


def test_set_target_sizes_validation():
    from paper_1807_09807_amd import tmop as T
    mesh, prob, x, sizes = _case(*CASES[0])
    ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 2, None, fixed=mesh.fixed, target_sizes=sizes)
    xd = to_dev(x)
    F0 = ctx.energy(xd)[0]
    bad = torch.from_numpy(sizes).cuda().clone()
    bad[3, 5] = 0.0
    with pytest.raises(T.TMOPError) as ei:
        ctx.set_target_sizes(bad)
    assert ei.value.status == T.TMOP_E_TARGET
    bad[3, 5] = float("nan")
    with pytest.raises(T.TMOPError):
        ctx.set_target_sizes(bad)
    assert ctx.energy(xd)[0] == F0                        # unchanged
    ctx.set_target_sizes(torch.from_numpy(2.0 * sizes).cuda())
    # mu_2 is a shape metric: doubling every size leaves T's shape and scales det W by 4
    assert ctx.energy(xd)[0] == pytest.approx(4.0 * F0, rel=1e-13)
    const = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 2, mesh.h * np.eye(2))
    with pytest.raises(T.TMOPError):
        const.set_target_sizes(torch.from_numpy(sizes).cuda())


def test_newton_mu9_w3_target():
    """Shape + initial size (Section 5.2.2 with synthetic data): mu_9 with
    the W_3 target of the initial mesh.  The GPU's W_3 sizes feed both
    sides; F history against the oracle for the first steps, convergence to
    the Newton tolerance on both."""
    from paper_1807_09807_amd import tmop as T
    say("[targets] newton mu_9 + W_3")
    mesh = meshgen.box_mesh(2, 6, 2)
    prob0 = O.Problem(2, 2, 4, mesh.elem_node, 9, mesh.h * np.eye(2))
    x0 = meshgen.perturb(mesh, 0.15, 70, bad_elements=prob0.bad_elements)
    s_ref = prob0.point_sizes(x0)
    ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 9, None, fixed=mesh.fixed,
                    target_sizes=np.full((mesh.n_elem, 16), mesh.h))
    xd = to_dev(x0)
    s, st = ctx.target_sizes_w3(xd)
    assert st == 0 and rel_max_err(s.cpu().numpy(), s_ref) <= 1e-13
    ctx.set_target_sizes(s)
    prob = O.Problem(2, 2, 4, mesh.elem_node, 9, s_ref[:, :, None, None] * np.eye(2))
    xo, rep_o = O.newton_solve(prob, x0, mesh.fixed, O.NewtonOptions(max_it=40, cg_rtol=1e-10))
    st, rep = ctx.newton_solve(xd, max_it=40, cg_rtol=1e-10)
    F_o = [h[0] for h in rep_o.history]
    F_g = rep["history_F"]
    say(f"  oracle {rep_o.iters} it F {F_o[0]:.6e} -> {F_o[-1]:.3e}; gpu {rep['iters']} it -> {F_g[-1]:.3e}")
    assert st == T.TMOP_OK and rep_o.stop == O.STOP_CONVERGED
    for k in range(3):
        assert abs(F_g[k] - F_o[k]) <= 1e-9 * abs(F_o[k])
    x = xd.cpu().numpy()
    assert np.max(np.abs(x - xo)) < 1e-6 * mesh.h
    assert F_g[-1] < F_g[0]


def test_learned_guess_needs_a_constant_target():
    """The MLP works in units of a constant target size h; a context with
    per-point targets is refused (TMOP_E_UNSUPPORTED), not run with h = 1."""
    from paper_1807_09807_amd import mlp as ML
    from paper_1807_09807_amd import tmop as T
    mesh, prob, x, sizes = _case(*CASES[0])
    ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, 2, None, fixed=mesh.fixed, target_sizes=sizes)
    with pytest.raises(T.TMOPError) as ei:
        ML.features(ctx, to_dev(x))
    assert ei.value.status == T.TMOP_E_UNSUPPORTED
