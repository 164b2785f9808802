"""Degenerate and edge cases of the element operations on the GPU."""
import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen
from tests._helpers import rel_max_err, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _ctx(mesh, Q, metric, W=None, precision=0):
    from paper_1807_09807_amd import tmop as T
    W = mesh.h * np.eye(mesh.dim) if W is None else W
    return T.Context(mesh.dim, mesh.order, mesh.elem_node, mesh.n_node, Q, metric, W, fixed=mesh.fixed,
                     precision=precision)


@pytest.mark.parametrize("dim,p,Q,metric", [(2, 2, 4, 2), (2, 3, 5, 7), (3, 2, 4, 303), (3, 3, 5, 302)])
@pytest.mark.parametrize("precision", [0, 1])
def test_grid_is_zero(dim, p, Q, metric, precision):
    """T = I everywhere on the unperturbed grid: F = 0 and g = 0."""
    say(f"[edge] grid dim={dim} p={p} metric={metric} prec={precision}")
    mesh = meshgen.box_mesh(dim, 4, p)
    ctx = _ctx(mesh, Q, metric, precision=precision)
    x = to_dev(mesh.x_grid)
    F, md, st = ctx.energy(x)
    g = ctx.gradient(x)
    # FP32: mu_303 and mu_302 have no cancellation-free form, so each point
    # may carry one FP32 rounding of "... - 1" (sum of w det W = 1)
    assert st == 0 and abs(F) < (1e-14 if precision == 0 else 4 * 2.0 ** -24)
    assert md == pytest.approx(mesh.h ** dim, rel=1e-12 if precision == 0 else 1e-6)
    assert float(g.abs().max()) < (1e-12 if precision == 0 else 1e-5) / mesh.h


@pytest.mark.parametrize("dim,p,Q,metric", [(2, 2, 4, 2), (3, 2, 4, 303)])
def test_inverted_mesh_warns(dim, p, Q, metric):
    """An interior node pushed past its neighbour inverts elements: the energy call reports
    TMOP_W_INVERTED with the (negative) smallest det A, as the oracle."""
    from paper_1807_09807_amd import tmop as T
    say(f"[edge] inverted dim={dim}")
    mesh = meshgen.box_mesh(dim, 4, p)
    x = mesh.x_grid.copy()
    m = mesh.n * p + 1
    a = m + 1 if dim == 2 else m * m + m + 1          # first interior node
    x[0, a] += 1.2 * mesh.h                           # push it past its neighbour
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, mesh.h * np.eye(dim))
    Fo, mdo = prob.energy(x)
    F, md, st = _ctx(mesh, Q, metric).energy(to_dev(x))
    assert st == T.TMOP_W_INVERTED and md < 0
    assert md == pytest.approx(mdo, rel=1e-12)
    assert F == pytest.approx(Fo, rel=1e-10)


@pytest.mark.parametrize("dim,p,Q,metric", [(2, 1, 2, 2), (2, 4, 5, 7), (3, 1, 2, 303), (3, 3, 4, 302)])
def test_single_element(dim, p, Q, metric):
    say(f"[edge] single element dim={dim} p={p}")
    mesh = meshgen.box_mesh(dim, 1, p)
    W = np.eye(dim)
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, W)
    x = meshgen.perturb(mesh, 0.0, 0) + np.random.default_rng(3).uniform(-0.05, 0.05, mesh.x_grid.shape)
    v = np.random.default_rng(4).uniform(-1, 1, x.shape)
    ctx = _ctx(mesh, Q, metric, W)
    F, md, st = ctx.energy(to_dev(x))
    assert abs(F - prob.energy(x)[0]) <= 1e-12 * abs(prob.energy(x)[0])
    assert rel_max_err(ctx.gradient(to_dev(x)).cpu().numpy(), prob.gradient(x)) <= 1e-12
    assert rel_max_err(ctx.hessian_apply(to_dev(x), to_dev(v)).cpu().numpy(), prob.hessian_apply(x, v)) <= 1e-12


def test_outputs_overwritten_and_aliasing_rejected():
    from paper_1807_09807_amd import tmop as T
    mesh = meshgen.box_mesh(2, 5, 2)
    prob = O.Problem(2, 2, 4, mesh.elem_node, 2, mesh.h * np.eye(2))
    x = meshgen.perturb(mesh, 0.1, 2, bad_elements=prob.bad_elements)
    ctx = _ctx(mesh, 4, 2)
    xd = to_dev(x)
    out = torch.full_like(xd, float("nan"))
    ctx.gradient(xd, out)
    assert rel_max_err(out.cpu().numpy(), prob.gradient(x)) <= 1e-12
    lib = T.load()
    import ctypes
    st = lib.tmop_gradient(ctx.handle, ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(xd.data_ptr()), None)
    assert st == T.TMOP_E_ARG
    with pytest.raises(ValueError):
        ctx.gradient(xd[:, :-1].contiguous())


def test_unused_nodes_get_zero():
    """A node no element references has zero gradient and Hessian action."""
    mesh = meshgen.box_mesh(2, 3, 2)
    n_node = mesh.n_node + 1
    x = np.concatenate([mesh.x_grid, np.array([[5.0], [5.0]])], axis=1)
    x[:, :mesh.n_node] += np.random.default_rng(1).uniform(-0.01, 0.01, mesh.x_grid.shape) * (1 - mesh.fixed)
    from paper_1807_09807_amd import tmop as T
    ctx = T.Context(2, 2, mesh.elem_node, n_node, 4, 2, mesh.h * np.eye(2))
    g = ctx.gradient(to_dev(x)).cpu().numpy()
    Hv = ctx.hessian_apply(to_dev(x), to_dev(np.ones_like(x))).cpu().numpy()
    assert g[0, -1] == 0.0 and g[1, -1] == 0.0 and Hv[0, -1] == 0.0 and Hv[1, -1] == 0.0


@pytest.mark.parametrize("mode,launches", [("COLOURS", 8), ("ELEMENTS", 1)])
def test_kernel_timing_counts_launches(mode, launches):
    """Timing on: one energy launch per energy call; for gradient and
    Hessian action one launch per colour (2^dim colours on a box mesh with at
    least two elements per direction) or one launch over every element with
    the element vector; results unchanged by timing."""
    from paper_1807_09807_amd import tmop as T
    say(f"[edge] kernel timing {mode}")
    mesh = meshgen.box_mesh(3, 4, 2)
    ctx = _ctx(mesh, 4, 303)
    ctx.set_scatter(getattr(T, f"TMOP_SCATTER_{mode}"))
    x = to_dev(meshgen.perturb(mesh, 0.05, 1))
    v = to_dev(meshgen.random_direction(mesh, 2))
    h0 = ctx.hessian_apply(x, v).clone()
    ctx.timing_enable(True)
    for _ in range(3):
        ctx.energy(x)
        ctx.gradient(x)
        h1 = ctx.hessian_apply(x, v)
    counts = [ctx.timing_read(op) for op in range(3)]
    ctx.timing_enable(False)
    assert [n for _, n in counts] == [3, 3 * launches, 3 * launches]
    assert all(ms > 0 for ms, _ in counts)
    assert torch.equal(h0, h1)
    ctx.energy(x)
    assert ctx.timing_read(0) == (0.0, 0)


@pytest.mark.parametrize("dim,p,Q,metric", [(2, 1, 2, 2), (2, 4, 5, 9), (3, 1, 2, 303), (3, 3, 4, 302)])
def test_single_element_section4(dim, p, Q, metric):
    """One element with every Section 4 term at once (the replication
    composite and the displacement penalty), against the oracle."""
    say(f"[edge] single element + Section 4 dim={dim} p={p}")
    mesh = meshgen.box_mesh(dim, 1, p)
    W = np.eye(dim)
    prob = O.Problem(dim, p, Q, mesh.elem_node, metric, W)
    rng = np.random.default_rng(5)
    x0 = mesh.x_grid + rng.uniform(-0.05, 0.05, mesh.x_grid.shape)
    x = x0 + rng.uniform(-0.03, 0.03, x0.shape)
    v = rng.uniform(-1, 1, x.shape)
    prob.set_replication(0.3, x0)
    prob.set_restriction(7.0, x0)
    ctx = _ctx(mesh, Q, metric, W)
    ctx.set_replication(0.3, to_dev(x0))
    ctx.set_restriction(7.0, to_dev(x0))
    F, md, st = ctx.energy(to_dev(x))
    assert st == 0 and abs(F - prob.energy(x)[0]) <= 1e-12 * abs(prob.energy(x)[0])
    assert rel_max_err(ctx.gradient(to_dev(x)).cpu().numpy(), prob.gradient(x)) <= 1e-12
    assert rel_max_err(ctx.hessian_apply(to_dev(x), to_dev(v)).cpu().numpy(), prob.hessian_apply(x, v)) <= 1e-12
    assert rel_max_err(ctx.hessian_diagonal(to_dev(x)).cpu().numpy(), prob.hessian_diagonal(x)) <= 1e-12


def test_unused_nodes_get_zero_with_penalty():
    """The penalty kernels leave a node no element references at zero."""
    mesh = meshgen.box_mesh(2, 3, 2)
    n_node = mesh.n_node + 1
    x = np.concatenate([mesh.x_grid, np.array([[5.0], [5.0]])], axis=1)
    x[:, :mesh.n_node] += np.random.default_rng(1).uniform(-0.01, 0.01, mesh.x_grid.shape) * (1 - mesh.fixed)
    from paper_1807_09807_amd import tmop as T
    ctx = T.Context(2, 2, mesh.elem_node, n_node, 4, 2, mesh.h * np.eye(2))
    ctx.set_restriction(3.0, to_dev(x + 0.01))
    for out in (ctx.gradient(to_dev(x)), ctx.hessian_apply(to_dev(x), to_dev(np.ones_like(x))),
                ctx.hessian_diagonal(to_dev(x))):
        o = out.cpu().numpy()
        assert o[0, -1] == 0.0 and o[1, -1] == 0.0 and np.all(np.isfinite(o))


def test_dfo_with_every_node_fixed_moves_nothing():
    mesh = meshgen.box_mesh(2, 1, 2)
    from paper_1807_09807_amd import tmop as T
    fixed = np.ones((2, mesh.n_node), dtype=np.uint8)
    ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 3, 2, mesh.h * np.eye(2), fixed=fixed)
    x = to_dev(mesh.x_grid + 0.01)
    x0 = x.clone()
    assert ctx.dfo_sweep(x) == 0.0 and torch.equal(x, x0)
    st, rep = ctx.dfo_solve(x)
    assert st == T.TMOP_OK and rep["sweeps"] == 1 and rep["converged"] == 1
