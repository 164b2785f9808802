"""The seeded input generator: topology, sizes, determinism, repair."""
import numpy as np
import pytest

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen


@pytest.mark.parametrize("name,dofs", [("q2_square_8", 578), ("q3_square_256", 1_182_722),
                                       ("q2_cube_64", 6_440_067), ("q3_cube_48", 9_145_875),
                                       ("q2_square_512", 2_101_250), ("q2_cube_32", 3 * 65 ** 3)])
def test_workload_sizes(name, dofs):
    w = meshgen.WORKLOADS[name]
    m = w["n"] * w["p"] + 1
    assert w["dim"] * m ** w["dim"] == dofs


@pytest.mark.parametrize("dim,n,p", [(2, 3, 2), (2, 2, 3), (3, 2, 2), (3, 2, 3)])
def test_box_topology(dim, n, p):
    mesh = meshgen.box_mesh(dim, n, p)
    P = p + 1
    assert mesh.elem_node.shape == (n ** dim, P ** dim)
    assert mesh.n_node == (n * p + 1) ** dim
    # every node is used; vertices of the box are in exactly one element
    counts = np.bincount(mesh.elem_node.ravel(), minlength=mesh.n_node)
    assert counts.min() >= 1 and counts.max() == 2 ** dim
    # local lexicographic order: the element's nodes sit at (e + xi)/n
    xi = meshgen.gll_points_unit(p)
    e = n ** dim - 1                                  # last element
    X = mesh.x_grid[:, mesh.elem_node[e]]
    assert X[0, 1] - X[0, 0] == pytest.approx((xi[1] - xi[0]) / n)
    assert X[1, P] - X[1, 0] == pytest.approx((xi[1] - xi[0]) / n)
    assert X[0, 0] == pytest.approx((n - 1 + xi[0]) / n)
    # boundary mask: exactly the nodes on the faces of the box
    on_bnd = np.any((mesh.x_grid < 1e-12) | (mesh.x_grid > 1 - 1e-12), axis=0)
    np.testing.assert_array_equal(mesh.fixed[0].astype(bool), on_bnd)


def test_perturbation_deterministic_and_boundary_fixed():
    mesh = meshgen.box_mesh(2, 6, 2)
    a = meshgen.perturb(mesh, 0.1, 5)
    b = meshgen.perturb(mesh, 0.1, 5)
    np.testing.assert_array_equal(a, b)
    fx = mesh.fixed.astype(bool)
    np.testing.assert_array_equal(a[fx], mesh.x_grid[fx])
    d = np.abs(a - mesh.x_grid)[~fx]
    assert d.max() <= 0.1 * mesh.h and d.max() > 0.05 * mesh.h


def test_repair_removes_inversions():
    w = meshgen.WORKLOADS["q3_square_256"]
    mesh = meshgen.box_mesh(2, 16, 3)
    prob = O.Problem(2, 3, w["Q"], mesh.elem_node, 7, mesh.h * np.eye(2))
    base = mesh.x_grid + meshgen.sinusoid(mesh, 0.05)
    raw = meshgen.perturb(mesh, w["noise"], w["seed"], base=base)
    assert prob.bad_elements(raw).size > 0          # the literal noise level inverts some Q3 elements
    bad = lambda x, e: prob.bad_elements(x, e, w["tau_min"])
    x = meshgen.perturb(mesh, w["noise"], w["seed"], base=base, bad_elements=bad)
    assert prob.bad_elements(x, None, w["tau_min"]).size == 0
    assert prob.element_min_det(x).min() > w["tau_min"] * mesh.h ** 2
    assert mesh.info["repair_rounds"] >= 1
    x2 = meshgen.perturb(mesh, w["noise"], w["seed"], base=base, bad_elements=bad)
    np.testing.assert_array_equal(x, x2)
    # the incremental re-check agrees with a full one
    untouched = np.setdiff1d(np.arange(mesh.n_elem), bad(x, None))
    assert untouched.size == mesh.n_elem


def test_training_mesh_valid():
    mesh = meshgen.box_mesh(2, 8, 2)
    prob = O.Problem(2, 2, 4, mesh.elem_node, 2, mesh.h * np.eye(2))
    tm = meshgen.training_mesh(8, 1000, bad_elements=prob.bad_elements)
    assert prob.bad_elements(tm.x).size == 0
    assert 1 <= tm.info["kx"] <= 4 and 1 <= tm.info["ky"] <= 4


def test_sliding_boundary_mask():
    """slide=True fixes only the component normal to each boundary face a
    node lies on (Section 4.1, axis-parallel boundaries); interior nodes are
    free and the perturbation leaves the boundary alone."""
    for dim in (2, 3):
        m = meshgen.box_mesh(dim, 3, 2, slide=True)
        full = meshgen.box_mesh(dim, 3, 2)
        x = m.x_grid
        for c in range(dim):
            on = (np.abs(x[c]) < 1e-15) | (np.abs(x[c] - 1.0) < 1e-15)
            np.testing.assert_array_equal(m.fixed[c].astype(bool), on)
        # a node is fixed in some component exactly when it is on the boundary
        np.testing.assert_array_equal(m.fixed.any(axis=0), full.fixed.any(axis=0))
        xp = meshgen.perturb(m, 0.1, 1)
        bnd = full.fixed.any(axis=0)
        np.testing.assert_array_equal(xp[:, bnd], x[:, bnd])
