"""Seeded synthetic high-order box meshes (inputs only).

This module produces the *inputs* of the mesh-optimization problem: the
topology of a structured quad/hex mesh of the unit box, the coordinate
vector x of a continuous Q_p position field (paper, Section 2.1, eq. 2.1),
the Dirichlet mask of the boundary degrees of freedom, and seeded
perturbations of the nodes.  It deliberately holds none of the method's
arithmetic (no Jacobians, no metrics, no quadrature): where a perturbed mesh
must be checked for inverted elements, the caller passes a function that
returns the ids of the bad elements.

Conventions (shared by everything that consumes these arrays):

* Reference element [0,1]^d; element nodes sit on the tensor grid of the
  1D Gauss-Lobatto-Legendre (GLL) points of order p, local index
  i = i0 + (p+1)*(i1 + (p+1)*i2) (first coordinate fastest).
* Elements are numbered lexicographically, e = e0 + n*(e1 + n*e2); the
  global grid node (j0, j1, j2), j_c = e_c*p + i_c, has index
  I = j0 + m*(j1 + m*j2) with m = n*p + 1.
* x is stored component-major ("SoA"): x[c, I], shape (d, n_node), float64.
* fixed[c, I] = 1 marks a Dirichlet degree of freedom; every component of
  every node on the boundary of the box is fixed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


def gll_points_unit(p: int) -> np.ndarray:
    """The p+1 Gauss-Lobatto-Legendre points on [0,1]: both endpoints plus
    the roots of the derivative of the degree-p Legendre polynomial."""
    if p < 1:
        raise ValueError("order must be >= 1")
    if p == 1:
        t = np.array([-1.0, 1.0])
    else:
        dP = np.polynomial.legendre.Legendre.basis(p).deriv()
        inner = np.sort(np.real(dP.roots()))
        # polish the interior roots with a few Newton steps on P_p'
        d2P = dP.deriv()
        for _ in range(3):
            inner = inner - dP(inner) / d2P(inner)
        t = np.concatenate(([-1.0], inner, [1.0]))
    return 0.5 * (t + 1.0)


@dataclass
class BoxMesh:
    dim: int
    order: int
    n: int                      # elements per direction
    elem_node: np.ndarray       # int32 (n_elem, (p+1)^d)
    x_grid: np.ndarray          # float64 (d, n_node), unperturbed positions
    fixed: np.ndarray           # uint8 (d, n_node), 1 = Dirichlet DOF
    x: Optional[np.ndarray] = None   # perturbed positions (d, n_node)
    info: dict = field(default_factory=dict)

    @property
    def n_elem(self) -> int:
        return int(self.elem_node.shape[0])

    @property
    def n_node(self) -> int:
        return int(self.x_grid.shape[1])

    @property
    def h(self) -> float:
        return 1.0 / self.n

    @property
    def n_dof(self) -> int:
        return self.dim * self.n_node


def box_mesh(dim: int, n: int, order: int, slide: bool = False) -> BoxMesh:
    """Structured mesh of the unit square/cube with n^dim Q_order elements.

    fixed: every component of every boundary node (slide=False), or, for
    motion along the axis-parallel boundary (slide=True), only the
    component normal to each boundary face the node lies on (edge and corner
    nodes of several faces keep several components)."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    p = order
    m = n * p + 1
    xi = gll_points_unit(p)
    # 1D node coordinates along one direction of the box
    line = np.empty(m)
    for e in range(n):
        line[e * p:(e + 1) * p + 1] = (e + xi) / n
    line[-1] = 1.0
    # element -> node map
    loc = np.arange(p + 1)
    eidx = np.arange(n)
    if dim == 2:
        j0 = eidx[None, :, None, None] * p + loc[None, None, None, :]   # (1, n_e0, 1, i0)
        j1 = eidx[:, None, None, None] * p + loc[None, None, :, None]   # (n_e1, 1, i1, 1)
        nodes = j0 + m * j1                                             # (e1, e0, i1, i0)
        elem_node = nodes.reshape(n * n, (p + 1) ** 2)
        g0, g1 = np.meshgrid(line, line, indexing="xy")
        x_grid = np.stack([g0.ravel(), g1.ravel()])
        J = np.arange(m)
        on_bnd_1d = (J == 0) | (J == m - 1)
        # on_face[c]: nodes on a face with normal c (grid index j_c at an end)
        on_face = [np.broadcast_to(on_bnd_1d[None, :], (m, m)).ravel(),
                   np.broadcast_to(on_bnd_1d[:, None], (m, m)).ravel()]
    else:
        e = eidx
        j0 = e[None, None, :, None, None, None] * p + loc[None, None, None, None, None, :]
        j1 = e[None, :, None, None, None, None] * p + loc[None, None, None, None, :, None]
        j2 = e[:, None, None, None, None, None] * p + loc[None, None, None, :, None, None]
        nodes = j0 + m * (j1 + m * j2)                                  # (e2,e1,e0,i2,i1,i0)
        elem_node = nodes.reshape(n ** 3, (p + 1) ** 3)
        g2, g1, g0 = np.meshgrid(line, line, line, indexing="ij")
        x_grid = np.stack([g0.ravel(), g1.ravel(), g2.ravel()])
        J = np.arange(m)
        b = (J == 0) | (J == m - 1)
        on_face = [np.broadcast_to(b[None, None, :], (m, m, m)).ravel(),
                   np.broadcast_to(b[None, :, None], (m, m, m)).ravel(),
                   np.broadcast_to(b[:, None, None], (m, m, m)).ravel()]
    if slide:
        fixed = np.stack([f.astype(np.uint8) for f in on_face])
    else:
        bnd = np.logical_or.reduce(on_face)
        fixed = np.repeat(bnd[None, :].astype(np.uint8), dim, axis=0)
    return BoxMesh(dim=dim, order=p, n=n,
                   elem_node=np.ascontiguousarray(elem_node, dtype=np.int32),
                   x_grid=np.ascontiguousarray(x_grid, dtype=np.float64),
                   fixed=np.ascontiguousarray(fixed))


def sinusoid(mesh: BoxMesh, amplitude, kx: int = 1, ky: int = 1, kz: int = 1) -> np.ndarray:
    """Displacement amplitude_c * prod_k sin(2 pi k_k x_k) at the grid nodes,
    on interior nodes only (it vanishes on the boundary of the box anyway).
    `amplitude` is a scalar (same for every component) or one value per
    component."""
    xg = mesh.x_grid
    s = np.sin(2 * np.pi * kx * xg[0]) * np.sin(2 * np.pi * ky * xg[1])
    if mesh.dim == 3:
        s = s * np.sin(2 * np.pi * kz * xg[2])
    amp = np.broadcast_to(np.asarray(amplitude, dtype=np.float64), (mesh.dim,))
    u = amp[:, None] * s[None, :]
    u[mesh.fixed.astype(bool)] = 0.0
    return u


def perturb(mesh: BoxMesh, noise: float, seed: int, base: Optional[np.ndarray] = None,
            bad_elements: Optional[Callable[..., np.ndarray]] = None,
            max_rounds: int = 200) -> np.ndarray:
    """Add i.i.d. uniform noise U(-noise*h, noise*h) to every free node and
    component, drawn in ascending node order from numpy's PCG64 stream
    `default_rng(seed)`.  `base` defaults to the grid positions.

    If `bad_elements(x, elems)` is given, it returns the ids of the
    unacceptable elements among `elems` (None = all).  Their free nodes are
    redrawn from the same stream, and only the elements touching redrawn
    nodes are checked again, until none is reported (at most `max_rounds`
    rounds; then ValueError).  Rounds and redrawn nodes go to mesh.info."""
    rng = np.random.default_rng(seed)
    a = noise * mesh.h
    x = (mesh.x_grid if base is None else base).copy()
    free_node = ~mesh.fixed.astype(bool).any(axis=0)
    free_ids = np.flatnonzero(free_node)
    if a > 0:
        x[:, free_ids] += rng.uniform(-a, a, (free_ids.size, mesh.dim)).T
    rounds, redrawn = 0, 0
    if bad_elements is not None:
        base_x = (mesh.x_grid if base is None else base)
        bad = np.asarray(bad_elements(x, None), dtype=np.int64)
        node_elems = None
        while bad.size:
            if rounds >= max_rounds or a == 0:
                raise ValueError(f"mesh repair failed: {bad.size} bad elements after {rounds} rounds")
            nodes = np.unique(mesh.elem_node[bad].ravel())
            nodes = nodes[free_node[nodes]]
            x[:, nodes] = base_x[:, nodes] + rng.uniform(-a, a, (nodes.size, mesh.dim)).T
            rounds += 1
            redrawn += int(nodes.size)
            if node_elems is None:
                node_elems = _node_to_elements(mesh)
            touched = np.unique(np.concatenate([node_elems[n] for n in nodes]))
            bad = touched[np.asarray(bad_elements(x, touched), dtype=np.int64)] if touched.size else touched
    mesh.info.update(repair_rounds=rounds, redrawn_nodes=redrawn, seed=seed, noise=noise)
    return x


def _node_to_elements(mesh: BoxMesh):
    en = mesh.elem_node
    order = np.argsort(en.ravel(), kind="stable")
    elems = order // en.shape[1]
    counts = np.bincount(en.ravel(), minlength=mesh.n_node)
    return np.split(elems, np.cumsum(counts)[:-1])


def random_direction(mesh: BoxMesh, seed: int) -> np.ndarray:
    """Direction v ~ U(-1,1) per DOF (unmasked), shape (d, n_node)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, (mesh.dim, mesh.n_node)))


# ---------------------------------------------------------------------------
# The synthetic workloads.  Each stands in for one of the paper's quad/hex
# test meshes (Section 5), which are not available.

# tau_min: an element is accepted when det(A)/det(W) > tau_min at all its
# quadrature points (0 = plain positivity).  The Q3 square workload needs a
# margin: its noise inverts about one element in six, and redrawing only
# until det > 0 leaves nearly degenerate elements (det T ~ 4e-5, condition
# ~2e4); with det T > 0.02 the worst condition is ~90, as on the 8x8 mesh.
WORKLOADS = {
    # name: (dim, n, p, Q, metric, noise (x h), sinusoid amplitude, seed, tau_min)
    "q2_square_8":    dict(dim=2, n=8,   p=2, Q=4, metric=2,   noise=0.15, amp=0.0,  seed=0,     tau_min=0.0),
    "q3_square_256":  dict(dim=2, n=256, p=3, Q=5, metric=7,   noise=0.10, amp=0.05, seed=1,     tau_min=0.02),
    "q2_cube_64":     dict(dim=3, n=64,  p=2, Q=4, metric=303, noise=0.10, amp=0.0,  seed=2,     tau_min=0.0),
    "q3_cube_48":     dict(dim=3, n=48,  p=3, Q=5, metric=302, noise=0.05, amp=0.03, seed=3,     tau_min=0.0),
    "q2_square_512":  dict(dim=2, n=512, p=2, Q=4, metric=2,   noise=0.10, amp=0.0,  seed=10000, tau_min=0.0),
    # one GPU's share of q2_cube_64 split over 8 GPUs (a 2 x 2 x 2 block decomposition), at its real shape
    "q2_cube_32":     dict(dim=3, n=32,  p=2, Q=4, metric=303, noise=0.10, amp=0.0,  seed=20,    tau_min=0.0),
}


def make_workload(name: str, n: Optional[int] = None,
                  bad_elements: Optional[Callable[..., np.ndarray]] = None) -> BoxMesh:
    """Build a named workload (optionally shrunk to n elements per direction).
    `bad_elements(x, elems)` must apply the workload's acceptance floor
    WORKLOADS[name]["tau_min"]."""
    cfg = dict(WORKLOADS[name])
    if n is not None:
        cfg["n"] = n
    mesh = box_mesh(cfg["dim"], cfg["n"], cfg["p"])
    base = None
    if cfg["amp"]:
        base = mesh.x_grid + sinusoid(mesh, cfg["amp"])
    mesh.x = perturb(mesh, cfg["noise"], cfg["seed"], base=base, bad_elements=bad_elements)
    mesh.info.update(workload=name, Q=cfg["Q"], metric=cfg["metric"])
    return mesh


def training_mesh(n: int, seed: int, noise: float = 0.1,
                  bad_elements: Optional[Callable[..., np.ndarray]] = None,
                  max_tries: int = 50) -> BoxMesh:
    """2D Q2 mesh with a random smooth displacement plus noise, for the
    learned initial guess: per component c, a_c ~ U(0, 0.05) with a random
    sign, wave numbers kx, ky in {1..4}, displacement
    a_c sin(2 pi kx x) sin(2 pi ky y), then U(-noise h, noise h) noise.
    Redrawn whole (same stream) while `bad_elements` reports inversions."""
    mesh = box_mesh(2, n, 2)
    rng = np.random.default_rng(seed)
    for attempt in range(max_tries):
        kx, ky = (int(k) for k in rng.integers(1, 5, size=2))
        amp = rng.uniform(0.0, 0.05, size=2) * rng.choice([-1.0, 1.0], size=2)
        base = mesh.x_grid + sinusoid(mesh, amp, kx, ky)
        x = perturb(mesh, noise, int(rng.integers(0, 2**62)), base=base)
        if bad_elements is None or np.asarray(bad_elements(x, None)).size == 0:
            mesh.x = x
            mesh.info.update(kx=kx, ky=ky, amp=amp.tolist(), attempts=attempt + 1, seed=seed)
            return mesh
    raise ValueError("could not draw a valid training mesh")
