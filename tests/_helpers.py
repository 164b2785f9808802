"""Shared set-up for the GPU tests: seeded meshes (repaired with the
oracle's element check), the oracle problem and the library context."""
from __future__ import annotations

import sys
from dataclasses import dataclass

import numpy as np

from oracle import tmop_oracle as O
from paper_1807_09807_amd import meshgen


@dataclass
class Case:
    name: str
    dim: int
    n: int
    p: int
    Q: int
    metric: int
    noise: float
    amp: float = 0.0
    seed: int = 0
    rule: str = "gl"
    W0: tuple | None = None     # target = h * W0 (default identity)
    tau_min: float = 0.0        # repair floor on det T (see meshgen.WORKLOADS)

    def __str__(self):
        return self.name


def small_cases():
    """Shrunken versions of the five workloads plus variants that reach the
    other kernel shapes, rules and targets, with ragged element counts."""
    C = Case
    return [
        C("q2_square_8", 2, 8, 2, 4, 2, 0.15, seed=0),                     # full size
        C("q3_square_256@8", 2, 8, 3, 5, 7, 0.10, 0.05, seed=1, tau_min=0.02),
        C("q2_cube_64@4", 3, 4, 2, 4, 303, 0.10, seed=2),
        C("q3_cube_48@3", 3, 3, 3, 5, 302, 0.05, 0.03, seed=3),
        C("q2_square_512@16", 2, 16, 2, 4, 2, 0.10, seed=10000),
        C("p1_q2_2d_mu7", 2, 7, 1, 2, 7, 0.15, seed=11),
        C("p1_q3_3d_mu303", 3, 5, 1, 3, 303, 0.10, seed=12),
        C("p3_q4_2d_mu2", 2, 5, 3, 4, 2, 0.05, seed=13),
        C("p3_q4_3d_mu303", 3, 3, 3, 4, 303, 0.05, seed=14),
        C("p2_q3_3d_mu302", 3, 3, 2, 3, 302, 0.08, seed=15),
        C("p4_q6_2d_mu2", 2, 3, 4, 6, 2, 0.03, seed=16),
        C("p4_q5_3d_mu302", 3, 2, 4, 5, 302, 0.03, seed=17),
        C("lobatto_2d_mu7", 2, 5, 2, 4, 7, 0.10, seed=18, rule="gll"),
        C("lobatto_3d_mu303", 3, 3, 2, 4, 303, 0.10, seed=19, rule="gll"),
        C("aniso_W_2d_mu2", 2, 6, 2, 4, 2, 0.10, seed=20, W0=((1.0, 0.4), (0.1, 1.3))),
        C("aniso_W_3d_mu302", 3, 3, 2, 4, 302, 0.05, seed=21, W0=((1.0, 0.2, 0.0), (0.0, 1.1, 0.3), (0.1, 0.0, 0.9))),
        # the other 2D metrics of Table 3.1 and Sections 3.2 / 4.3
        C("p2_q4_2d_mu1", 2, 6, 2, 4, 1, 0.10, seed=30),
        C("p3_q5_2d_mu9", 2, 5, 3, 5, 9, 0.08, seed=31, W0=((1.0, 0.3), (-0.2, 1.1))),
        C("p2_q3_2d_mu14", 2, 7, 2, 3, 14, 0.10, seed=32),
        C("p1_q2_2d_mu77", 2, 9, 1, 2, 77, 0.15, seed=33),
        C("p4_q5_2d_mu98_lobatto", 2, 3, 4, 5, 98, 0.03, seed=34, rule="gll"),
        # mu_7 in 3D (Section 3.2 states it for any dimension), general target
        C("p2_q4_3d_mu7", 3, 3, 2, 4, 7, 0.08, seed=35, W0=((1.0, 0.1, 0.0), (0.0, 0.9, 0.2), (0.1, 0.0, 1.1))),
    ]


def build(case: Case):
    mesh = meshgen.box_mesh(case.dim, case.n, case.p)
    W = mesh.h * (np.eye(case.dim) if case.W0 is None else np.asarray(case.W0))
    prob = O.Problem(case.dim, case.p, case.Q, mesh.elem_node, case.metric, W, rule=case.rule)
    base = mesh.x_grid + meshgen.sinusoid(mesh, case.amp) if case.amp else None
    bad = lambda x, elems: prob.bad_elements(x, elems, case.tau_min)
    mesh.x = meshgen.perturb(mesh, case.noise, case.seed, base=base, bad_elements=bad)
    return mesh, prob, W


def context(case: Case, mesh, W, precision=0, fixed=True):
    from paper_1807_09807_amd import tmop as T
    rule = T.TMOP_GAUSS_LEGENDRE if case.rule == "gl" else T.TMOP_GAUSS_LOBATTO
    return T.Context(case.dim, case.p, mesh.elem_node, mesh.n_node, case.Q, case.metric, W,
                     fixed=mesh.fixed if fixed else None, precision=precision, rule=rule)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def rel_max_err(got, ref):
    """max_i |got_i - ref_i| / max_i |ref_i|: element-by-element comparison
    scaled by the vector's magnitude (entries of g and Hv pass through zero)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def mixed_tol(prob, x, v=None, diag=False):
    """Bars of the mixed FP32 path, one per result: the first-order
    worst-case rounding bounds of oracle/fp32_bound.py (F and min det A
    relative to their values; g, Hv and the diagonal as max DOF error over
    the largest exact entry).  Derived from the arithmetic, not fitted; the
    CPU tests hold an FP32 emulation to them."""
    from oracle import fp32_bound
    return fp32_bound.bounds(prob, x, v, diag=diag)


TARGET_FP32 = 1e-5   # the stated accuracy target of the FP32 path (F, |dF/dx|, Hessian action)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
