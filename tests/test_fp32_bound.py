"""Pins of the mixed-precision error bound (oracle/fp32_bound.py) on the CPU:
an FP32 emulation of the mixed path's data flow -- element deviations from
the vertex-affine map rounded to FP32, FP32 1D tables, d sum-factorized FP32
passes, the oracle's metric derivatives evaluated in FP32, the transposed
FP32 passes and an FP64 scatter -- must stay within the bound on every
small test mesh (2D and 3D, each metric family, general targets).  The
emulation is a different program from the library's kernels (other summation
orders, no fused multiply-adds), so it checks the bound's model of the
roundings rather than the kernels; the GPU tests then hold the kernels to the
same bound."""
import numpy as np
import pytest

from oracle import fp32_bound as B
from oracle import tmop_oracle as O
from tests._helpers import build, small_cases

f32 = np.float32


def _tables(p, Q, rule):
    s, _ = O.gauss_legendre(Q) if rule == "gl" else O.gauss_lobatto(Q)
    L, G = O.lagrange(O.gll_nodes(p), s)
    return L.astype(f32), G.astype(f32)


def _fwd32(prob, f, Bt, Gt):
    """A in FP32 at every point, shape (ne, nq, d, d), point index q0 fastest."""
    d, P = prob.dim, prob.order + 1
    Xd = B._vertex_affine_deviation(prob, f, 0, prob.n_elem)                 # (d, ne, npe)
    X = Xd.astype(f32).reshape((d, prob.n_elem) + (P,) * d)                  # [c][e][(i2)][i1][i0]
    X0 = f[:, prob.elem_node[:, 0]]
    corner = [P - 1, P * (P - 1), P * P * (P - 1)][:d]
    J0 = np.stack([f[:, prob.elem_node[:, c]] - X0 for c in corner], axis=-1).astype(f32)   # (d, ne, l)
    if d == 2:
        ub = np.einsum("qj,ceji->ceqi", Bt, X)          # [c][e][q1][i0]
        ug = np.einsum("qj,ceji->ceqi", Gt, X)
        a0 = np.einsum("pi,ceqi->ceqp", Gt, ub)         # [c][e][q1][q0]
        a1 = np.einsum("pi,ceqi->ceqp", Bt, ug)
        comps = [a0, a1]
    else:
        vb = np.einsum("rk,cekji->cerji", Bt, X)        # [c][e][q2][i1][i0]
        vg = np.einsum("rk,cekji->cerji", Gt, X)
        bb = np.einsum("qj,cerji->cerqi", Bt, vb)       # [c][e][q2][q1][i0]
        gb = np.einsum("qj,cerji->cerqi", Gt, vb)
        bg = np.einsum("qj,cerji->cerqi", Bt, vg)
        comps = [np.einsum("pi,cerqi->cerqp", Gt, bb), np.einsum("pi,cerqi->cerqp", Bt, gb),
                 np.einsum("pi,cerqi->cerqp", Bt, bg)]
    A = np.stack([c.reshape(d, prob.n_elem, -1) for c in comps], axis=-1)   # (d, ne, nq, l)
    A = (A + J0[:, :, None, :]).astype(f32)
    return np.moveaxis(A, 0, 2)                         # (ne, nq, c, l)


def _bwd32(prob, Y, Bt, Gt):
    """out[c, e, i] = sum_q sum_l Y[e, q, c, l] d_l w_i(q) by transposed FP32 passes."""
    d, P, Q = prob.dim, prob.order + 1, prob.Q
    Yc = np.moveaxis(Y, (2, 3), (0, 1)).astype(f32)    # [c][l][e][q]
    if d == 2:
        y = Yc.reshape(d, d, prob.n_elem, Q, Q)         # [c][l][e][q1][q0]
        r0 = np.einsum("pi,ceqp->ceqi", Gt, y[:, 0])
        r1 = np.einsum("pi,ceqp->ceqi", Bt, y[:, 1])
        out = np.einsum("qj,ceqi->ceji", Bt, r0) + np.einsum("qj,ceqi->ceji", Gt, r1)
    else:
        y = Yc.reshape(d, d, prob.n_elem, Q, Q, Q)      # [c][l][e][q2][q1][q0]
        r0 = np.einsum("pi,cerqp->cerqi", Gt, y[:, 0])
        r1 = np.einsum("pi,cerqp->cerqi", Bt, y[:, 1])
        r2 = np.einsum("pi,cerqp->cerqi", Bt, y[:, 2])
        sb = np.einsum("qj,cerqi->cerji", Bt, r0) + np.einsum("qj,cerqi->cerji", Gt, r1)
        sg = np.einsum("qj,cerqi->cerji", Bt, r2)
        out = np.einsum("rk,cerji->cekji", Bt, sb) + np.einsum("rk,cerji->cekji", Gt, sg)
    return out.astype(f32).reshape(d, prob.n_elem, -1)


def emulate(prob, x, v, rule):
    """(F, min det A, g, Hv) of the FP32 data flow (single metric term)."""
    Bt, Gt = _tables(prob.order, prob.Q, rule)
    A = _fwd32(prob, x, Bt, Gt)
    dA = _fwd32(prob, v, Bt, Gt)
    (metric, Wi, wt), = prob._terms(0, prob.n_elem)
    Wi = np.broadcast_to(Wi, A.shape)
    wt = np.broadcast_to(wt, A.shape[:2])
    T64 = O._mm(A.astype(np.float64), Wi)
    F = float(np.sum(wt * O.mu(metric, T64)))
    mind = float(np.min(O._det(A.astype(np.float64))))
    Wi32 = Wi.astype(f32)
    T, E = O._mm(A, Wi32).astype(f32), O._mm(dA, Wi32).astype(f32)
    k = wt.astype(f32)[..., None, None]
    Y = (k * O._mm(O.dmu(metric, T).astype(f32), O._tr(Wi32))).astype(f32)
    dY = (k * O._mm(O.d2mu(metric, T, E).astype(f32), O._tr(Wi32))).astype(f32)
    g, Hv = np.zeros_like(x), np.zeros_like(x)
    for Yv, out in ((Y, g), (dY, Hv)):
        oe = _bwd32(prob, Yv, Bt, Gt)
        for c in range(prob.dim):
            np.add.at(out[c], prob.elem_node, oe[c].astype(np.float64))
    return F, mind, g, Hv


CASES = [c for c in small_cases() if c.name not in ("q3_cube_48@3", "p4_q5_3d_mu302")]


@pytest.mark.parametrize("case", CASES, ids=str)
def test_fp32_emulation_within_bound(case):
    mesh, prob, W = build(case)
    v = np.random.default_rng(3).uniform(-1.0, 1.0, mesh.x.shape)
    F, md = prob.energy(mesh.x)
    g, Hv = prob.gradient(mesh.x), prob.hessian_apply(mesh.x, v)
    Fe, mde, ge, He = emulate(prob, mesh.x, v, case.rule)
    err = dict(F=abs(Fe - F) / abs(F), min_detA=abs(mde - md) / abs(md),
               g=np.max(np.abs(ge - g)) / np.max(np.abs(g)), Hv=np.max(np.abs(He - Hv)) / np.max(np.abs(Hv)))
    b = B.bounds(prob, mesh.x, v)
    for k in err:
        print(f"{case.name} {k}: emulated {err[k]:.2e} bound {b[k]:.2e} ({err[k] / b[k]:.3f})")
        assert err[k] <= b[k], k


def test_bound_scales_with_conditioning():
    """A nearly degenerate mesh has a larger bound than a mild one (the
    derivatives' 1/tau powers amplify the rounding of T)."""
    mild = [c for c in CASES if c.name == "p3_q4_2d_mu2"][0]
    harsh = [c for c in CASES if c.name == "q2_square_8"][0]
    out = []
    for c in (mild, harsh):
        mesh, prob, W = build(c)
        out.append(B.bounds(prob, mesh.x)["g"])
    assert out[1] > 5 * out[0]
