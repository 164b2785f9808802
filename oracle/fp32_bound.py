"""Test infrastructure, not product code: a first-order worst-case bound on
the rounding error of the mixed-precision form of the element operations,
against which the tests judge the library's TMOP_MIXED_FP32 results.

In that form the Jacobian contraction and the metric derivatives run in FP32
with FP32 accumulation; det A, the metric value and the sums of F and of the
scatter stay FP64 (the precision split the benchmark configuration states;
the paper fixes no precision).  The FP32 contraction works on each element's
nodal deviations X_i = x_i - a(xi_i) from its vertex-affine map a (the map
through the element's first node and the d corners next to it, evaluated in
FP64, so that the summands stay at the size of the deviation).

The bound follows the standard model of floating-point arithmetic,
fl(a op b) = (a op b)(1 + e), |e| <= u = 2^-24, to first order in u:

  A      Each entry of A is a sum over the element's nodes of table entries
         times deviations, formed by d sum-factorized passes of P terms and
         then added to the affine part.  Every table entry, every X_i and
         each of the d P accumulation steps rounds once (Higham, Accuracy
         and Stability of Numerical Algorithms, 2nd ed., Sec. 3.1):
           |dA|_F <= u (2 |A|_F + (d P + 2) S_A),
           S_A = | sum_i |X_i| |grad w_i|^t |_F     (entrywise absolute values),
         the 2 |A|_F covering the rounding of the affine part and of the
         final sum.  T = A W^-1 adds d roundings of its own:
           |dT|_F <= |W^-1|_2 (|dA|_F + d u |A|_F).
  P, dP  The exact change of the derivative under that perturbation is
         mu''(T)[dT] (first order), so |.|_F <= |mu''(T)|_2 |dT|_F with the
         spectral norm of the d^2 x d^2 matrix of mu''; for the Hessian
         action also |mu'''(T)[., E]|_2 |dT|_F for the direction E = dA W^-1
         and |mu''(T)|_2 |dE|_F for the perturbation of E.  Evaluating the
         chain-rule formulas in FP32 adds at most gamma_e u S, S the sum of
         the Frobenius norms of the formula's terms, gamma_e the rounding
         depth of the formula: 10 for P (coefficients of 1/tau powers,
         products and the sum of up to four terms), 20 for dP (also the
         contractions a_1, a_2, a_tau of up to 9 products).
  Y      Y = w det W (P or dP) W^-t: d + 1 roundings, folded into gamma_e.
  out    The transposed contraction sums d Q terms per pass over d passes
         and d components: gamma_t = d (Q + 3) roundings (with the d of
         Y = P W^-t) on sum_q |P|_F |W^-1|_2 |grad w_i|.
  F      The metric value is FP64 from the perturbed T: |dF| <= sum_q
         w_q det W |P(T)|_F |dT|_F.
  det A  FP64 from the perturbed A: |d det A| <= |cof A|_F |dA|_F per point,
         so the smallest det A moves by at most the largest of these.

The bound on each nodal entry is the sum of these contributions over the
quadrature points of the elements that hold the node; the reported figure
is its maximum over the DOFs divided by max |exact result|, the quantity
the tests compare.  No constant here was fitted to measured errors; the
CPU tests check the bound against an FP32 emulation of the same data flow.
"""
from __future__ import annotations

import numpy as np

from oracle import tmop_oracle as O

U32 = 2.0 ** -24


def _vertex_affine_deviation(prob, x, e0, e1):
    """X_i = x_i - a(xi_i) for the elements [e0, e1): shape (d, ne, npe)."""
    d, p = prob.dim, prob.order
    P = p + 1
    xi = O.gll_nodes(p)
    X = x[:, prob.elem_node[e0:e1]]
    org = X[:, :, 0]
    corner = [P - 1, P * (P - 1), P * P * (P - 1)][:d]
    J0 = np.stack([X[:, :, c] - org for c in corner], axis=-1)          # (d, ne, d)
    loc = np.arange(P ** d)
    ref = np.stack([xi[(loc // P ** k) % P] for k in range(d)], axis=-1)   # (npe, d)
    return X - org[:, :, None] - np.einsum("cel,il->cei", J0, ref)


def _unit_dirs(d):
    E = np.zeros((d * d, d, d))
    for k in range(d * d):
        E[k, k // d, k % d] = 1.0
    return E


def _second_matrix(metric, T):
    """The d^2 x d^2 matrix of mu''(T): column k = vec(mu''(T)[E_k])."""
    d = T.shape[-1]
    cols = [O.d2mu(metric, T, np.broadcast_to(E, T.shape)).reshape(T.shape[:-2] + (d * d,))
            for E in _unit_dirs(d)]
    return np.stack(cols, axis=-1)


def _third_matrix(metric, T, Edir, h=1e-30):
    """The d^2 x d^2 matrix of dT -> mu'''(T)[dT, Edir] by complex-step
    differentiation of mu''(T)[Edir] (the oracle's formulas are written for
    complex arguments)."""
    d = T.shape[-1]
    cols = []
    for E in _unit_dirs(d):
        Tc = T + 1j * h * np.broadcast_to(E, T.shape)
        cols.append((np.imag(O.d2mu(metric, Tc, Edir.astype(complex))) / h).reshape(T.shape[:-2] + (d * d,)))
    return np.stack(cols, axis=-1)


def _spec(M):
    return np.linalg.norm(M, ord=2, axis=(-2, -1))


def _fro(M):
    return np.sqrt(np.sum(M * M, axis=(-2, -1)))


def _terms_first(metric, T):
    """Sum of the Frobenius norms of the terms of P's chain-rule formula."""
    I1, I2, tau, C, J = O._inv(T)
    f = O._all_partials(metric, I1, I2, tau, J, T.shape[-1])
    dI2 = 2.0 * (I1[..., None, None] * T - O._mm(O._mm(T, O._tr(T)), T))
    d = T.shape[-1]
    return (np.abs(2.0 * f["f1"]) * _fro(T) + np.abs(f["f2"]) * _fro(dI2) + np.abs(f["ft"]) * _fro(C)
            + np.abs(f["fJ"]) * np.sqrt(d))


def _terms_second(metric, T, E):
    """Sum of the Frobenius norms of the terms of dP's chain-rule formula."""
    I1, I2, tau, C, J = O._inv(T)
    f = O._all_partials(metric, I1, I2, tau, J, T.shape[-1])
    d = T.shape[-1]
    TtT = O._mm(O._tr(T), T)
    dI2 = 2.0 * (I1[..., None, None] * T - O._mm(T, TtT))
    TE = O._ddot(T, E)
    ddI2 = (np.abs(4.0 * TE) * _fro(T) + 2.0 * np.abs(I1) * _fro(E) + 2.0 * _fro(O._mm(E, TtT))
            + 2.0 * _fro(O._mm(O._mm(T, O._tr(E)), T)) + 2.0 * _fro(O._mm(O._mm(T, O._tr(T)), E)))
    a1, a2, at = np.abs(2.0 * TE), np.abs(O._ddot(dI2, E)), np.abs(O._ddot(C, E))
    aJ = np.abs(np.trace(E, axis1=-2, axis2=-1))
    A = {k: np.abs(v) for k, v in f.items()}
    return (2.0 * A["f1"] * _fro(E) + A["f2"] * ddI2 + A["ft"] * _fro(O.dcof(T, E))
            + 2.0 * _fro(T) * (A["f11"] * a1 + A["f12"] * a2 + A["f1t"] * at)
            + _fro(dI2) * (A["f12"] * a1 + A["f22"] * a2 + A["f2t"] * at)
            + _fro(C) * (A["f1t"] * a1 + A["f2t"] * a2 + A["ftt"] * at + A["fJt"] * aJ)
            + np.sqrt(d) * A["fJt"] * at)


def _contraction_error(prob, f, e0, e1):
    """(A, bound on |dA|_F) of the FP32 contraction of field f, per point."""
    d, P = prob.dim, prob.order + 1
    Xd = _vertex_affine_deviation(prob, f, e0, e1)
    A = prob._jac(f, e0, e1)
    S = np.moveaxis(np.tensordot(np.abs(Xd), np.abs(prob.D), axes=([2], [1])), 0, 2)   # (ne, nq, c, l)
    return A, U32 * (2.0 * _fro(A) + (d * P + 2) * _fro(S))


def dof_bounds(prob, x, v=None, elems=None, grad=True, diag=False):
    """Per-DOF first-order bounds (arrays shaped like x) of the errors of the
    mixed-precision gradient (grad), Hessian action (v given) and Hessian
    diagonal (diag), and the absolute bounds of F and of the smallest
    det A.  With elems, only those elements' terms: exact at the nodes whose
    elements are all among them.

    The diagonal entry of DOF (c, i) is E : mu''(T)[E] with the rank-one
    E = e_c (W^-t grad w_i)^t; its first-order error is bounded through
    |mu'''(T)[dT, E]| <= sum_l |E_cl| |mu'''(T)[., E_cl]|_2 |dT|_F and the
    evaluation term gamma_e u |E| sum_l |E_cl| S(E_cl) (the terms of the
    second-derivative formula are linear in E, so their norms are
    subadditive)."""
    p = prob if elems is None else prob.subset(elems)
    d, Q = p.dim, p.Q
    n_node = x.shape[1]
    bg = np.zeros((d, n_node)) if grad else None
    bh = np.zeros((d, n_node)) if v is not None else None
    bd = np.zeros((d, n_node)) if diag else None
    dF, ddet = 0.0, 0.0
    gam_t = d * (Q + 3)
    ng_ref = np.sqrt(np.sum(p.D * p.D, axis=-1))                               # |grad w_i(q)|, (nq, npe)
    units = _unit_dirs(d)
    for e0, e1 in p._chunks():
        A, eA = _contraction_error(p, x, e0, e1)
        if v is not None:
            dA, edA = _contraction_error(p, v, e0, e1)
        ddet = max(ddet, float(np.max(_fro(O.cof(A)) * eA)))
        for metric, Wi, wt in p._terms(e0, e1):
            nW = np.broadcast_to(_spec(np.asarray(Wi)), A.shape[:2])   # on the stored targets, then broadcast
            Wi = np.broadcast_to(Wi, A.shape)
            wt = np.abs(np.broadcast_to(wt, A.shape[:2]))
            T = O._mm(A, Wi)
            eT = nW * (eA + d * U32 * _fro(A))
            Pm = O.dmu(metric, T)
            dF += float(np.sum(wt * _fro(Pm) * eT))
            if not (grad or v is not None or diag):
                continue
            M2 = _spec(_second_matrix(metric, T))
            gW = np.einsum("qil,eqml->eqim", p.D, Wi)                           # W^-t grad w_i, (ne, nq, npe, d)
            ngW = np.sqrt(np.sum(gW * gW, axis=-1))                            # (ne, nq, npe)
            en = p.elem_node[e0:e1]
            if grad:   # perturbation of T, formula evaluation, transposed contraction
                eY = wt * (M2 * eT + 10 * U32 * _terms_first(metric, T))
                sY = wt * _fro(Pm) * nW
                share = np.einsum("eq,eqi->ei", eY, ngW) + gam_t * U32 * np.einsum("eq,qi->ei", sY, ng_ref)
                for c in range(d):
                    np.add.at(bg[c], en, share)
            if v is not None:
                E = O._mm(dA, Wi)
                eE = nW * (edA + d * U32 * _fro(dA))
                M3 = _spec(_third_matrix(metric, T, E))
                dP = O.d2mu(metric, T, E)
                eY = wt * (M3 * eT + M2 * eE + 20 * U32 * _terms_second(metric, T, E))
                sY = wt * _fro(dP) * nW
                share = np.einsum("eq,eqi->ei", eY, ngW) + gam_t * U32 * np.einsum("eq,qi->ei", sY, ng_ref)
                for c in range(d):
                    np.add.at(bh[c], en, share)
            if diag:
                N3 = np.stack([_spec(_third_matrix(metric, T, np.broadcast_to(Ek, T.shape))) for Ek in units], -1)
                S2 = np.stack([_terms_second(metric, T, np.broadcast_to(Ek, T.shape)) for Ek in units], -1)
                N3 = N3.reshape(N3.shape[:2] + (d, d))          # [e][q][c][l]
                S2 = S2.reshape(S2.shape[:2] + (d, d))
                agW = np.abs(gW)                                # [e][q][i][l]
                pert = np.einsum("eqil,eqcl->eqic", agW, N3) * eT[..., None, None]
                ev = 20 * U32 * np.einsum("eqil,eqcl->eqic", agW, S2)
                rnd = gam_t * U32 * (M2 * nW * nW)[..., None] * (ng_ref * ng_ref)[None]   # [e][q][i]
                share = np.einsum("eq,eqic->eic", wt, (pert + ev) * ngW[..., None]) + \
                    np.einsum("eq,eqi->ei", wt, rnd)[..., None]
                for c in range(d):
                    np.add.at(bd[c], en, share[..., c])
    return dict(F=dF, min_detA=ddet, g=bg, Hv=bh, diag=bd)


def bounds(prob, x, v=None, diag=False):
    """The bounds as the tests compare them: F and min det A relative to
    their exact values, g, Hv and the diagonal as max DOF error over max
    |exact entry|."""
    b = dof_bounds(prob, x, v, diag=diag)
    F, md = prob.energy(x)
    out = dict(F=b["F"] / abs(F), min_detA=b["min_detA"] / abs(md),
               g=float(np.max(b["g"]) / np.max(np.abs(prob.gradient(x)))))
    if v is not None:
        out["Hv"] = float(np.max(b["Hv"]) / np.max(np.abs(prob.hessian_apply(x, v))))
    if diag:
        out["diag"] = float(np.max(b["diag"]) / np.max(np.abs(prob.hessian_diagonal(x))))
    return out
