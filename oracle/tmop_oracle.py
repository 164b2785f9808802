"""Plain FP64 CPU oracle for the TMOP hot path.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  The GPU library never calls it and shares
no code with it: it builds its own basis tables, its own metric derivatives
and its own solver.

Source: Dobrev, Knupp, Kolev, Mittal, Tomov, "The Target-Matrix Optimization
Paradigm for High-Order Meshes" (arXiv:1807.09807).  Every function below
names the passage it follows.  The oracle computes the plain definitions:

* the basis gradients at every quadrature point form a dense table and the
  Jacobian A = sum_i x_i (grad w_i)^T is a dense contraction (eq. 2.2) -- no
  sum factorization;
* mu is evaluated from its definition (Table 3.1 and Section 3.2) with
  numpy's det/inv; its first and second derivatives in T are the invariant
  forms the paper recommends (Section 3.4), pinned by complex-step tests;
* F_V (eq. 2.4) is summed with math.fsum (exactly rounded);
* the gradient (Section 3.4) and the Hessian action are assembled
  element by element and scattered with numpy.add.at;
* Newton's method with the positivity / 1.2-growth line search follows
  Section 3.4, with truncated CG (Steihaug) or MINRES (the inner solver of
  Section 5) on the masked Hessian, optionally Jacobi preconditioned;
* the Section 4 objectives: a second weighted metric term (eq. 4.1), the
  replication composite of Section 4.3.2 and the displacement penalty of
  eq. 4.2, whose field values x(q) come from a dense basis-value table.

Readings where the paper is silent: reference element [0,1]^d; nodal basis =
Lagrange polynomials at the Gauss-Lobatto-Legendre points; Gauss-Legendre
quadrature on [0,1]; x stored as (d, n_node).

Everything is written dtype-generic (no abs, no conj, no maximum on the
data path) so that a complex-step derivative can run through the whole
objective.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

METRICS_2D = (1, 2, 7, 9, 14, 77, 98)
METRICS_3D = (7, 302, 303)


# ---------------------------------------------------------------------------
# Section 2.1 / Section 3.3: 1D points, weights and Lagrange basis

def gll_nodes(p: int) -> np.ndarray:
    """GLL points on [0,1]: 0, 1 and the interior roots of P_p'.  The interior
    roots are the eigenvalues of the symmetric tridiagonal Jacobi matrix of
    the Jacobi(1,1) polynomials, whose off-diagonal entries are
    sqrt(k(k+2) / ((2k+1)(2k+3))), k = 1..p-2."""
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        t = np.array([-1.0, 1.0])
    else:
        k = np.arange(1, p - 1, dtype=np.float64)
        off = np.sqrt(k * (k + 2.0) / ((2.0 * k + 1.0) * (2.0 * k + 3.0)))
        J = np.diag(off, 1) + np.diag(off, -1)
        inner = np.sort(np.linalg.eigvalsh(J)) if p > 2 else np.array([0.0])
        t = np.concatenate(([-1.0], inner, [1.0]))
    return (t + 1.0) / 2.0


def gauss_legendre(Q: int):
    """Q-point Gauss-Legendre rule mapped to [0,1] (Section 3.3); weights
    sum to 1."""
    t, w = np.polynomial.legendre.leggauss(Q)
    return (t + 1.0) / 2.0, w / 2.0


def gauss_lobatto(Q: int):
    """Q-point Gauss-Lobatto rule on [0,1] (the rule of Section 5): the GLL
    points with weights 2/(Q(Q-1) P_{Q-1}(t)^2) on [-1,1], halved."""
    s = gll_nodes(Q - 1)
    t = 2.0 * s - 1.0
    PQ = np.polynomial.legendre.Legendre.basis(Q - 1)(t)
    w = 2.0 / (Q * (Q - 1) * PQ ** 2)
    return s, w / 2.0


def lagrange(nodes: np.ndarray, s: np.ndarray):
    """Values L[k, a] = l_a(s_k) and derivatives G[k, a] = l_a'(s_k) of the
    Lagrange polynomials through `nodes`, from the product formula."""
    n = nodes.size
    dt = np.result_type(s, np.float64)
    L = np.ones((s.size, n), dtype=dt)
    G = np.zeros((s.size, n), dtype=dt)
    for a in range(n):
        for b in range(n):
            if b != a:
                L[:, a] *= (s - nodes[b]) / (nodes[a] - nodes[b])
        for k in range(n):
            if k == a:
                continue
            term = np.full(s.size, 1.0 / (nodes[a] - nodes[k]), dtype=dt)
            for b in range(n):
                if b != a and b != k:
                    term *= (s - nodes[b]) / (nodes[a] - nodes[b])
            G[:, a] += term
    return L, G


def dense_tables(dim: int, p: int, Q: int, rule: str = "gl"):
    """Dense table D[q, i, l] = d w_i / d xbar_l at quadrature point q and
    the tensor weights wq[q] (eq. 2.2, Section 3.3).  Local node index
    i = i0 + (p+1) i1 (+ (p+1)^2 i2); quadrature index q = q0 + Q q1 (+ Q^2 q2)."""
    s, w1 = gauss_legendre(Q) if rule == "gl" else gauss_lobatto(Q)
    L, G = lagrange(gll_nodes(p), s)
    P1 = p + 1
    if dim == 2:
        D = np.zeros((Q, Q, P1, P1, 2))
        # axes: q1, q0, i1, i0
        D[..., 0] = G[None, :, None, :] * L[:, None, :, None]
        D[..., 1] = L[None, :, None, :] * G[:, None, :, None]
        wq = (w1[:, None] * w1[None, :]).ravel()
        return D.reshape(Q * Q, P1 * P1, 2), wq
    D = np.zeros((Q, Q, Q, P1, P1, P1, 3))
    # axes: q2, q1, q0, i2, i1, i0
    D[..., 0] = G[None, None, :, None, None, :] * L[None, :, None, None, :, None] * L[:, None, None, :, None, None]
    D[..., 1] = L[None, None, :, None, None, :] * G[None, :, None, None, :, None] * L[:, None, None, :, None, None]
    D[..., 2] = L[None, None, :, None, None, :] * L[None, :, None, None, :, None] * G[:, None, None, :, None, None]
    wq = (w1[:, None, None] * w1[None, :, None] * w1[None, None, :]).ravel()
    return D.reshape(Q ** 3, P1 ** 3, 3), wq


def basis_table(dim: int, p: int, Q: int, rule: str = "gl"):
    """Dense table Bv[q, i] = w_i(s_q): the nodal basis functions of eq. 2.1
    at the quadrature points, with the index orders of dense_tables."""
    s, _ = gauss_legendre(Q) if rule == "gl" else gauss_lobatto(Q)
    L, _ = lagrange(gll_nodes(p), s)
    P1 = p + 1
    if dim == 2:
        # axes: q1, q0, i1, i0
        return (L[None, :, None, :] * L[:, None, :, None]).reshape(Q * Q, P1 * P1)
    # axes: q2, q1, q0, i2, i1, i0
    Bv = (L[None, None, :, None, None, :] * L[None, :, None, None, :, None]
          * L[:, None, None, :, None, None])
    return Bv.reshape(Q ** 3, P1 ** 3)


# ---------------------------------------------------------------------------
# Section 3.2, Table 3.1: metrics by definition

def _det(T):
    return np.linalg.det(T)


def _frob2(M):
    return np.sum(M * M, axis=(-2, -1))


def _tau23(tau):
    """tau^(2/3) with the real cube root, so that the formula also has a
    value for tau <= 0 (outside the barrier domain, Section 3.2).  Complex
    arguments (complex-step derivatives, tau > 0) use the principal power."""
    if np.iscomplexobj(tau):
        return tau ** (2.0 / 3.0)
    c = np.cbrt(tau)
    return c * c


def mu(metric: int, T: np.ndarray) -> np.ndarray:
    """mu(T) for T of shape (..., d, d).
    1:   |T|^2                                (Table 3.1, no barrier, 2D)
    2:   |T|^2 / (2 tau) - 1                 (Table 3.1, shape, 2D)
    7:   |T - T^{-t}|^2                       (Section 3.2, shape+size, 2D and 3D)
    9:   tau |T - T^{-t}|^2                   (Table 3.1, shape+size, 2D)
    14:  |T - I|^2                            (Section 3.2, shape+size+alignment, 2D)
    77:  (tau - 1/tau)^2 / 2                  (Table 3.1, size, 2D)
    98:  |T - I|^2 / tau                     (Section 4.3, shape+size+alignment; a primary
         metric in 2D, and the replication metric in 2D and 3D)
    303: |T|^2 / (3 tau^{2/3}) - 1           (Table 3.1, shape, 3D)
    302: |T|^2 |T^{-1}|^2 / 9 - 1            (3D shape metric of the workloads)
    with tau = det T and |.| the Frobenius norm."""
    tau = _det(T)
    I1 = _frob2(T)
    if metric == 1:
        return I1
    if metric == 2:
        return I1 / (2.0 * tau) - 1.0
    if metric in (7, 9):
        Tinv_t = np.swapaxes(np.linalg.inv(T), -1, -2)
        return _frob2(T - Tinv_t) * (tau if metric == 9 else 1.0)
    if metric in (14, 98):
        d = T.shape[-1]
        return _frob2(T - np.eye(d)) / (tau if metric == 98 else 1.0)
    if metric == 77:
        return 0.5 * (tau - 1.0 / tau) ** 2
    if metric == 303:
        return I1 / (3.0 * _tau23(tau)) - 1.0
    if metric == 302:
        return I1 * _frob2(np.linalg.inv(T)) / 9.0 - 1.0
    raise ValueError(f"unknown metric {metric}")


# Invariant forms of the derivatives (Section 3.4: write mu through matrix
# invariants).  mu = f(I1, I2, tau, J), I1 = |T|^2, tau = det T, C = cof T =
# d tau / dT, I2 = |C|^2 (3D only), J = tr T (dJ/dT = I, for the metrics
# measured against T = I).

def cof(T):
    """Cofactor matrix C = d(det T)/dT."""
    d = T.shape[-1]
    if d == 2:
        C = np.empty_like(T)
        C[..., 0, 0] = T[..., 1, 1]
        C[..., 0, 1] = -T[..., 1, 0]
        C[..., 1, 0] = -T[..., 0, 1]
        C[..., 1, 1] = T[..., 0, 0]
        return C
    r0, r1, r2 = T[..., 0, :], T[..., 1, :], T[..., 2, :]
    return np.stack([_cross(r1, r2), _cross(r2, r0), _cross(r0, r1)], axis=-2)


def dcof(T, E):
    """Directional derivative of cof at T along E."""
    d = T.shape[-1]
    if d == 2:
        return cof(E)
    t0, t1, t2 = T[..., 0, :], T[..., 1, :], T[..., 2, :]
    e0, e1, e2 = E[..., 0, :], E[..., 1, :], E[..., 2, :]
    return np.stack([_cross(e1, t2) + _cross(t1, e2),
                     _cross(e2, t0) + _cross(t2, e0),
                     _cross(e0, t1) + _cross(t0, e1)], axis=-2)


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def _ddot(A, B):
    return np.sum(A * B, axis=(-2, -1))


def _mm(A, B):
    return np.einsum("...ij,...jk->...ik", A, B)


def _tr(A):
    return np.swapaxes(A, -1, -2)


def _partials(metric, I1, I2, tau, J=None, d=2):
    """The nonzero partials among (f1, f2, ft, fJ, f11, f12, f1t, f22, f2t,
    ftt, fJt) of mu = f(I1, I2, tau, J) for d x d matrices; the others are
    zero."""
    z = 0.0 * tau
    if metric == 1:          # f = I1
        return dict(f1=1.0 + z)
    if metric == 9:          # tau |T - T^-t|^2 = tau I1 + I1 / tau - 4 tau in 2D
        return dict(f1=tau + 1.0 / tau, ft=I1 - I1 / tau ** 2 - 4.0, f1t=1.0 - 1.0 / tau ** 2,
                    ftt=2.0 * I1 / tau ** 3)
    if metric == 77:         # (tau - 1/tau)^2 / 2
        return dict(ft=(tau - 1.0 / tau) * (1.0 + 1.0 / tau ** 2), ftt=1.0 + 3.0 / tau ** 4)
    if metric == 14:         # |T - I|^2 = I1 - 2 J + d
        return dict(f1=1.0 + z, fJ=-2.0 + z)
    if metric == 98:         # (I1 - 2 J + d) / tau
        n = I1 - 2.0 * J + d
        return dict(f1=1.0 / tau, fJ=-2.0 / tau, ft=-n / tau ** 2, f1t=-1.0 / tau ** 2,
                    fJt=2.0 / tau ** 2, ftt=2.0 * n / tau ** 3)
    if metric == 2:          # f = I1/(2 tau) - 1
        return dict(f1=1.0 / (2.0 * tau), f2=z, ft=-I1 / (2.0 * tau ** 2),
                    f11=z, f12=z, f1t=-1.0 / (2.0 * tau ** 2), f22=z, f2t=z, ftt=I1 / tau ** 3)
    if metric == 7 and d == 3:   # |T - T^-t|^2 = I1 + |T^-1|^2 - 6, |T^-1|^2 = |cof T|^2/tau^2 = I2/tau^2
        return dict(f1=1.0 + z, f2=tau ** -2, ft=-2.0 * I2 * tau ** -3,
                    f11=z, f12=z, f1t=z, f22=z, f2t=-2.0 * tau ** -3, ftt=6.0 * I2 * tau ** -4)
    if metric == 7:          # |T - T^-t|^2 = I1 + |T^-1|^2 - 4, |T^-1|^2 = I1/tau^2 in 2D
        return dict(f1=1.0 + tau ** -2, f2=z, ft=-2.0 * I1 * tau ** -3,
                    f11=z, f12=z, f1t=-2.0 * tau ** -3, f22=z, f2t=z, ftt=6.0 * I1 * tau ** -4)
    if metric == 303:        # f = I1 tau^{-2/3} / 3 - 1
        t23 = 1.0 / _tau23(tau)
        return dict(f1=t23 / 3.0, f2=z, ft=-(2.0 / 9.0) * I1 * t23 / tau,
                    f11=z, f12=z, f1t=-(2.0 / 9.0) * t23 / tau, f22=z, f2t=z,
                    ftt=(10.0 / 27.0) * I1 * t23 / tau ** 2)
    if metric == 302:        # |T^-1|^2 = I2/tau^2 in 3D: f = I1 I2 tau^-2 / 9 - 1
        return dict(f1=I2 * tau ** -2 / 9.0, f2=I1 * tau ** -2 / 9.0, ft=-2.0 * I1 * I2 * tau ** -3 / 9.0,
                    f11=z, f12=tau ** -2 / 9.0, f1t=-2.0 * I2 * tau ** -3 / 9.0,
                    f22=z, f2t=-2.0 * I1 * tau ** -3 / 9.0, ftt=6.0 * I1 * I2 * tau ** -4 / 9.0)
    raise ValueError(f"unknown metric {metric}")


def _inv(T):
    I1 = _frob2(T)
    tau = _det(T)
    C = cof(T)
    I2 = _frob2(C)
    J = np.trace(T, axis1=-2, axis2=-1)
    return I1, I2, tau, C, J


_PARTIAL_NAMES = ("f1", "f2", "ft", "fJ", "f11", "f12", "f1t", "f22", "f2t", "ftt", "fJt")


def _all_partials(metric, I1, I2, tau, J, d=2):
    f = _partials(metric, I1, I2, tau, J, d)
    z = 0.0 * tau
    return {k: f.get(k, z) for k in _PARTIAL_NAMES}


def dmu(metric: int, T: np.ndarray) -> np.ndarray:
    """First derivative P = d mu / dT (the matrix of Section 3.4)."""
    I1, I2, tau, C, J = _inv(T)
    f = _all_partials(metric, I1, I2, tau, J, T.shape[-1])
    e = lambda s: s[..., None, None]
    dI2 = 2.0 * (e(I1) * T - _mm(_mm(T, _tr(T)), T))
    Id = np.eye(T.shape[-1])
    return e(f["f1"]) * 2.0 * T + e(f["f2"]) * dI2 + e(f["ft"]) * C + e(f["fJ"]) * Id


def d2mu(metric: int, T: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Second derivative of mu applied to a direction: dP = d/de P(T + e E)
    at e = 0 (the Hessian ingredient of Section 3.4).  The partials f1J and
    fJJ vanish for every metric here."""
    I1, I2, tau, C, J = _inv(T)
    f = _all_partials(metric, I1, I2, tau, J, T.shape[-1])
    e = lambda s: s[..., None, None]
    TtT = _mm(_tr(T), T)
    dI2 = 2.0 * (e(I1) * T - _mm(T, TtT))
    ddI2 = 2.0 * (2.0 * e(_ddot(T, E)) * T + e(I1) * E
                  - _mm(E, TtT) - _mm(_mm(T, _tr(E)), T) - _mm(_mm(T, _tr(T)), E))
    a1 = 2.0 * _ddot(T, E)
    a2 = _ddot(dI2, E)
    at = _ddot(C, E)
    aJ = np.trace(E, axis1=-2, axis2=-1)
    Id = np.eye(T.shape[-1])
    return (e(f["f1"]) * 2.0 * E + e(f["f2"]) * ddI2 + e(f["ft"]) * dcof(T, E)
            + 2.0 * T * e(f["f11"] * a1 + f["f12"] * a2 + f["f1t"] * at)
            + dI2 * e(f["f12"] * a1 + f["f22"] * a2 + f["f2t"] * at)
            + C * e(f["f1t"] * a1 + f["f2t"] * a2 + f["ftt"] * at + f["fJt"] * aJ)
            + Id * e(f["fJt"] * at))


# ---------------------------------------------------------------------------
# Section 2.2-2.3, eq. 2.4: the variational objective and its derivatives

class Problem:
    """F_V(x) = sum_E sum_q w_q det W mu(A W^{-1}) on a Q_p quad/hex mesh.

    elem_node: (n_elem, (p+1)^d) int array, lexicographic local node order.
    W: None (identity), a (d, d) matrix, per-element (n_elem, d, d) or
       per-quadrature-point (n_elem, Q^d, d, d) targets; det W > 0
       (Section 3.1).

    Section 4 adds to F_V (each optional, see set_combo, set_replication and
    set_restriction):
      a weight eta_1 on the term above and a second term
      sum_E sum_q w_q omega_q mu_2(A W_2^{-1})  (eq. 4.1 with two metrics,
      or the replication composite of Section 4.3.2), and
      sum_E sum_q w_q det W delta |x(q) - x_init(q)|^2  (eq. 4.2).
    """

    def __init__(self, dim, order, n_q1d, elem_node, metric, W=None, rule="gl", chunk=4096):
        if dim == 2 and metric not in METRICS_2D or dim == 3 and metric not in METRICS_3D:
            raise ValueError("metric/dimension mismatch")
        self.dim, self.order, self.Q, self.metric = dim, order, n_q1d, metric
        self.elem_node = np.asarray(elem_node, dtype=np.int64)
        self.n_elem = self.elem_node.shape[0]
        self.D, self.wq = dense_tables(dim, order, n_q1d, rule)
        self.nq = self.wq.size
        W = np.eye(dim) if W is None else np.asarray(W, dtype=np.float64)
        detW = np.linalg.det(W)
        if np.any(detW <= 0):
            raise ValueError("target matrices need det W > 0 (Section 3.1)")
        self.Winv = np.linalg.inv(W)
        self.detW = detW
        self.chunk = chunk
        self.Bv = basis_table(dim, order, n_q1d, rule)
        self.eta1 = 1.0
        self.second = None       # dict(metric, Winv (n_elem, nq, d, d), omega (n_elem, nq))
        self.delta = 0.0
        self.x_init = None

    # ------------------------------------------------------------ Section 4
    def _primary_detW(self):
        """det W of the primary target at every point, shape (n_elem, nq)."""
        _, dW = self._targets(0, self.n_elem)
        return np.broadcast_to(dW, (self.n_elem, self.nq)).astype(np.float64)

    def set_combo(self, metric2, W2, eta1=1.0, eta2=None):
        """Composite metric of eq. 4.1 with two terms: eta_1 mu(T) with the
        primary target plus eta_2 mu_2(A W_2^{-1}), each integrated over its
        own target element (as in the combined objective of Section 5.2.4),
        so the second term's weight is omega_q = eta_2(q) det W_2.  W2: a
        (d, d) matrix or (n_elem, nq, d, d); eta2: None (1), a scalar or
        (n_elem, nq) per-point weights."""
        ok = METRICS_2D if self.dim == 2 else METRICS_3D
        if metric2 not in ok:
            raise ValueError("metric/dimension mismatch")
        W2 = np.asarray(W2, dtype=np.float64)
        W2 = np.broadcast_to(W2, (self.n_elem, self.nq, self.dim, self.dim))
        d2 = np.linalg.det(W2)
        if np.any(d2 <= 0):
            raise ValueError("target matrices need det W > 0 (Section 3.1)")
        eta2 = 1.0 if eta2 is None else np.asarray(eta2, dtype=np.float64)
        self.eta1 = float(eta1)
        self.second = dict(metric=metric2, Winv=np.linalg.inv(W2),
                           omega=np.broadcast_to(eta2, (self.n_elem, self.nq)) * d2)

    def set_replication(self, gamma, x_init):
        """Second restricted node movement algorithm (Section 4.3.2): the
        metric (1 - gamma) mu_98(T_0) + gamma mu(T) with T_0 = A W_0^{-1} and
        W_0 = A(x_init) at every point.  The composite metric is integrated
        over the primary target element (weight det W for both parts)."""
        if not (0.0 <= gamma <= 1.0):
            raise ValueError("gamma must lie in [0, 1]")
        A0 = self._jac(np.asarray(x_init, dtype=np.float64), 0, self.n_elem)
        if np.any(_det(A0) <= 0):
            raise ValueError("the initial mesh is inverted: W_0 = A_init needs det > 0")
        self.eta1 = float(gamma)
        self.second = dict(metric=98, Winv=np.linalg.inv(A0), omega=(1.0 - gamma) * self._primary_detW())

    def set_restriction(self, delta, x_init=None):
        """First restricted node movement algorithm (Section 4.3.1, eq. 4.2):
        adds delta |x - x_init|^2 integrated over the target elements, i.e.
        sum_E sum_q w_q det W delta |x(q) - x_init(q)|^2 with x(q) the
        finite element field of eq. 2.1 at the point.  delta = 0 removes it."""
        if not (delta >= 0.0 and math.isfinite(delta)):
            raise ValueError("delta must be finite and >= 0")
        self.delta = float(delta)
        self.x_init = None if delta == 0.0 else np.array(x_init, dtype=np.float64)

    def _terms(self, e0, e1):
        """(metric, W^{-1}, per-point weight) of every metric term on a chunk,
        W^{-1} broadcastable to (ne, nq, d, d), weight to (ne, nq)."""
        Wi, dW = self._targets(e0, e1)
        out = [(self.metric, Wi, self.eta1 * self.wq[None, :] * dW)]
        if self.second is not None:
            s = self.second
            out.append((s["metric"], s["Winv"][e0:e1], self.wq[None, :] * s["omega"][e0:e1]))
        return out

    def _penalty_weight(self, e0, e1):
        """2 delta w_q det W per point (the weight of the eq. 4.2 term's
        derivatives), shape broadcastable to (ne, nq)."""
        _, dW = self._targets(e0, e1)
        return 2.0 * self.delta * self.wq[None, :] * dW

    def _field_at_points(self, f, e0, e1):
        """f(q)[e, q, c] = sum_i f_{node(e,i), c} w_i(s_q) (eq. 2.1)."""
        return np.einsum("cei,qi->eqc", f[:, self.elem_node[e0:e1]], self.Bv, optimize=True)

    def _assemble_values(self, m, e0, e1, out):
        """out[c, node(e,i)] += sum_q m[e,q,c] w_i(s_q)."""
        G = np.einsum("eqc,qi->cei", m, self.Bv, optimize=True)
        for c in range(self.dim):
            np.add.at(out[c], self.elem_node[e0:e1], G[c])

    # per-chunk target data broadcast to (ne, nq, d, d) / (ne, nq)
    def _targets(self, e0, e1):
        Wi, dW = self.Winv, self.detW
        if Wi.ndim == 2:
            return Wi[None, None], np.broadcast_to(dW, (1, 1))
        if Wi.ndim == 3:
            return Wi[e0:e1, None], dW[e0:e1, None]
        return Wi[e0:e1], dW[e0:e1]

    def _jac(self, x, e0, e1):
        """A[e, q, c, l] = sum_i x_{node(e,i), c} dw_i/dxbar_l (eq. 2.2).

        The basis gradients sum to zero, so A is unchanged when the element's
        first node is subtracted from all its nodes; doing so keeps the
        summands at the size of the element rather than of the domain, which
        is what the rounding error of the sum is proportional to."""
        X = x[:, self.elem_node[e0:e1]]                  # (d, ne, N)
        X = X - X[:, :, :1]
        return np.einsum("cei,qil->eqcl", X, self.D, optimize=True)

    def _chunks(self):
        for e0 in range(0, self.n_elem, self.chunk):
            yield e0, min(e0 + self.chunk, self.n_elem)

    def subset(self, elems):
        """The same objective restricted to the given elements."""
        elems = np.asarray(elems, dtype=np.int64)
        sub = Problem.__new__(Problem)
        sub.__dict__.update(self.__dict__)
        sub.elem_node = self.elem_node[elems]
        sub.n_elem = elems.size
        if self.Winv.ndim > 2:
            sub.Winv, sub.detW = self.Winv[elems], self.detW[elems]
        if self.second is not None:
            sub.second = dict(self.second, Winv=self.second["Winv"][elems], omega=self.second["omega"][elems])
        return sub

    def pointwise(self, x, elems=None):
        """Per point contributions w_q det W mu(T) (plus the Section 4 terms
        that are set) and det A, shape (n_elem, nq); with elems, of those
        elements only."""
        if elems is not None:
            return self.subset(elems).pointwise(x)
        contrib, detA = [], []
        for e0, e1 in self._chunks():
            A = self._jac(x, e0, e1)
            c = 0.0
            for metric, Wi, wt in self._terms(e0, e1):
                c = c + wt * mu(metric, _mm(A, Wi))
            if self.delta > 0.0:
                u = self._field_at_points(x - self.x_init, e0, e1)
                c = c + 0.5 * self._penalty_weight(e0, e1) * np.sum(u * u, axis=-1)
            contrib.append(c)
            detA.append(_det(A))
        return np.concatenate(contrib), np.concatenate(detA)

    def energy(self, x):
        """(F_V, min det A) -- eq. 2.4 summed with math.fsum; positivity is
        judged at the quadrature points (Section 3.4)."""
        c, detA = self.pointwise(x)
        if np.iscomplexobj(c):
            F = math.fsum(c.real.ravel()) + 1j * math.fsum(c.imag.ravel())
            return F, float(np.min(detA.real))
        return math.fsum(c.ravel()), float(np.min(detA))

    def point_sizes(self, x):
        """(det A)^(1/d) at every quadrature point, shape (n_elem, nq): the
        sizes of the target W_3 = (det A(x_0))^(1/d) I of Section 3.1 when
        x is the initial mesh (real root: negative where det A < 0 in 3D,
        NaN in 2D)."""
        _, detA = self.pointwise(x)
        return np.sqrt(detA) if self.dim == 2 else np.cbrt(detA)

    def max_condition(self, x, elems=None):
        """max over quadrature points of (|T|^2/d)^(d/2) / det T: 1 for a
        scaled rotation, large for nearly degenerate points.  It bounds how
        much a relative perturbation of A is amplified in mu's derivatives."""
        en_all, n_all = self.elem_node, self.n_elem
        if elems is not None:
            self.elem_node, self.n_elem = en_all[np.asarray(elems)], len(elems)
        try:
            k = 0.0
            for e0, e1 in self._chunks():
                Wi, _ = self._targets(e0, e1)
                T = _mm(self._jac(x, e0, e1), Wi)
                k = max(k, float(np.max((_frob2(T) / self.dim) ** (self.dim / 2.0) / _det(T))))
            return k
        finally:
            self.elem_node, self.n_elem = en_all, n_all

    def element_min_det(self, x, elems=None):
        """Smallest det A over the quadrature points of each element."""
        en_all, n_all = self.elem_node, self.n_elem
        if elems is not None:
            self.elem_node, self.n_elem = en_all[np.asarray(elems)], len(elems)
        try:
            _, detA = self.pointwise(x)
        finally:
            self.elem_node, self.n_elem = en_all, n_all
        return np.min(np.real(detA), axis=1)

    def bad_elements(self, x, elems=None, tau_min=0.0):
        """Positions (within `elems`, default all elements) of the elements
        with det A <= tau_min det W at some quadrature point."""
        md = self.element_min_det(x, elems)
        dW = self.detW if np.ndim(self.detW) == 0 else None
        if dW is None:
            dWe = self.detW if self.detW.ndim == 1 else self.detW.min(axis=1)
            dW = dWe if elems is None else dWe[np.asarray(elems)]
        return np.flatnonzero(md <= tau_min * dW)

    def _assemble(self, Y, e0, e1, out):
        """out[c, node(e,i)] += sum_q sum_l Y[e,q,c,l] dw_i/dxbar_l."""
        G = np.einsum("eqcl,qil->cei", Y, self.D, optimize=True)
        for c in range(self.dim):
            np.add.at(out[c], self.elem_node[e0:e1], G[c])

    def gradient(self, x):
        """dF_V/dx (Section 3.4): sum_E sum_q w_q det W (P W^{-t}) grad w_i,
        full (all DOFs, boundary included)."""
        g = np.zeros(x.shape, dtype=np.result_type(x, np.float64))
        for e0, e1 in self._chunks():
            A = self._jac(x, e0, e1)
            for metric, Wi, wt in self._terms(e0, e1):
                P = dmu(metric, _mm(A, Wi))
                self._assemble(wt[..., None, None] * _mm(P, _tr(Wi)), e0, e1, g)
            if self.delta > 0.0:
                u = self._field_at_points(x - self.x_init, e0, e1)
                self._assemble_values(self._penalty_weight(e0, e1)[..., None] * u, e0, e1, g)
        return g

    def _elements_touching(self, nodes):
        hit = np.isin(self.elem_node, np.asarray(nodes)).any(axis=1)
        return np.flatnonzero(hit)

    def gradient_at(self, x, nodes):
        """dF/dx at the given nodes only, shape (d, len(nodes)): the same sum
        as gradient(), restricted to the elements that contain the nodes."""
        return self._restricted(x, None, nodes)

    def hessian_apply_at(self, x, v, nodes):
        """(Hv) at the given nodes only, shape (d, len(nodes))."""
        return self._restricted(x, v, nodes)

    def _restricted(self, x, v, nodes):
        nodes = np.asarray(nodes, dtype=np.int64)
        sub = self.subset(self._elements_touching(nodes))
        out = sub.gradient(x) if v is None else sub.hessian_apply(x, v)
        return out[:, nodes]

    def hessian_apply(self, x, v):
        """(d^2 F_V / dx^2) v with dT = dA W^{-1}, dA from v as in eq. 2.2,
        and the second derivative of mu applied to dT (Section 3.4)."""
        Hv = np.zeros(x.shape, dtype=np.result_type(x, v, np.float64))
        for e0, e1 in self._chunks():
            A = self._jac(x, e0, e1)
            dA = self._jac(v, e0, e1)
            for metric, Wi, wt in self._terms(e0, e1):
                dP = d2mu(metric, _mm(A, Wi), _mm(dA, Wi))
                self._assemble(wt[..., None, None] * _mm(dP, _tr(Wi)), e0, e1, Hv)
            if self.delta > 0.0:
                vq = self._field_at_points(v, e0, e1)
                self._assemble_values(self._penalty_weight(e0, e1)[..., None] * vq, e0, e1, Hv)
        return Hv

    def hessian_diagonal(self, x):
        """The diagonal of d^2 F_V / dx^2 (Section 3.4), shape (d, n_node):
        entry (c, I) is the Hessian action on the unit vector of DOF (c, I),
        read at (c, I).  Element E's share for its local node i is
        sum_q w_q det W  dT : mu''(T)[dT]  with dT = e_c (grad w_i)^T W^{-1}
        (the unit vector's dA, row c = grad w_i, times W^{-1})."""
        Dg = np.zeros(x.shape, dtype=np.result_type(x, np.float64))
        d = self.dim
        for e0, e1 in self._chunks():
            A = self._jac(x, e0, e1)
            ne = e1 - e0
            share = np.zeros((d, ne, self.D.shape[1]), dtype=Dg.dtype)
            for metric, Wi, wt in self._terms(e0, e1):
                T = _mm(A, Wi)
                for i in range(self.D.shape[1]):
                    for c in range(d):
                        dA = np.zeros((ne, self.nq, d, d), dtype=Dg.dtype)
                        dA[:, :, c, :] = self.D[None, :, i, :]
                        dT = _mm(dA, Wi)
                        q = _ddot(dT, d2mu(metric, T, dT))
                        share[c, :, i] += np.sum(wt * q, axis=1)
            if self.delta > 0.0:
                # the unit vector's field at the points is w_i(s_q) in component c
                pw = np.broadcast_to(self._penalty_weight(e0, e1), (ne, self.nq))
                share += (pw @ (self.Bv * self.Bv))[None]
            for c in range(d):
                np.add.at(Dg[c], self.elem_node[e0:e1], share[c])
        return Dg


# ---------------------------------------------------------------------------
# Section 3.4: Newton's method with the scaled update and line search

@dataclass
class NewtonOptions:
    rtol: float = 1e-12          # Newton relative tolerance (Section 5)
    atol: float = 0.0            # absolute floor on |g| (for meshes already at the optimum)
    max_it: int = 50
    cg_rtol: float = 1e-8
    cg_max_it: int = 1000
    ls_shrink: float = 0.5
    ls_max: int = 30
    f_growth: float = 1.2        # F(x+) < 1.2 F(x)
    g_growth: float = 1.2        # |g(x+)| < 1.2 |g(x)|
    ftarget: float = -math.inf   # also stop once F <= ftarget
    cg_forcing: int = 0          # 1: inner tolerance max(cg_rtol, min(0.5, sqrt(|g|/|g0|)))
    inner: str = "shifted_cg"    # "shifted_cg": CG on H + tau I (see shifted_cg); "cg": truncated CG;
                                 # "minres": MINRES, the solver of Section 5
    shift_beta: float = 1e-3     # shifted_cg: the floor of tau relative to the mean |diag H| (free DOFs)
    precond: str = "none"        # "none" or "jacobi": M = |diag H| on the free DOFs


STOP_CONVERGED, STOP_MAXIT, STOP_LSFAIL, STOP_INVERTED = 0, 1, 2, 3


@dataclass
class NewtonReport:
    iters: int = 0
    cg_iters: int = 0
    ls_shrinks: int = 0
    stop: int = STOP_MAXIT
    F0: float = 0.0
    F: float = 0.0
    gnorm0: float = 0.0
    gnorm: float = 0.0
    min_detA: float = 0.0
    history: list = field(default_factory=list)   # per iteration: (F, |g|, alpha, cg_iters, neg_curv)
                                                  # (neg_curv: a flag for "cg", the CG restarts for "shifted_cg")


def truncated_cg(apply_H, g, rtol, max_it, minv=None):
    """Steihaug's truncated conjugate gradients for H d = -g from d = 0, with
    an optional diagonal preconditioner M (minv = 1 / diag M): on
    non-positive curvature return the preconditioned steepest-descent
    direction -M^{-1} g (-g without M) at the first step, else the current
    iterate; stop once the residual |r|_2 <= rtol |g|_2.  Returns
    (d, iterations, negative-curvature flag)."""
    d = np.zeros_like(g)
    r = -g
    z = r if minv is None else minv * r
    p = z.copy()
    rz = float(np.dot(r, z))
    gnorm = math.sqrt(float(np.dot(g, g)))
    for j in range(max_it):
        Hp = apply_H(p)
        pHp = float(np.dot(p, Hp))
        if pHp <= 0.0:
            return (p if j == 0 else d), j + 1, True
        alpha = rz / pHp
        d = d + alpha * p
        r = r - alpha * Hp
        if math.sqrt(float(np.dot(r, r))) <= rtol * gnorm:
            return d, j + 1, False
        z = r if minv is None else minv * r
        rz_new = float(np.dot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return d, max_it, False


def _cg_or_negative(apply_H, g, rtol, max_it, minv=None):
    """Preconditioned CG for H d = -g from d = 0, stopped once |r|_2 <=
    rtol |g|_2, or at the first non-positive curvature p.Hp <= 0.  Returns
    (d, iterations, negative-curvature flag)."""
    d = np.zeros_like(g)
    r = -g
    z = r if minv is None else minv * r
    p = z.copy()
    rz = float(np.dot(r, z))
    gnorm = math.sqrt(float(np.dot(g, g)))
    for j in range(max_it):
        Hp = apply_H(p)
        pHp = float(np.dot(p, Hp))
        if not pHp > 0.0:
            return d, j + 1, True
        alpha = rz / pHp
        d = d + alpha * p
        r = r - alpha * Hp
        if math.sqrt(float(np.dot(r, r))) <= rtol * gnorm:
            return d, j + 1, False
        z = r if minv is None else minv * r
        rz_new = float(np.dot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return d, max_it, False


def shifted_cg(apply_H, g, rtol, max_it, diag, beta_rel=1e-3, minv=None, max_shifts=64):
    """CG on the modified Hessian H + tau I: the added multiple of the
    identity of Nocedal and Wright (Numerical Optimization, 2nd ed., Alg.
    3.3), with a CG run standing in for their Cholesky factorization as the
    test of positive definiteness.  beta = beta_rel times the mean |diag H|
    (diag: the diagonal on the free DOFs, a scale of H); tau_0 = 0 if every
    diagonal entry is positive, else -min diag + beta; while CG meets
    curvature p.(H + tau I)p <= 0, tau <- max(2 tau, beta) and CG restarts
    from d = 0.  The direction solves (H + tau I) d = -g to the CG tolerance
    with H + tau I positive definite on the Krylov space, so it descends.
    Returns (d, total CG iterations, number of restarts, tau)."""
    diag = np.asarray(diag, dtype=np.float64)
    beta = beta_rel * float(np.mean(np.abs(diag)))
    dmin = float(np.min(diag))
    tau = 0.0 if dmin > 0.0 else -dmin + beta
    total = 0
    for k in range(max_shifts):
        op = apply_H if tau == 0.0 else (lambda p, t=tau: apply_H(p) + t * p)
        d, it, neg = _cg_or_negative(op, g, rtol, max_it, minv)
        total += it
        if not neg:
            return d, total, k, tau
        tau = max(2.0 * tau, beta)
    return -g if minv is None else -minv * g, total, max_shifts, tau


def minres(apply_H, b, rtol, max_it, minv=None):
    """MINRES (Paige and Saunders, 1975) for the symmetric, possibly
    indefinite system H d = b from d = 0, with an optional symmetric positive
    definite diagonal preconditioner M (minv = 1 / diag M).

    Preconditioned Lanczos builds the tridiagonal T_k (diagonal alpha_k,
    off-diagonal beta_{k+1}) of H in the M^{-1} inner product; Givens
    rotations keep its QR factorization up to date, so the iterate
    minimizing the M^{-1}-norm of the residual over the Krylov space is
    reached by a three-term update of the directions w_k, and |phibar_k| is
    that residual norm.  Stops when |phibar_k| <= rtol beta_1 (the residual
    relative to the right-hand side, both in the M^{-1} norm: the 2-norm
    without M).  Returns (d, iterations)."""
    prec = (lambda u: u) if minv is None else (lambda u: minv * u)
    d = np.zeros_like(b)
    r_prev = np.zeros_like(b)            # r_{k-1}
    r_cur = b.copy()                     # r_k
    y = prec(r_cur)
    beta = math.sqrt(float(np.dot(r_cur, y)))
    beta1 = beta
    if beta1 == 0.0:
        return d, 0
    beta_prev = 0.0
    c, s = -1.0, 0.0                     # rotation of the previous step
    dbar, eps = 0.0, 0.0                 # entries of the next column, pre-rotated
    phibar = beta1
    w_prev = np.zeros_like(b)            # w_{k-2}
    w_cur = np.zeros_like(b)             # w_{k-1}
    for k in range(1, max_it + 1):
        v = y / beta                     # Lanczos vector v_k
        Hv = apply_H(v)
        alpha = float(np.dot(v, Hv))
        r_next = Hv - (alpha / beta) * r_cur
        if k > 1:
            r_next = r_next - (beta / beta_prev) * r_prev
        y = prec(r_next)
        beta_next = math.sqrt(float(np.dot(r_next, y)))
        # previous rotation on column k (entries dbar at row k-1, alpha at
        # row k) and on column k+1 (beta_next at row k)
        eps_k = eps
        delta = c * dbar + s * alpha
        gbar = s * dbar - c * alpha
        eps = s * beta_next
        dbar = -c * beta_next
        # new rotation annihilating beta_next under gbar
        gamma = math.hypot(gbar, beta_next)
        if gamma == 0.0:
            gamma = np.finfo(np.float64).tiny
        c, s = gbar / gamma, beta_next / gamma
        phi = c * phibar
        phibar = s * phibar
        w_new = (v - eps_k * w_prev - delta * w_cur) / gamma
        d = d + phi * w_new
        w_prev, w_cur = w_cur, w_new
        r_prev, r_cur = r_cur, r_next
        beta_prev, beta = beta, beta_next
        if abs(phibar) <= rtol * beta1 or beta == 0.0:
            return d, k
    return d, max_it


def jacobi_inverse(diag, m):
    """1 / M for the Jacobi preconditioner M = |diag H| on the free DOFs
    (mask m = 1) and 1 on fixed DOFs or where the diagonal vanishes."""
    a = np.abs(np.asarray(diag, dtype=np.float64))
    M = np.where((m > 0) & (a > 0.0), a, 1.0)
    return 1.0 / M


def newton_solve(prob: Problem, x0, fixed, opts: NewtonOptions = NewtonOptions()):
    """Minimize F_V over the free DOFs (fixed[c, I] = 1 marks Dirichlet).

    Each iteration: masked gradient g, a direction from the masked Hessian
    (CG on the Hessian plus a multiple of the identity where it is not
    positive definite (shifted_cg), truncated CG, or MINRES as in Section 5;
    optionally Jacobi preconditioned), then alpha = 1, 1/2, ... until the new mesh has det A > 0 at
    every quadrature point, F(x+) < 1.2 F(x) and |g(x+)| < 1.2 |g(x)|;
    stops when no alpha works (Section 3.4), when |g| <= rtol |g0|
    (Section 5), or after max_it iterations."""
    m = (1 - np.asarray(fixed, dtype=np.float64)).ravel()
    shape = x0.shape
    x = np.array(x0, dtype=np.float64).ravel()
    rep = NewtonReport()
    F, mindet = prob.energy(x.reshape(shape))
    rep.F0, rep.F, rep.min_detA = F, F, mindet
    if mindet <= 0.0:
        rep.stop = STOP_INVERTED
        return x.reshape(shape), rep
    grad = lambda y: m * prob.gradient(y.reshape(shape)).ravel()
    g = grad(x)
    gn = math.sqrt(float(np.dot(g, g)))
    rep.gnorm0 = rep.gnorm = gn
    rep.history.append((F, gn, 0.0, 0, False))
    for it in range(opts.max_it):
        if gn <= max(opts.rtol * rep.gnorm0, opts.atol) or F <= opts.ftarget:
            rep.stop = STOP_CONVERGED
            break
        cg_tol = opts.cg_rtol
        if opts.cg_forcing:
            cg_tol = max(opts.cg_rtol, min(0.5, math.sqrt(gn / rep.gnorm0)))
        Hm = lambda p: m * prob.hessian_apply(x.reshape(shape), (m * p).reshape(shape)).ravel()
        minv = None
        if opts.precond == "jacobi":
            minv = jacobi_inverse(prob.hessian_diagonal(x.reshape(shape)).ravel(), m)
        elif opts.precond != "none":
            raise ValueError(f"unknown preconditioner {opts.precond}")
        if opts.inner == "shifted_cg":
            diag = prob.hessian_diagonal(x.reshape(shape)).ravel()[m > 0]
            dvec, ncg, nshift, _ = shifted_cg(Hm, g, cg_tol, opts.cg_max_it, diag, opts.shift_beta, minv)
            neg = nshift
        elif opts.inner == "cg":
            dvec, ncg, neg = truncated_cg(Hm, g, cg_tol, opts.cg_max_it, minv)
        elif opts.inner == "minres":
            dvec, ncg = minres(Hm, -g, cg_tol, opts.cg_max_it, minv)
            neg = False
        else:
            raise ValueError(f"unknown inner solver {opts.inner}")
        rep.cg_iters += ncg
        accepted = False
        for k in range(opts.ls_max):
            alpha = opts.ls_shrink ** k
            xt = x + alpha * dvec
            Ft, mindet_t = prob.energy(xt.reshape(shape))
            if mindet_t > 0.0 and Ft < opts.f_growth * F:
                gt = grad(xt)
                gnt = math.sqrt(float(np.dot(gt, gt)))
                if gnt < opts.g_growth * gn:
                    accepted = True
                    break
            rep.ls_shrinks += 1
        if not accepted:
            rep.stop = STOP_LSFAIL
            break
        x, F, g, gn, mindet = xt, Ft, gt, gnt, mindet_t
        rep.iters = it + 1
        rep.history.append((F, gn, alpha, ncg, neg))
    else:
        rep.stop = (STOP_CONVERGED if gn <= max(opts.rtol * rep.gnorm0, opts.atol) or F <= opts.ftarget
                    else STOP_MAXIT)
    rep.F, rep.gnorm, rep.min_detA = F, gn, mindet
    return x.reshape(shape), rep
