"""Python binding of libtmop (ctypes).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.

The functions carry the names of the C ABI (include/tmop.h):
tmop_setup, tmop_energy, tmop_gradient, tmop_energy_gradient, tmop_hessian_apply,
tmop_hessian_diagonal, tmop_newton_solve, tmop_destroy.  Device arrays are torch tensors of shape
(dim, n_node), float64, contiguous, on a HIP device; the work is enqueued
on torch's current stream of that device.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtmop.so")

TMOP_OK, TMOP_W_INVERTED, TMOP_W_MAXIT, TMOP_W_LSFAIL = 0, 1, 2, 3
TMOP_E_ARG, TMOP_E_TARGET, TMOP_E_NOMEM, TMOP_E_HIP, TMOP_E_UNSUPPORTED, TMOP_E_SCRATCH = -1, -2, -3, -4, -5, -6
TMOP_MU1, TMOP_MU2, TMOP_MU7, TMOP_MU9, TMOP_MU14, TMOP_MU77, TMOP_MU98 = 1, 2, 7, 9, 14, 77, 98
TMOP_MU302, TMOP_MU303 = 302, 303
TMOP_GAUSS_LEGENDRE, TMOP_GAUSS_LOBATTO = 0, 1
TMOP_FP64, TMOP_MIXED_FP32 = 0, 1
TMOP_TGT_CONST, TMOP_TGT_ISO_PER_QP, TMOP_TGT_PER_ELEM, TMOP_TGT_PER_QP = 0, 1, 2, 3
TMOP_INNER_CG, TMOP_INNER_MINRES, TMOP_INNER_SHIFTED_CG = 0, 1, 2
TMOP_PREC_NONE, TMOP_PREC_JACOBI = 0, 1
TMOP_SCATTER_COLOURS, TMOP_SCATTER_TILES, TMOP_SCATTER_ELEMENTS = 0, 1, 2

EXPORTS = ("tmop_setup", "tmop_energy", "tmop_gradient", "tmop_gradient_scaled", "tmop_hessian_apply",
           "tmop_newton_solve", "tmop_destroy", "tmop_strerror", "tmop_newton_default_opts",
           "tmop_timing_enable", "tmop_timing_read", "tmop_energy_gradient", "tmop_hessian_diagonal",
           "tmop_target_sizes_w3", "tmop_set_target_sizes", "tmop_set_restriction", "tmop_set_combo",
           "tmop_set_replication", "tmop_dfo_default_opts", "tmop_dfo_sweep", "tmop_dfo_solve",
           "tmop_energy_noalloc", "tmop_set_scatter", "tmop_get_scatter")
# timing slots: the element-kernel operations, then the W_0 data and the penalty kernels
TIMING_ENERGY, TIMING_GRAD, TIMING_HESS, TIMING_EG, TIMING_DIAG, TIMING_SIZE = 0, 1, 2, 3, 4, 5
TIMING_W0, TIMING_PENALTY = 6, 7


class TMOPError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {tmop_strerror(status)} (status {status})")
        self.status = status


class tmop_mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("order", ctypes.c_int32), ("n_elem", ctypes.c_int64),
                ("n_node", ctypes.c_int64), ("elem_node", ctypes.POINTER(ctypes.c_int32)),
                ("fixed", ctypes.POINTER(ctypes.c_uint8))]


class tmop_quadrature(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n1d", ctypes.c_int32)]


class tmop_target(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("W", ctypes.POINTER(ctypes.c_double))]


class tmop_newton_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("max_it", ctypes.c_int32),
                ("cg_rtol", ctypes.c_double), ("cg_max_it", ctypes.c_int32), ("ls_shrink", ctypes.c_double),
                ("ls_max", ctypes.c_int32), ("f_growth", ctypes.c_double), ("g_growth", ctypes.c_double),
                ("hist_F", ctypes.POINTER(ctypes.c_double)), ("hist_gnorm", ctypes.POINTER(ctypes.c_double)),
                ("hist_cg", ctypes.POINTER(ctypes.c_int32)), ("ftarget", ctypes.c_double),
                ("cg_forcing", ctypes.c_int32), ("hist_time", ctypes.POINTER(ctypes.c_double)),
                ("inner", ctypes.c_int32), ("precond", ctypes.c_int32), ("shift_beta", ctypes.c_double)]


class tmop_newton_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("cg_iters", ctypes.c_int32), ("ls_shrinks", ctypes.c_int32),
                ("neg_curv", ctypes.c_int32), ("F0", ctypes.c_double), ("F", ctypes.c_double),
                ("gnorm0", ctypes.c_double), ("gnorm", ctypes.c_double), ("min_detA", ctypes.c_double)]


class tmop_dfo_opts(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("max_sweeps", ctypes.c_int32), ("step", ctypes.c_double),
                ("xtol", ctypes.c_double), ("max_evals", ctypes.c_int32)]


class tmop_dfo_report(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("converged", ctypes.c_int32), ("F0", ctypes.c_double),
                ("F", ctypes.c_double), ("max_move", ctypes.c_double)]


_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtmop.so; raises (never falls back) when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_1807_09807_amd.build`")
    lib = ctypes.CDLL(path)
    P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.tmop_setup.argtypes = [ctypes.POINTER(tmop_mesh), ctypes.POINTER(tmop_quadrature),
                               ctypes.POINTER(tmop_target), i32, i32, ctypes.POINTER(P)]
    lib.tmop_setup.restype = ctypes.c_int
    lib.tmop_energy.argtypes = [P, P, ctypes.POINTER(dbl), ctypes.POINTER(dbl), P]
    lib.tmop_energy.restype = ctypes.c_int
    lib.tmop_energy_noalloc.argtypes = [P, P, ctypes.POINTER(dbl), ctypes.POINTER(dbl), P]
    lib.tmop_energy_noalloc.restype = ctypes.c_int
    lib.tmop_gradient.argtypes = [P, P, P, P]
    lib.tmop_gradient.restype = ctypes.c_int
    lib.tmop_gradient_scaled.argtypes = [P, P, P, P, P]
    lib.tmop_gradient_scaled.restype = ctypes.c_int
    lib.tmop_hessian_apply.argtypes = [P, P, P, P, P]
    lib.tmop_hessian_apply.restype = ctypes.c_int
    lib.tmop_hessian_diagonal.argtypes = [P, P, P, P]
    lib.tmop_hessian_diagonal.restype = ctypes.c_int
    lib.tmop_set_scatter.argtypes = [P, ctypes.c_int32]
    lib.tmop_set_scatter.restype = ctypes.c_int
    lib.tmop_get_scatter.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    lib.tmop_get_scatter.restype = ctypes.c_int
    lib.tmop_target_sizes_w3.argtypes = [P, P, P, P]
    lib.tmop_target_sizes_w3.restype = ctypes.c_int
    lib.tmop_set_target_sizes.argtypes = [P, P, P]
    lib.tmop_set_target_sizes.restype = ctypes.c_int
    lib.tmop_set_restriction.argtypes = [P, ctypes.c_double, P, P]
    lib.tmop_set_restriction.restype = ctypes.c_int
    lib.tmop_set_combo.argtypes = [P, ctypes.c_int32, P, ctypes.c_double, ctypes.c_double, P, P]
    lib.tmop_set_combo.restype = ctypes.c_int
    lib.tmop_set_replication.argtypes = [P, ctypes.c_double, P, P]
    lib.tmop_set_replication.restype = ctypes.c_int
    lib.tmop_dfo_default_opts.argtypes = [ctypes.POINTER(tmop_dfo_opts)]
    lib.tmop_dfo_default_opts.restype = None
    lib.tmop_dfo_sweep.argtypes = [P, P, ctypes.POINTER(tmop_dfo_opts), ctypes.POINTER(dbl), P]
    lib.tmop_dfo_sweep.restype = ctypes.c_int
    lib.tmop_dfo_solve.argtypes = [P, P, ctypes.POINTER(tmop_dfo_opts), ctypes.POINTER(tmop_dfo_report), P]
    lib.tmop_dfo_solve.restype = ctypes.c_int
    lib.tmop_newton_solve.argtypes = [P, P, ctypes.POINTER(tmop_newton_opts),
                                      ctypes.POINTER(tmop_newton_report), P]
    lib.tmop_newton_solve.restype = ctypes.c_int
    lib.tmop_destroy.argtypes = [P]
    lib.tmop_destroy.restype = None
    lib.tmop_strerror.argtypes = [ctypes.c_int]
    lib.tmop_strerror.restype = ctypes.c_char_p
    lib.tmop_newton_default_opts.argtypes = [ctypes.POINTER(tmop_newton_opts)]
    lib.tmop_newton_default_opts.restype = None
    lib.tmop_energy_gradient.argtypes = [P, P, ctypes.POINTER(dbl), ctypes.POINTER(dbl), P, P]
    lib.tmop_energy_gradient.restype = ctypes.c_int
    lib.tmop_timing_enable.argtypes = [P, ctypes.c_int]
    lib.tmop_timing_enable.restype = ctypes.c_int
    lib.tmop_timing_read.argtypes = [P, ctypes.c_int, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.tmop_timing_read.restype = ctypes.c_int
    _lib = lib
    return lib


def tmop_strerror(status: int) -> str:
    return load().tmop_strerror(int(status)).decode()


def _stream(t) -> ctypes.c_void_p:
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _check_field(t, dim, n_node, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 tensor on a HIP device")
    if tuple(t.shape) != (dim, n_node) or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with shape ({dim}, {n_node}), got {tuple(t.shape)}")


class Context:
    """Owns one tmop_ctx (tmop_setup ... tmop_destroy).  The target is the
    constant matrix W; or, when `target_sizes` ([n_elem][n_q1d^dim] host
    array) is given, the per-point isotropic targets W_q = s_q I; or, when W
    is a host array of shape (n_elem, dim, dim) or (n_elem, n_q1d^dim, dim,
    dim), general targets per element or per quadrature point."""

    def __init__(self, dim: int, order: int, elem_node: np.ndarray, n_node: int, n_q1d: int, metric: int,
                 W, fixed: Optional[np.ndarray] = None, precision: int = TMOP_FP64,
                 rule: int = TMOP_GAUSS_LEGENDRE, target_sizes: Optional[np.ndarray] = None):
        lib = load()
        self._lib = lib
        self.dim, self.order, self.n_node, self.metric, self.precision = dim, order, int(n_node), metric, precision
        en = np.ascontiguousarray(elem_node, dtype=np.int32)
        self.n_elem = en.shape[0]
        m = tmop_mesh(dim, order, self.n_elem, int(n_node), en.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None)
        if fixed is not None:
            fx = np.ascontiguousarray(fixed, dtype=np.uint8)
            if fx.shape != (dim, n_node):
                raise ValueError("fixed must have shape (dim, n_node)")
            m.fixed = fx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        q = tmop_quadrature(rule, n_q1d)
        self.nq = n_q1d ** dim
        if target_sizes is not None:
            Wa = np.ascontiguousarray(target_sizes, dtype=np.float64)
            if Wa.shape != (self.n_elem, self.nq):
                raise ValueError(f"target_sizes must have shape ({self.n_elem}, {self.nq})")
            t = tmop_target(TMOP_TGT_ISO_PER_QP, Wa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        else:
            Wa = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
            if Wa.shape == (self.n_elem, dim, dim) and Wa.ndim == 3:
                kind = TMOP_TGT_PER_ELEM
            elif Wa.shape == (self.n_elem, self.nq, dim, dim):
                kind = TMOP_TGT_PER_QP
            elif Wa.size == dim * dim:
                kind = TMOP_TGT_CONST
                Wa = Wa.reshape(dim, dim)
            else:
                raise ValueError(f"W must be ({dim}, {dim}), (n_elem, {dim}, {dim}) or "
                                 f"(n_elem, {self.nq}, {dim}, {dim}), got {Wa.shape}")
            t = tmop_target(kind, Wa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        h = ctypes.c_void_p()
        st = lib.tmop_setup(ctypes.byref(m), ctypes.byref(q), ctypes.byref(t), metric, precision, ctypes.byref(h))
        if st < 0:
            raise TMOPError(st, "tmop_setup")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tmop_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def energy(self, x):
        """(F, min det A, status).  status is TMOP_OK or TMOP_W_INVERTED."""
        _check_field(x, self.dim, self.n_node, "x")
        F, md = ctypes.c_double(), ctypes.c_double()
        st = self._lib.tmop_energy(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(F), ctypes.byref(md), _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_energy")
        return F.value, md.value, st

    def energy_noalloc(self, x):
        """(F, min det A, status) as energy(), from the library's fixed
        scratch (tmop_energy_noalloc: no device allocation)."""
        _check_field(x, self.dim, self.n_node, "x")
        F, md = ctypes.c_double(), ctypes.c_double()
        st = self._lib.tmop_energy_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(F), ctypes.byref(md),
                                           _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_energy_noalloc")
        return F.value, md.value, st

    def energy_gradient(self, x, out=None):
        """(F, min det A, status, g) from one pass over the elements."""
        import torch
        _check_field(x, self.dim, self.n_node, "x")
        out = torch.empty_like(x) if out is None else out
        _check_field(out, self.dim, self.n_node, "out")
        F, md = ctypes.c_double(), ctypes.c_double()
        st = self._lib.tmop_energy_gradient(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(F), ctypes.byref(md),
                                            ctypes.c_void_p(out.data_ptr()), _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_energy_gradient")
        return F.value, md.value, st, out

    def gradient(self, x, out=None):
        import torch
        _check_field(x, self.dim, self.n_node, "x")
        out = torch.empty_like(x) if out is None else out
        _check_field(out, self.dim, self.n_node, "out")
        st = self._lib.tmop_gradient(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_gradient")
        return out

    def gradient_scaled(self, x, scale, out=None):
        """out = scale * dF/dx with `scale` a one-element float64 device
        tensor (the reverse-mode upstream gradient)."""
        import torch
        _check_field(x, self.dim, self.n_node, "x")
        if not (isinstance(scale, torch.Tensor) and scale.dtype == torch.float64 and scale.numel() == 1
                and scale.device == x.device):
            raise TypeError("scale must be a one-element float64 tensor on x's device")
        scale = scale.contiguous()
        out = torch.empty_like(x) if out is None else out
        _check_field(out, self.dim, self.n_node, "out")
        st = self._lib.tmop_gradient_scaled(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(scale.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_gradient_scaled")
        return out

    def hessian_apply(self, x, v, out=None):
        import torch
        _check_field(x, self.dim, self.n_node, "x")
        _check_field(v, self.dim, self.n_node, "v")
        out = torch.empty_like(x) if out is None else out
        _check_field(out, self.dim, self.n_node, "out")
        st = self._lib.tmop_hessian_apply(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_hessian_apply")
        return out

    def set_scatter(self, mode):
        """TMOP_SCATTER_ELEMENTS, TMOP_SCATTER_COLOURS or TMOP_SCATTER_TILES
        (2D): how the gradient and Hessian action add element contributions
        at shared nodes."""
        st = self._lib.tmop_set_scatter(self._h, int(mode))
        if st < 0:
            raise TMOPError(st, "tmop_set_scatter")

    @property
    def scatter(self):
        """The scatter mode in effect (the mesh's default until set_scatter)."""
        m = ctypes.c_int32(-1)
        st = self._lib.tmop_get_scatter(self._h, ctypes.byref(m))
        if st < 0:
            raise TMOPError(st, "tmop_get_scatter")
        return m.value

    def hessian_diagonal(self, x, out=None):
        """diag(d^2F/dx^2) over all DOFs, shape (dim, n_node)."""
        import torch
        _check_field(x, self.dim, self.n_node, "x")
        out = torch.empty_like(x) if out is None else out
        _check_field(out, self.dim, self.n_node, "out")
        st = self._lib.tmop_hessian_diagonal(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                             _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_hessian_diagonal")
        return out

    def target_sizes_w3(self, x0, out=None):
        """(sizes, status): (det A(x0))^(1/dim) at every quadrature point,
        a float64 device tensor [n_elem][n_q1d^dim]; status TMOP_OK or
        TMOP_W_INVERTED."""
        import torch
        _check_field(x0, self.dim, self.n_node, "x0")
        out = torch.empty((self.n_elem, self.nq), dtype=torch.float64, device=x0.device) if out is None else out
        if tuple(out.shape) != (self.n_elem, self.nq) or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of shape (n_elem, n_q1d^dim)")
        st = self._lib.tmop_target_sizes_w3(self._h, ctypes.c_void_p(x0.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                            _stream(x0))
        if st < 0:
            raise TMOPError(st, "tmop_target_sizes_w3")
        return out, st

    def set_target_sizes(self, sizes):
        """Replaces the per-point target sizes (device tensor [n_elem][n_q1d^dim])."""
        import torch
        if not (isinstance(sizes, torch.Tensor) and sizes.dtype == torch.float64 and sizes.is_cuda
                and tuple(sizes.shape) == (self.n_elem, self.nq) and sizes.is_contiguous()):
            raise ValueError("sizes must be a contiguous float64 device tensor of shape (n_elem, n_q1d^dim)")
        st = self._lib.tmop_set_target_sizes(self._h, ctypes.c_void_p(sizes.data_ptr()), _stream(sizes))
        if st < 0:
            raise TMOPError(st, "tmop_set_target_sizes")

    def set_restriction(self, delta: float, x_init=None):
        """Displacement penalty delta |x - x_init|^2 of Section 4.3.1 (eq. 4.2);
        x_init: device tensor (dim, n_node), copied; delta = 0 removes it."""
        ptr = None
        if x_init is not None:
            _check_field(x_init, self.dim, self.n_node, "x_init")
            ptr = ctypes.c_void_p(x_init.data_ptr())
        st = self._lib.tmop_set_restriction(self._h, float(delta), ptr,
                                            _stream(x_init) if x_init is not None else None)
        if st < 0:
            raise TMOPError(st, "tmop_set_restriction")

    def set_combo(self, metric2: int, W2=None, eta1: float = 1.0, eta2: float = 1.0, eta2_q=None):
        """Second metric term of eq. 4.1: eta1 mu + eta2 eta2_q det W2 mu2(A W2^-1)
        (W2: dim x dim host matrix; eta2_q: host (n_elem, n_q1d^dim) weights or
        None); metric2 = 0 removes it."""
        W2p, Wbuf, qbuf = None, None, None
        if W2 is not None:
            Wbuf = np.ascontiguousarray(np.asarray(W2, dtype=np.float64).reshape(-1))
            if Wbuf.size != self.dim * self.dim:
                raise ValueError(f"W2 must be a {self.dim}x{self.dim} matrix")
            W2p = Wbuf.ctypes.data_as(ctypes.c_void_p)
        qp = None
        if eta2_q is not None:
            qbuf = np.ascontiguousarray(np.asarray(eta2_q, dtype=np.float64))
            if qbuf.shape != (self.n_elem, self.nq):
                raise ValueError(f"eta2_q must have shape ({self.n_elem}, {self.nq})")
            qp = qbuf.ctypes.data_as(ctypes.c_void_p)
        st = self._lib.tmop_set_combo(self._h, int(metric2), W2p, float(eta1), float(eta2), qp, None)
        if st < 0:
            raise TMOPError(st, "tmop_set_combo")

    def set_replication(self, gamma: float, x_init):
        """The replication composite of Section 4.3.2 with W0 = A(x_init)."""
        _check_field(x_init, self.dim, self.n_node, "x_init")
        st = self._lib.tmop_set_replication(self._h, float(gamma), ctypes.c_void_p(x_init.data_ptr()),
                                            _stream(x_init))
        if st < 0:
            raise TMOPError(st, "tmop_set_replication")

    def _dfo_opts(self, opts):
        o = tmop_dfo_opts()
        self._lib.tmop_dfo_default_opts(ctypes.byref(o))
        for k, v in opts.items():
            if not hasattr(o, k):
                raise ValueError(f"unknown derivative-free option {k}")
            setattr(o, k, v)
        return o

    def dfo_sweep(self, x, **opts):
        """One sweep of the derivative-free solver (Section 3.4) over x in
        place; returns the largest node move.  Options: tmop_dfo_opts fields."""
        _check_field(x, self.dim, self.n_node, "x")
        o = self._dfo_opts(opts)
        mv = ctypes.c_double()
        st = self._lib.tmop_dfo_sweep(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(o), ctypes.byref(mv),
                                      _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_dfo_sweep")
        return mv.value

    def dfo_solve(self, x, **opts):
        """Derivative-free solve of x in place; returns (status, report dict)."""
        _check_field(x, self.dim, self.n_node, "x")
        o = self._dfo_opts(opts)
        rep = tmop_dfo_report()
        st = self._lib.tmop_dfo_solve(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(o), ctypes.byref(rep),
                                      _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_dfo_solve")
        return st, {k: getattr(rep, k) for k, _ in tmop_dfo_report._fields_}

    def timing_enable(self, on: bool = True):
        """Clears the per-launch kernel timing totals and turns timing on/off."""
        st = self._lib.tmop_timing_enable(self._h, int(bool(on)))
        if st < 0:
            raise TMOPError(st, "tmop_timing_enable")

    def timing_read(self, op: int):
        """(summed device ms, launch count) of the element kernels of one
        operation (0 energy, 1 gradient, 2 Hessian action, 3 energy +
        gradient, 4 Hessian diagonal, 5 target sizes, 6 replication W0 data,
        7 displacement penalty) since the last timing_enable."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        st = self._lib.tmop_timing_read(self._h, int(op), ctypes.byref(ms), ctypes.byref(n))
        if st < 0:
            raise TMOPError(st, "tmop_timing_read")
        return ms.value, n.value

    def newton_solve(self, x, **opts):
        """Optimizes x in place.  Keyword options are the fields of
        tmop_newton_opts; returns (status, report dict with per-iteration
        history lists F, gnorm, cg)."""
        _check_field(x, self.dim, self.n_node, "x")
        o = tmop_newton_opts()
        self._lib.tmop_newton_default_opts(ctypes.byref(o))
        for k, v in opts.items():
            if k.startswith("hist_") or not hasattr(o, k):
                raise ValueError(f"unknown Newton option {k}")
            setattr(o, k, v)
        n = o.max_it + 1
        hF = (ctypes.c_double * n)()
        hg = (ctypes.c_double * n)()
        hc = (ctypes.c_int32 * n)()
        ht = (ctypes.c_double * n)()
        o.hist_time = ctypes.cast(ht, ctypes.POINTER(ctypes.c_double))
        o.hist_F = ctypes.cast(hF, ctypes.POINTER(ctypes.c_double))
        o.hist_gnorm = ctypes.cast(hg, ctypes.POINTER(ctypes.c_double))
        o.hist_cg = ctypes.cast(hc, ctypes.POINTER(ctypes.c_int32))
        rep = tmop_newton_report()
        st = self._lib.tmop_newton_solve(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.byref(o), ctypes.byref(rep),
                                         _stream(x))
        if st < 0:
            raise TMOPError(st, "tmop_newton_solve")
        r = {k: getattr(rep, k) for k, _ in tmop_newton_report._fields_}
        k = r["iters"] + 1
        r.update(history_F=list(hF[:k]), history_gnorm=list(hg[:k]), history_cg=list(hc[:k]),
                 history_time=list(ht[:k]), status=st)
        return st, r


# C-ABI names, for callers that prefer the flat interface.
def tmop_setup(*args, **kw) -> Context:
    return Context(*args, **kw)


def tmop_energy(ctx: Context, x):
    return ctx.energy(x)


def tmop_gradient(ctx: Context, x, g=None):
    return ctx.gradient(x, g)


def tmop_energy_gradient(ctx: Context, x, g=None):
    return ctx.energy_gradient(x, g)


def tmop_hessian_apply(ctx: Context, x, v, Hv=None):
    return ctx.hessian_apply(x, v, Hv)


def tmop_hessian_diagonal(ctx: Context, x, diag=None):
    return ctx.hessian_diagonal(x, diag)


def tmop_newton_solve(ctx: Context, x, **opts):
    return ctx.newton_solve(x, **opts)


def tmop_destroy(ctx: Context):
    ctx.close()
