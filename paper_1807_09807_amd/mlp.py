"""Learned initial guess for the Newton solver (binding + pipeline).

The per-element network and its kernels live in the library
(tmop_mlp_*); this module marshals arguments and drives the pipeline:

  data      seeded 2D Q2 training meshes (random sinusoid + noise), each
            optimized by the library's own Newton solver; per element the
            features (nodes relative to the centroid, / h) and labels (the
            Newton displacement minus its element mean, / h)
  train     Adam on the mean squared error, mini-batches of consecutive
            samples taken in a seeded random order of mesh chunks
  evaluate  plain Newton from x0 against Newton from the proposal, the
            proposal accepted only if det A > 0 everywhere and F < F(x0)
            (otherwise plain Newton is the fallback); wall time includes
            the proposal
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np

from . import meshgen
from . import tmop as T

NPARAMS = 10706
LAYERS = ((18, 64), (64, 64), (64, 64), (64, 18))
_P = ctypes.c_void_p


def _bind(lib):
    if getattr(lib, "_mlp_bound", False):
        return lib
    lib.tmop_mlp_create.argtypes = [_P, ctypes.POINTER(_P)]
    lib.tmop_mlp_destroy.argtypes = [_P]
    lib.tmop_mlp_destroy.restype = None
    lib.tmop_mlp_get_params.argtypes = [_P, _P]
    lib.tmop_mlp_forward.argtypes = [_P, _P, _P, ctypes.c_int64, _P]
    lib.tmop_mlp_backward.argtypes = [_P, _P, _P, ctypes.c_int64, _P, _P, _P]
    lib.tmop_mlp_train_step.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_float, ctypes.POINTER(ctypes.c_double), _P]
    lib.tmop_mlp_features.argtypes = [_P, _P, _P, _P]
    lib.tmop_mlp_labels.argtypes = [_P, _P, _P, _P, _P]
    lib.tmop_mlp_propose.argtypes = [_P, _P, _P, _P, _P]
    for f in ("create", "get_params", "forward", "backward", "train_step", "features", "labels", "propose"):
        getattr(lib, f"tmop_mlp_{f}").restype = ctypes.c_int
    lib._mlp_bound = True
    return lib


def _check(st, what):
    if st < 0:
        raise T.TMOPError(st, what)
    return st


def _ptr(t):
    return _P(t.data_ptr())


def _stream(t):
    import torch
    return _P(torch.cuda.current_stream(t.device).cuda_stream)


def init_params(seed: int) -> np.ndarray:
    """Seeded initial parameters: W ~ U(-a, a), a = sqrt(6 / (k + n))
    (Glorot), biases 0; the output layer scaled by 0.1 so the untrained
    network proposes small displacements."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (k, n) in enumerate(LAYERS):
        a = np.sqrt(6.0 / (k + n)) * (0.1 if li == 3 else 1.0)
        parts.append(rng.uniform(-a, a, k * n))
        parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


class MLP:
    """Owns one tmop_mlp."""

    def __init__(self, params: np.ndarray):
        self._lib = _bind(T.load())
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != NPARAMS:
            raise ValueError(f"expected {NPARAMS} parameters")
        h = _P()
        _check(self._lib.tmop_mlp_create(p.ctypes.data_as(_P), ctypes.byref(h)), "tmop_mlp_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tmop_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(NPARAMS, np.float32)
        _check(self._lib.tmop_mlp_get_params(self._h, out.ctypes.data_as(_P)), "tmop_mlp_get_params")
        return out

    def forward(self, X, Y=None):
        import torch
        Y = torch.empty_like(X) if Y is None else Y
        _check(self._lib.tmop_mlp_forward(self._h, _ptr(X), _ptr(Y), X.shape[0], _stream(X)), "tmop_mlp_forward")
        return Y

    def backward(self, X, dY, want_dX=False):
        import torch
        dp = torch.empty(NPARAMS, dtype=torch.float32, device=X.device)
        dX = torch.empty_like(X) if want_dX else None
        _check(self._lib.tmop_mlp_backward(self._h, _ptr(X), _ptr(dY), X.shape[0], _ptr(dp),
                                           _ptr(dX) if want_dX else None, _stream(X)), "tmop_mlp_backward")
        return dp, dX

    def train_step(self, X, L, lr, want_loss=False):
        loss = ctypes.c_double()
        _check(self._lib.tmop_mlp_train_step(self._h, _ptr(X), _ptr(L), X.shape[0], ctypes.c_float(lr),
                                             ctypes.byref(loss) if want_loss else None, _stream(X)),
               "tmop_mlp_train_step")
        return loss.value if want_loss else None


def features(ctx: T.Context, x):
    import torch
    X = torch.empty((ctx.n_elem, 18), dtype=torch.float32, device=x.device)
    _check(_bind(T.load()).tmop_mlp_features(ctx.handle, _ptr(x), _ptr(X), _stream(x)), "tmop_mlp_features")
    return X


def labels(ctx: T.Context, x, xstar, out=None):
    import torch
    L = torch.empty((ctx.n_elem, 18), dtype=torch.float32, device=x.device) if out is None else out
    _check(_bind(T.load()).tmop_mlp_labels(ctx.handle, _ptr(x), _ptr(xstar), _ptr(L), _stream(x)), "tmop_mlp_labels")
    return L


def propose(ctx: T.Context, mlp: MLP, x, out=None):
    import torch
    xo = torch.empty_like(x) if out is None else out
    _check(_bind(T.load()).tmop_mlp_propose(ctx.handle, mlp.handle, _ptr(x), _ptr(xo), _stream(x)),
           "tmop_mlp_propose")
    return xo


# ----------------------------------------------------------------------------- pipeline

NEWTON_OPTS = dict(max_it=300, rtol=1e-10, cg_forcing=1)
EVAL_OPTS = NEWTON_OPTS


@dataclass
class TrainingData:
    X: object            # torch float32 (n, 18)
    L: object
    n_mesh: int
    per_mesh: int
    info: dict = field(default_factory=dict)


def _valid_by_library(ctx):
    import torch

    def bad(x, elems):
        _, md, st = ctx.energy(torch.from_numpy(x).cuda())
        return np.array([0]) if st != T.TMOP_OK else np.array([], dtype=np.int64)
    return bad


def box_context(n: int, precision=T.TMOP_FP64):
    mesh = meshgen.box_mesh(2, n, 2)
    ctx = T.Context(2, 2, mesh.elem_node, mesh.n_node, 4, T.TMOP_MU2, mesh.h * np.eye(2), fixed=mesh.fixed,
                    precision=precision)
    return mesh, ctx


def union_context(n: int, copies: int, precision=T.TMOP_FP64):
    """One context for `copies` disjoint n x n Q2 meshes (node ids of copy k
    offset by k n_node): the objective is the sum of the copies' objectives,
    so one Newton solve optimizes all of them with full-size launches."""
    mesh = meshgen.box_mesh(2, n, 2)
    en = np.concatenate([mesh.elem_node + k * mesh.n_node for k in range(copies)])
    fixed = np.tile(mesh.fixed, (1, copies))
    ctx = T.Context(2, 2, en, copies * mesh.n_node, 4, T.TMOP_MU2, mesh.h * np.eye(2), fixed=fixed,
                    precision=precision)
    return mesh, ctx


def generate_training_data(n_mesh: int = 2000, n: int = 64, seed0: int = 1000, batch: int = 125,
                           log=None) -> TrainingData:
    """Features and labels of n_mesh seeded n x n Q2 mu_2 meshes (seeds
    seed0, seed0 + 1, ...); labels from the library's Newton solution,
    solved `batch` meshes at a time on a union context."""
    import torch
    mesh, one = box_context(n)
    ne, nn = mesh.n_elem, mesh.n_node
    X = torch.empty((n_mesh * ne, 18), dtype=torch.float32, device="cuda")
    L = torch.empty_like(X)
    bad = _valid_by_library(one)
    ctxs = {}
    t0 = time.perf_counter()
    iters, cg, statuses, grel = 0, 0, [], []
    for k0 in range(0, n_mesh, batch):
        b = min(batch, n_mesh - k0)
        if b not in ctxs:
            ctxs[b] = union_context(n, b)[1]
        ctx = ctxs[b]
        xs_host = [meshgen.training_mesh(n, seed0 + k0 + j, bad_elements=bad).x for j in range(b)]
        x0 = torch.from_numpy(np.concatenate(xs_host, axis=1)).cuda()
        xs = x0.clone()
        st, rep = ctx.newton_solve(xs, **NEWTON_OPTS)
        iters += rep["iters"]
        cg += rep["cg_iters"]
        statuses.append(st)
        grel.append(rep["gnorm"] / rep["gnorm0"])
        sl = slice(k0 * ne, (k0 + b) * ne)
        _check(_bind(T.load()).tmop_mlp_features(ctx.handle, _ptr(x0), _ptr(X[sl]), _stream(x0)), "features")
        labels(ctx, x0, xs, out=L[sl])
        if log:
            log(f"  training data: {k0 + b}/{n_mesh} meshes ({b * nn} nodes per solve, status {st}, "
                f"{rep['iters']} it, {rep['cg_iters']} CG), {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    return TrainingData(X, L, n_mesh, ne, dict(seconds=time.perf_counter() - t0, newton_iters=iters, cg_iters=cg,
                                               batch=batch, newton_status=statuses,
                                               max_rel_gnorm=max(grel)))


def train(data: TrainingData, epochs: int = 4, batch_meshes: int = 2, lr: float = 1e-3, seed: int = 0,
          params=None, log=None):
    """Adam over mini-batches of `batch_meshes` consecutive meshes' samples,
    in a seeded random order each epoch; lr decays by half per epoch."""
    import torch
    mlp = MLP(init_params(seed) if params is None else params)
    rng = np.random.default_rng(seed + 1)
    nb = data.n_mesh // batch_meshes
    B = batch_meshes * data.per_mesh
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(nb)
        for j, b in enumerate(order):
            sl = slice(int(b) * B, int(b) * B + B)
            want = j == len(order) - 1
            loss = mlp.train_step(data.X[sl], data.L[sl], lr * 0.5 ** ep, want_loss=want)
            if want:
                hist.append(loss)
        if log:
            log(f"  epoch {ep}: last-batch loss {hist[-1]:.4e}")
    torch.cuda.synchronize()
    return mlp, dict(seconds=time.perf_counter() - t0, loss_history=hist, steps=epochs * nb, batch=B)


def evaluate(mlp, n: int = 512, seeds=(10000,), precision=T.TMOP_FP64, log=None):
    """Plain Newton from x0 against learned-guess Newton, per seed: wall
    seconds and iterations to F_tol = F_ref + 1e-8 F0 (F_ref: final F of
    plain Newton run to its relative gradient tolerance; the row records
    whether that reference converged).  Plain Newton from x0 is the
    fallback, both when the proposal is unusable (inverted or not below
    F0) and when Newton from the proposal does not reach F_tol; the
    fallback's time counts against the learned run."""
    import torch
    mesh, ctx = box_context(n, precision)
    bad = _valid_by_library(ctx)
    rows = []
    for sd in seeds:
        tm = meshgen.training_mesh(n, sd, bad_elements=bad)
        x0 = torch.from_numpy(tm.x).cuda()
        # reference: plain Newton to the relative tolerance
        xr = x0.clone()
        st_ref, ref = ctx.newton_solve(xr, **EVAL_OPTS)
        F0 = ref["F0"]
        F_tol = ref["F"] + 1e-8 * F0
        # plain Newton to F_tol
        xp = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_p, rp = ctx.newton_solve(xp, ftarget=F_tol, **EVAL_OPTS)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        # learned: propose, check, Newton (fallback to x0)
        xl = torch.empty_like(x0) if mlp is not None else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        used = False
        if mlp is not None:
            propose(ctx, mlp, x0, xl)
            Fm, md, stm = ctx.energy(xl)
            used = stm == T.TMOP_OK and md > 0 and Fm < F0
        xs = xl if used else x0.clone()
        st_l, rl = ctx.newton_solve(xs, ftarget=F_tol, **EVAL_OPTS)
        # a learned start that does not reach F_tol falls back to plain Newton
        # from x0, whose time is added to the learned run's
        fell_back = used and (st_l != T.TMOP_OK or not rl["F"] <= F_tol)
        iters_l, cg_l = rl["iters"], rl["cg_iters"]
        if fell_back:
            xs = x0.clone()
            st_l, rl = ctx.newton_solve(xs, ftarget=F_tol, **EVAL_OPTS)
            iters_l += rl["iters"]
            cg_l += rl["cg_iters"]
        torch.cuda.synchronize()
        t_learn = time.perf_counter() - t0
        row = dict(seed=sd, F0=F0, F_tol=F_tol, F_proposal=Fm if mlp is not None else None, used_proposal=used,
                   reference=dict(iters=ref["iters"], F=ref["F"], status=st_ref, converged=st_ref == T.TMOP_OK),
                   plain=dict(iters=rp["iters"], cg=rp["cg_iters"], wall_s=t_plain, F=rp["F"], status=st_p,
                              reached_F_tol=bool(rp["F"] <= F_tol)),
                   learned=dict(iters=iters_l, cg=cg_l, wall_s=t_learn, F=rl["F"], status=st_l,
                                reached_F_tol=bool(rl["F"] <= F_tol), fell_back_after_solve=fell_back))
        rows.append(row)
        if log:
            kind = "(proposal used, then fallback) " if fell_back else "(proposal used) " if used else "(fallback) "
            log(f"  eval seed {sd}: reference {ref['iters']} it (status {st_ref}); plain {rp['iters']} it / "
                f"{rp['cg_iters']} CG / {t_plain:.3f} s; learned {kind}{iters_l} it / {cg_l} CG / "
                f"{t_learn:.3f} s; F0 {F0:.4e} -> proposal {row['F_proposal']}")
    return rows
