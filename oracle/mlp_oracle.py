"""FP64 numpy oracle of the learned initial guess.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this module; the GPU library shares no code with it.

The per-element network maps the 9 nodes of a Q2 quadrilateral, relative
to the element centroid and divided by the target size h, to a displacement
of the same 9 nodes (in units of h):
    18 -> 64 -> 64 -> 64 -> 18, GELU(z) = z Phi(z) after the three hidden
    layers, no activation on the output.
Feature / output index: c * 9 + i (component c, local node i = i0 + 3 i1).
Weights take BF16 values (rounded to nearest even from the FP32 master
copy); biases stay FP32; every product and sum here is exact FP64.

The proposal merges the per-element displacements at shared nodes by
averaging over the elements that contain the node, and leaves fixed DOFs
alone.  The label of an element is its Newton-optimized displacement minus
the displacement's element mean: a per-element network cannot observe a
rigid translation of the element.
"""
from __future__ import annotations

import math

import numpy as np

LAYERS = ((18, 64), (64, 64), (64, 64), (64, 18))
N_PARAMS = sum(k * n + n for k, n in LAYERS)          # 10706


def unpack(theta):
    """Flat parameter vector -> [(W (k x n), b (n)), ...] in layer order."""
    out, o = [], 0
    for k, n in LAYERS:
        W = theta[o:o + k * n].reshape(k, n)
        o += k * n
        b = theta[o:o + n]
        o += n
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def bf16_round(a):
    """Round FP32 values to the nearest BF16 value (ties to even), returned
    as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _erf(z):
    if np.iscomplexobj(z):
        from scipy.special import erf
        return erf(z)
    return np.vectorize(math.erf, otypes=[np.float64])(z) if np.ndim(z) else math.erf(z)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    """d/dz z Phi(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def effective_layers(theta_master):
    """The layers the network computes with: BF16 weights, FP32 biases."""
    return [(bf16_round(W), np.asarray(b, dtype=np.float32).astype(np.float64))
            for W, b in unpack(np.asarray(theta_master, dtype=np.float32))]


def forward_layers(layers, X):
    """Y for explicit layers [(W, b), ...]; returns (Y, cache)."""
    H = np.asarray(X, dtype=np.float64)
    Zs, Hs = [], [H]
    for li, (W, b) in enumerate(layers):
        Z = H @ W + b
        if li < 3:
            Zs.append(Z)
            H = gelu(Z)
            Hs.append(H)
        else:
            H = Z
    return H, (Zs, Hs)


def backward_layers(layers, cache, dY):
    """Gradients [(dW, db), ...] of sum(dY * Y) w.r.t. the layers, and w.r.t. X."""
    Zs, Hs = cache
    grads = [None] * 4
    dZ = np.asarray(dY, dtype=np.float64)
    dX = None
    for li in range(3, -1, -1):
        W, _ = layers[li]
        grads[li] = (Hs[li].T @ dZ, dZ.sum(axis=0))
        dH = dZ @ W.T
        if li > 0:
            dZ = dH * gelu_prime(Zs[li - 1])
        else:
            dX = dH
    return grads, dX


def forward(theta_master, X):
    """Y = MLP(X) for X (n, 18) with the BF16-valued weights of theta."""
    return forward_layers(effective_layers(theta_master), X)


def backward(theta_master, cache, dY):
    """Flat gradient (theta layout, taken through the BF16-valued weights)
    of sum(dY * Y), and dL/dX."""
    grads, dX = backward_layers(effective_layers(theta_master), cache, dY)
    return pack(grads), dX


def mse_grad(Y, L):
    """loss = mean over samples and outputs of (Y - L)^2; returns (loss, dY)."""
    n = Y.shape[0] * Y.shape[1]
    D = Y - L
    return float(np.sum(D * D) / n), 2.0 * D / n


def adam_step(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction, step t >= 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(x, elem_node, h):
    """(x_E - centroid_E) / h, shape (n_elem, 18), index c * 9 + i."""
    X = x[:, elem_node]                                   # (2, ne, 9)
    X = (X - X.mean(axis=2, keepdims=True)) / h
    return np.transpose(X, (1, 0, 2)).reshape(-1, 18)


def labels(x, xstar, elem_node, h):
    """((x*_E - x_E) - its element mean) / h, shape (n_elem, 18)."""
    D = (xstar - x)[:, elem_node]
    D = (D - D.mean(axis=2, keepdims=True)) / h
    return np.transpose(D, (1, 0, 2)).reshape(-1, 18)


def propose(x, Y, elem_node, h, fixed):
    """x + h * (average over the elements containing each node of the
    element's predicted displacement); fixed DOFs keep their value."""
    n_node = x.shape[1]
    acc = np.zeros_like(x)
    cnt = np.zeros(n_node)
    Yr = np.asarray(Y, dtype=np.float64).reshape(-1, 2, 9)
    for c in range(2):
        np.add.at(acc[c], elem_node, Yr[:, c, :])
    np.add.at(cnt, elem_node, 1.0)
    out = x.copy()
    free = ~np.asarray(fixed, dtype=bool)
    upd = x + h * acc / np.maximum(cnt, 1.0)[None, :]
    out[free] = upd[free]
    return out
