"""Plain CPU oracle of the derivative-free TMOP solver.  TEST
INFRASTRUCTURE ONLY: imported by the test suite alone; the GPU library
shares no code with it.

Section 3.4 (eq. 3.3, variational form): every node x_i in turn moves to
the position that minimizes its local patch quality

    Q(x_i) = sum over the elements E holding node i of
             sum_q w_q det W mu(A W^{-1})          (eq. 2.4 restricted to E),

found by the Nelder-Mead simplex method; the sweeps over the nodes stop
when no node moved more than t in a sweep (max_k |x_k^{m+1} - x_k^m| < t).

Readings where the paper is silent:
* node order: by colour, where no two nodes of a colour share an element
  (greedy colouring in node order: each node takes the smallest colour not
  used by a node it shares an element with), and by node index within a
  colour.  Nodes of one colour have disjoint patches, so visiting them one
  after the other (Gauss-Seidel) gives the same result as moving them all
  at once, which is what makes the method parallel;
* |.| in the stopping rule: the max norm over the node's components;
* Q = +inf when det A <= 0 at a patch point (positivity, Section 3.4);
* only the free components of a node move (fixed or sliding boundaries);
* Nelder-Mead as stated by Lagarias, Reeds, Wright and Wright (SIAM J.
  Optim. 9, 1998) with the standard coefficients (reflection 1, expansion
  2, contraction 1/2, shrink 1/2), the initial simplex x_i, x_i + s e_k
  (s = step times the target size (det W)^(1/d)), stopped when every vertex
  lies within xtol of the best one (max norm) or after max_evals
  evaluations; the best vertex is the new position.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from oracle import tmop_oracle as O


def node_colouring(elem_node, n_node):
    """Greedy colouring of the nodes in index order: node I takes the
    smallest colour not used by a node that shares an element with it.
    Returns the list of colours, each the ascending array of its nodes."""
    elem_node = np.asarray(elem_node)
    node_elems = [[] for _ in range(n_node)]
    for e, nodes in enumerate(elem_node):
        for I in nodes:
            node_elems[I].append(e)
    colour = np.full(n_node, -1, dtype=np.int64)
    for I in range(n_node):
        used = set()
        for e in node_elems[I]:
            for J in elem_node[e]:
                if colour[J] >= 0:
                    used.add(int(colour[J]))
        c = 0
        while c in used:
            c += 1
        colour[I] = c
    return [np.flatnonzero(colour == c) for c in range(int(colour.max()) + 1)]


def nelder_mead(f, x0, step, xtol, max_evals):
    """Minimize f over R^n from the simplex x0, x0 + step e_k (Lagarias et
    al. 1998).  Returns (best vertex, its value, evaluations)."""
    n = x0.size
    V = [np.array(x0, dtype=np.float64)]
    for k in range(n):
        v = V[0].copy()
        v[k] += step
        V.append(v)
    fv = [f(v) for v in V]
    evals = n + 1
    while True:
        order = sorted(range(n + 1), key=lambda k: fv[k])          # stable: ties keep their place
        V = [V[k] for k in order]
        fv = [fv[k] for k in order]
        if max(float(np.max(np.abs(V[k] - V[0]))) for k in range(1, n + 1)) <= xtol or evals >= max_evals:
            return V[0], fv[0], evals
        xb = sum(V[:n]) / n                                         # centroid of the n best
        xr = xb + (xb - V[n])
        fr = f(xr)
        evals += 1
        if fv[0] <= fr < fv[n - 1]:
            V[n], fv[n] = xr, fr
            continue
        if fr < fv[0]:
            xe = xb + 2.0 * (xr - xb)
            fe = f(xe)
            evals += 1
            V[n], fv[n] = (xe, fe) if fe < fr else (xr, fr)
            continue
        if fr < fv[n]:                                              # outside contraction
            xc = xb + 0.5 * (xr - xb)
            fc = f(xc)
            evals += 1
            if fc <= fr:
                V[n], fv[n] = xc, fc
                continue
        else:                                                       # inside contraction
            xc = xb + 0.5 * (V[n] - xb)
            fc = f(xc)
            evals += 1
            if fc < fv[n]:
                V[n], fv[n] = xc, fc
                continue
        for k in range(1, n + 1):                                   # shrink towards the best vertex
            V[k] = V[0] + 0.5 * (V[k] - V[0])
            fv[k] = f(V[k])
        evals += n


@dataclass
class DfoOptions:
    t: float = 1e-5              # sweep tolerance (Section 3.4: 1e-5 for unit volume)
    max_sweeps: int = 100
    step: float = 0.1            # initial simplex edge, in units of the target size
    xtol: float = 1e-6           # Nelder-Mead simplex size at which a node stops
    max_evals: int = 200         # Nelder-Mead evaluations per node and sweep


@dataclass
class DfoReport:
    sweeps: int = 0
    converged: bool = False
    F0: float = 0.0
    F: float = 0.0
    max_move: list = field(default_factory=list)     # per sweep


class Patches:
    """Node -> elements adjacency of a Problem, and the patch quality Q of
    eq. 3.3 (variational form)."""

    def __init__(self, prob: O.Problem, n_node):
        self.prob = prob
        self.elems = [[] for _ in range(n_node)]
        for e, nodes in enumerate(prob.elem_node):
            for I in nodes:
                self.elems[I].append(e)
        self.elems = [np.array(sorted(set(l)), dtype=np.int64) for l in self.elems]

    def quality(self, x, i):
        """Q(x_i) = sum over i's elements of sum_q w_q det W mu(T); +inf when
        det A <= 0 at one of their points."""
        c, detA = self.prob.pointwise(x, elems=self.elems[i])
        if np.any(detA <= 0.0):
            return math.inf
        return math.fsum(c.ravel())


def dfo_sweep(prob, patches, x, free, colours, opts):
    """One sweep over all nodes, colour by colour.  x (d, n_node) is updated
    in place; free (d, n_node) marks the movable components.  Returns the
    largest max-norm move of a node."""
    if np.ndim(prob.detW) != 0:
        raise ValueError("the derivative-free solver takes a constant target")
    h = float(prob.detW) ** (1.0 / prob.dim)                       # target size
    move = 0.0
    for nodes in colours:
        for i in nodes:
            comps = np.flatnonzero(free[:, i])
            if comps.size == 0:
                continue
            x_old = x[:, i].copy()

            def f(y):
                x[comps, i] = y
                return patches.quality(x, i)

            best, _, _ = nelder_mead(f, x_old[comps], opts.step * h, opts.xtol, opts.max_evals)
            x[:, i] = x_old
            x[comps, i] = best
            move = max(move, float(np.max(np.abs(x[:, i] - x_old))))
    return move


def dfo_solve(prob, x0, fixed, n_node, opts: DfoOptions = DfoOptions()):
    """Sweeps until no node moves more than t (Section 3.4) or max_sweeps."""
    x = np.array(x0, dtype=np.float64)
    free = 1 - np.asarray(fixed, dtype=np.int64)
    colours = node_colouring(prob.elem_node, n_node)
    patches = Patches(prob, n_node)
    rep = DfoReport(F0=prob.energy(x)[0])
    for _ in range(opts.max_sweeps):
        m = dfo_sweep(prob, patches, x, free, colours, opts)
        rep.sweeps += 1
        rep.max_move.append(m)
        if m < opts.t:
            rep.converged = True
            break
    rep.F = prob.energy(x)[0]
    return x, rep
