"""Sequential strict LPA that also records the learned gate's training samples
(test infrastructure only; pure Python, for graphs of a few thousand vertices).

The label update is Algorithm 1 (Section 4.2) with the strict rule of Eq. (2)
and the smallest-label tie rule (Section 2), vertex pruning as in Section
4.1.4, in an explicit vertex order, exactly as ``lpa_oracle.c`` does.  On top
of it, every processing of a vertex v in sweep s stores

  s0 = log2(1 + deg v)         (deg: stored entries of row v)
  s1 = (W1 - W2) / K_v         (W1 >= W2 the two largest label weights, 0 if absent)
  s2 = W(C_v before the update) / K_v
  s3 = 1 if the label changed now, else 0
  s4 = W1 / K_v
  s5 = distinct neighbour labels / deg v

(K_v the summed weights of row v; a zero K or deg gives 0; a vertex whose
only entries are self-loops is processed with W1 = W2 = 0 and keeps its
label), and the sample
of that processing, when v was processed before in an earlier sweep s', is
the decision vector
  (s0, s1, s2, s3 of sweep s', s / max_iters, s4, s5, min(s - s', 8) / 8)
with target 1 iff the label changes in this processing.
"""
from __future__ import annotations

import math

import numpy as np


def lpa_trace(g, order=None, tau: float = 0.05, max_iters: int = 20, prune: bool = True):
    """Returns dict(labels, changed per sweep, iterations, X [S, 8] float64, y [S] uint8, sweep [S])."""
    n = int(g.n)
    off = np.asarray(g.offsets, dtype=np.int64)
    idx = np.asarray(g.indices, dtype=np.int64)
    w = np.ones(len(idx), np.int64) if g.weights is None else np.asarray(g.weights, dtype=np.float64).astype(np.int64)
    order = list(range(n)) if order is None else [int(v) for v in order]
    C = list(range(n))
    F = [1] * n
    lastp = [-1] * n
    stored = [None] * n
    K = [int(w[off[v]:off[v + 1]].sum()) for v in range(n)]
    X, Y, S = [], [], []
    changed_per_sweep = []
    iterations = 0
    for s in range(max_iters):
        dN = 0
        for v in order:
            if prune and not F[v]:
                continue
            F[v] = 0
            W = {}
            for e in range(off[v], off[v + 1]):
                j = int(idx[e])
                if j == v:
                    continue
                W[C[j]] = W.get(C[j], 0) + int(w[e])
            deg = int(off[v + 1] - off[v])
            was = C[v]
            if W:
                best_w = max(W.values())
                best = min(c for c, x in W.items() if x == best_w)
            else:
                best = was  # no neighbour besides itself: the label stays
            ch = best != was
            if lastp[v] >= 0 and lastp[v] < s:
                st = stored[v]
                X.append([st[0], st[1], st[2], st[3], s / max_iters, st[4], st[5], min(s - lastp[v], 8) / 8.0])
                Y.append(1 if ch else 0)
                S.append(s)
            ws = sorted(W.values(), reverse=True) + [0, 0]
            w1, w2 = ws[0], ws[1]
            inv = 1.0 / K[v] if K[v] else 0.0
            stored[v] = (math.log2(1 + deg), (w1 - w2) * inv, W.get(was, 0) * inv, 1.0 if ch else 0.0, w1 * inv,
                         len(W) / deg if deg else 0.0)
            lastp[v] = s
            if ch:
                C[v] = best
                dN += 1
                if prune:
                    for e in range(off[v], off[v + 1]):
                        j = int(idx[e])
                        if j != v:
                            F[j] = 1
        changed_per_sweep.append(dN)
        iterations = s + 1
        if dN / n <= tau:
            break
    return dict(labels=np.array(C, np.int32), changed=np.array(changed_per_sweep, np.int64), iterations=iterations,
                X=np.array(X, np.float64).reshape(-1, 8), y=np.array(Y, np.uint8), sweep=np.array(S, np.int64))
