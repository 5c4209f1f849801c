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


def _logit_fp64(theta_bf16, x):
    """Logit z of the gate network (ReLU, ReLU, linear) in FP64 at the given weights."""
    from . import mlp
    P = mlp.unpack(theta_bf16)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 8)
    h1 = np.maximum(x @ P["W1"].T + P["b1"], 0.0)
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0.0)
    return (h2 @ P["W3"].T)[:, 0] + P["b3"][0]


def lpa_gated(g, params, threshold: float, order=None, tau: float = 0.05, max_iters: int = 20):
    """The gated method, sequentially, in an explicit vertex order.

    Algorithm 1 (Section 4.2) with vertex pruning (Section 4.1.4), plus the
    learned active-set gate as the library defines it:

    * at the start of every sweep s >= 1, each vertex that is flagged then
      and was processed in an earlier sweep gets a decision from the network
      evaluated (FP64) at the bf16 rounding of ``params`` on its decision
      features (see ``lpa_trace``): it is skipped in this sweep when
      p < threshold, i.e. when its logit is below log(t / (1 - t)); a skipped
      vertex keeps its flag and its stored features;
    * vertices flagged later in the sweep, or never processed, are not gated;
    * after the main loop (stop test dN/N <= tau, or max_iters sweeps) one
      verification sweep runs with the gate off over the flagged vertices; if
      it changes more than tau * N labels, plain pruned sweeps continue (gate
      off; the sweep cap grows by max_iters and counts the verification
      sweep, at most max_iters more sweeps) and a second verification sweep
      follows.

    Returns dict(labels, changed, processed, scanned, gated (per counted
    sweep), iterations, converged, verify_changed, verify_scanned, verified,
    margin = the smallest |logit - log(t / (1 - t))| over all decisions taken
    (inf when none)).
    """
    from . import mlp
    n = int(g.n)
    off = np.asarray(g.offsets, dtype=np.int64)
    idx = np.asarray(g.indices, dtype=np.int64)
    w = np.ones(len(idx), np.int64) if g.weights is None else np.asarray(g.weights, dtype=np.float64).astype(np.int64)
    order = list(range(n)) if order is None else [int(v) for v in order]
    theta = mlp.bf16_round(np.asarray(params, np.float32))
    if threshold <= 0.0:
        z = -math.inf
    elif threshold >= 1.0:
        z = math.inf
    else:
        z = math.log(threshold / (1.0 - threshold))
    C = list(range(n))
    F = [1 if off[v + 1] > off[v] else 0 for v in range(n)]  # vertices without entries are never listed
    lastp = [-1] * n
    stored = [None] * n
    K = [int(w[off[v]:off[v + 1]].sum()) for v in range(n)]
    out = dict(changed=[], processed=[], scanned=[], gated=[], verify_changed=0, verify_scanned=0)
    margin = math.inf

    def process(v, s, record):
        """One processing of flagged vertex v (flag already cleared); returns 1 if its label changed."""
        W = {}
        for e in range(off[v], off[v + 1]):
            j = int(idx[e])
            if j == v:
                continue
            W[C[j]] = W.get(C[j], 0) + int(w[e])
        was = C[v]
        best = was
        if W:
            bw = max(W.values())
            best = min(c for c, x in W.items() if x == bw)
        ch = best != was
        if record:
            deg = int(off[v + 1] - off[v])
            ws = sorted(W.values(), reverse=True) + [0, 0]
            inv = 1.0 / K[v] if K[v] else 0.0
            stored[v] = (math.log2(1 + deg), (ws[0] - ws[1]) * inv, W.get(was, 0) * inv, 1.0 if ch else 0.0,
                         ws[0] * inv, len(W) / deg if deg else 0.0)
            lastp[v] = s
        if ch:
            C[v] = best
            for e in range(off[v], off[v + 1]):
                j = int(idx[e])
                if j != v:
                    F[j] = 1
        return 1 if ch else 0

    def sweep(s, skip, record):
        dn = proc = scan = gated = 0
        for v in order:
            if not F[v]:
                continue
            if skip is not None and skip[v]:
                gated += 1
                continue
            F[v] = 0
            proc += 1
            scan += int(off[v + 1] - off[v])
            dn += process(v, s, record)
        return dn, proc, scan, gated

    def count(res):
        dn, proc, scan, gated = res
        out["changed"].append(dn)
        out["processed"].append(proc)
        out["scanned"].append(scan)
        out["gated"].append(gated)
        return dn

    converged = False
    sweep_no = 0     # every sweep, verification included (the library's sweep counter)
    cap = max_iters  # the library's sweep cap (grows by max_iters for a fallback)
    for s in range(max_iters):
        skip = None
        if s >= 1:
            cand = [v for v in range(n) if F[v] and lastp[v] >= 0]
            skip = [False] * n
            if cand:
                X = []
                for v in cand:
                    st = stored[v]
                    X.append([st[0], st[1], st[2], st[3], s / max_iters, st[4], st[5], min(s - lastp[v], 8) / 8.0])
                zl = _logit_fp64(theta, X)
                for v, lz in zip(cand, zl):
                    skip[v] = bool(lz < z)
                    if math.isfinite(z):
                        margin = min(margin, abs(float(lz) - z))
        dn = count(sweep(s, skip, True))
        sweep_no += 1
        if dn / n <= tau:
            converged = True
            break
    verified = False
    if max_iters > 0:
        for attempt in range(2):
            dn, _, scan, _ = sweep(sweep_no, None, False)
            sweep_no += 1
            out["verify_changed"] += dn
            out["verify_scanned"] += scan
            verified = dn / n <= tau
            if verified or attempt == 1:
                break
            cap += max_iters
            for _ in range(max_iters):
                dn = count(sweep(sweep_no, None, False))
                sweep_no += 1
                if dn / n <= tau:
                    converged = True
                    break
                if sweep_no >= cap:
                    break
    return dict(labels=np.array(C, np.int32), changed=np.array(out["changed"], np.int64),
                processed=np.array(out["processed"], np.int64), scanned=np.array(out["scanned"], np.int64),
                gated=np.array(out["gated"], np.int64), iterations=len(out["changed"]), converged=converged,
                verify_changed=out["verify_changed"], verify_scanned=out["verify_scanned"], verified=verified,
                margin=margin)
