"""Learned active-set gate: sample collection, training and threshold choice.

Host orchestration only.  The samples come from traced runs of the library
(``LPA_FLAG_TRACE``: for a re-processed vertex, the features it carried into
the decision and whether its label then changed), the network is trained by
the library's own forward/backward/Adam kernels (``lpa_gate_train``) and the
threshold is the largest one that keeps a given recall of label changes on
held-out samples (``lpa_gate_threshold``).  A gated run skips the flagged
vertices the network rates below the threshold (they stay flagged), which
narrows the frontier that vertex pruning (Section 4.1.4) leaves.
"""
from __future__ import annotations

import numpy as np

from . import abi


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights for the ReLU layers, zero biases (float32[1377])."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((8, 32), (32, 32), (32, 1)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, (fan_out, fan_in)).astype(np.float32).ravel())
        parts.append(np.zeros(fan_out, np.float32))
    p = np.concatenate(parts)
    assert p.shape == (abi.GATE_PARAMS,)
    return p


def collect(graphs, probability: float = 0.25, capacity: int = 1 << 22, tau: float = 0.05, max_iters: int = 20,
            mode: int = abi.LPA_MODE_ASYNC, schedule=None, bins=None):
    """Traces plain pruned runs of every CSR in ``graphs``; returns (X float32[S][8], y uint8[S]).

    ``schedule``: asynchronous schedule (early steps, early sweeps, late steps)
    of the traced runs, best that of the runs the gate will serve (the label
    dynamics, hence what the features predict, depend on it); "tuned" lets
    ``lpa_autotune`` pick it (and the bin limits) per graph, as for tuned
    handles; None keeps the library's default.  ``bins``: degree limits of
    the bins for the traced runs (they change the processing order too)."""
    xs, ys = [], []
    for csr in graphs:
        G = abi.LPAGraph(csr)
        if schedule == "tuned":
            G.autotune(tau, max_iters, mode)
        elif schedule is not None:
            G.set_async_schedule(*schedule)
        if bins is not None and schedule != "tuned":
            G.set_bins(list(bins))
        G.set_trace(capacity, probability)
        G.run(tau, max_iters, mode, True, flags=abi.LPA_FLAG_TRACE)
        x, y = G.gate_trace()
        G.close()
        xs.append(x)
        ys.append(y)
    return np.concatenate(xs), np.concatenate(ys)


def train(X, y, epochs: int = 4, batch: int = 4096, lr: float = 1e-3, holdout: float = 0.1, recall: float = 0.98,
          seed: int = 0, params=None, device: int = 0) -> dict:
    """Trains on a random (1 - holdout) share of the samples with pos_weight =
    #negatives / #positives and picks the threshold on the rest.

    Returns dict(params, threshold, pos_weight, losses, holdout_recall,
    holdout_skip): the share of held-out changes kept, and of held-out samples
    the gate would skip.
    """
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(y))
    nh = int(round(holdout * len(y)))
    tr, ho = perm[nh:], perm[:nh]
    Xt, yt = np.ascontiguousarray(X[tr]), np.ascontiguousarray(y[tr])
    npos = int(yt.sum())
    pw = float((len(yt) - npos) / max(npos, 1))
    p0 = init_params(seed) if params is None else np.asarray(params, np.float32)
    order = None
    if len(yt) * epochs <= (1 << 28):
        order = np.concatenate([rng.permutation(len(yt)) for _ in range(epochs)]).astype(np.int64)
    params, losses = abi.gate_train(p0, Xt, yt, epochs, batch, lr=lr, pos_weight=pw, order=order, device=device)
    Xh, yh = np.ascontiguousarray(X[ho]), np.ascontiguousarray(y[ho])
    thr = abi.gate_threshold(params, Xh, yh, recall, device=device) if nh else 0.5
    info = dict(params=params, threshold=float(thr), pos_weight=pw, losses=losses)
    if nh:
        p = abi.gate_forward(params, Xh, device=device)
        keep = p >= thr
        info["holdout_recall"] = float(keep[yh == 1].mean()) if (yh == 1).any() else 1.0
        info["holdout_skip"] = float(1.0 - keep.mean())
    return info
