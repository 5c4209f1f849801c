"""CPU oracle for strict label propagation (GVE-LPA, arXiv 2312.08140).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product library never
calls it and shares no code with it.

* ``lpa``          Algorithm 1 (Section 4.2) executed sequentially in an
                   explicit vertex order (C, ``lpa_oracle.c``), strict or
                   non-strict (Section 4.1.5; ``TIE_A``, ``TIE_P``).
* ``color``        greedy colouring in decreasing (degree, hash, id) priority; with
                   ``color_order`` it fixes the order of the deterministic mode.
* ``modularity``   Eq. (1), community form, exact integers + one FP64 division.
* ``nmi``          normalised mutual information (``metrics.py``).
* ``mlp``          FP64 forward/backward/Adam of the 8-32-32-1 gate (``mlp.py``).
"""
from __future__ import annotations

import ctypes
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

import numpy as np

from . import build as _build
from .metrics import nmi  # noqa: F401

MAX_STATS = 64
# Non-strict tie rule: among the labels of maximum weight, vertex v takes the
# label c of smallest rank ((c + 1) * TIE_A^(1 + v mod 64)) mod TIE_P (lpa_oracle.c)
TIE_P = 2147483647
TIE_A = 1580030173
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _build.LIB.exists():
            _build.build()
        lib = ctypes.CDLL(str(_build.LIB))
        vp = ctypes.c_void_p
        lib.oracle_lpa.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int]
        lib.oracle_lpa.restype = ctypes.c_int
        lib.oracle_color.argtypes = [ctypes.c_int64, vp, vp, ctypes.c_uint32, vp]
        lib.oracle_color.restype = ctypes.c_int64
        lib.oracle_color_order.argtypes = [ctypes.c_int64, vp, ctypes.c_int64, vp]
        lib.oracle_modularity.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _csr_arrays(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.float32)
    return off, idx, w


def lpa(g, order=None, tau: float = 0.05, max_iters: int = 20, prune: bool = True, init_labels=None,
        init_flags=None, strict: bool = True) -> dict:
    """Strict (or, with ``strict=False``, non-strict) LPA on CSR ``g``
    (attributes n, offsets, indices, weights).

    Returns a dict with ``labels``, ``flags``, per-sweep ``changed``,
    ``processed``, ``scanned`` (length = iterations, capped at 64),
    ``iterations`` and ``converged``.
    """
    lib = _load()
    n = int(g.n)
    off, idx, w = _csr_arrays(g)
    order = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    il = None if init_labels is None else np.ascontiguousarray(init_labels, dtype=np.int32)
    ifl = None if init_flags is None else np.ascontiguousarray(init_flags, dtype=np.uint8)
    labels = np.empty(max(n, 1), np.int32)
    flags = np.empty(max(n, 1), np.uint8)
    changed = np.zeros(MAX_STATS, np.int64)
    processed = np.zeros(MAX_STATS, np.int64)
    scanned = np.zeros(MAX_STATS, np.int64)
    it = ctypes.c_int32()
    conv = ctypes.c_int32()
    rc = lib.oracle_lpa(n, _p(off), _p(idx), _p(w), _p(order), float(tau), int(max_iters), int(bool(prune)),
                        _p(il), _p(ifl), _p(labels), _p(flags), _p(changed), _p(processed), _p(scanned),
                        ctypes.addressof(it), ctypes.addressof(conv), 0 if strict else 1)
    if rc != 0:
        raise ValueError(f"oracle_lpa failed ({rc})")
    k = min(it.value, MAX_STATS)
    return dict(labels=labels[:n], flags=flags[:n], changed=changed[:k], processed=processed[:k],
                scanned=scanned[:k], iterations=it.value, converged=bool(conv.value))


def color(g, seed: int = 0):
    """Greedy colouring in decreasing priority (deg(v), fmix32(v ^ seed), v)."""
    lib = _load()
    off, idx, _ = _csr_arrays(g)
    colors = np.empty(max(int(g.n), 1), np.int32)
    ncol = lib.oracle_color(int(g.n), _p(off), _p(idx), ctypes.c_uint32(seed & 0xFFFFFFFF), _p(colors))
    if ncol < 0:
        raise MemoryError("oracle_color failed")
    return colors[: g.n], int(ncol)


def color_order(colors, ncol: int):
    lib = _load()
    colors = np.ascontiguousarray(colors, dtype=np.int32)
    order = np.empty(max(len(colors), 1), np.int32)
    lib.oracle_color_order(len(colors), _p(colors), int(ncol), _p(order))
    return order[: len(colors)]


def lpa_deterministic(g, seed: int = 0, **kw) -> dict:
    """The deterministic mode's definition: LPA in (colour, id) order."""
    colors, ncol = color(g, seed)
    res = lpa(g, order=color_order(colors, ncol), **kw)
    res["colors"] = colors
    res["num_colors"] = ncol
    return res


def modularity(g, labels) -> float:
    lib = _load()
    off, idx, w = _csr_arrays(g)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    q = ctypes.c_double()
    rc = lib.oracle_modularity(int(g.n), _p(off), _p(idx), _p(w), _p(lab), ctypes.addressof(q))
    if rc != 0:
        raise ValueError(f"oracle_modularity failed ({rc})")
    return q.value


class _Sub:
    def __init__(self, n, offsets, indices, weights):
        self.n, self.offsets, self.indices, self.weights = n, offsets, indices, weights


def subgraph(g, lo: int, hi: int):
    """Rows [lo, hi) of a block-diagonal CSR, renumbered to local ids."""
    e0, e1 = int(g.offsets[lo]), int(g.offsets[hi])
    off = g.offsets[lo:hi + 1] - e0
    idx = g.indices[e0:e1] - lo
    w = None if g.weights is None else g.weights[e0:e1]
    return _Sub(hi - lo, off, idx.astype(np.int32), w)


def lpa_batch(g, graph_vptr, deterministic: bool = True, seed: int = 0, threads: int = 8, **kw) -> list:
    """Independent LPA per graph of a block-diagonal CSR (per-graph stop test).

    In deterministic mode the colouring is the greedy colouring of the whole
    block-diagonal graph (priorities from global ids); restricted to one graph
    it is that graph's colouring, so each graph runs in its own (colour, id)
    order.  Labels are returned as global vertex ids.
    """
    vptr = np.asarray(graph_vptr, dtype=np.int64)
    colors = color(g, seed)[0] if deterministic else None

    def one(k):
        lo, hi = int(vptr[k]), int(vptr[k + 1])
        sub = subgraph(g, lo, hi)
        order = None
        if deterministic:
            order = np.lexsort((np.arange(hi - lo), colors[lo:hi])).astype(np.int32)
        r = lpa(sub, order=order, **kw)
        r["labels"] = r["labels"] + lo
        return r

    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, range(len(vptr) - 1)))


__all__ = ["lpa", "color", "color_order", "lpa_deterministic", "modularity", "nmi", "lpa_batch", "subgraph"]
