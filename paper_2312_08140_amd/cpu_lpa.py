"""Multicore CPU label propagation in the paper's own design (ctypes binding
of ``include/gvelpa_cpu.h``, ``lib/libgvelpa_cpu.so``).

A host comparator for benchmarking the GPU library: OpenMP dynamic schedule
with chunk 2048, asynchronous in-place labels, 8-bit pruning flags and
per-thread Far-KV tables (Sections 4.1-4.2).  The GPU binding (``abi``) never
calls it.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _build.CPU_LIB.exists():
            raise RuntimeError(f"CPU comparator not built: {_build.CPU_LIB} (run __graft_entry__.build())")
        lib = ctypes.CDLL(str(_build.CPU_LIB))
        vp = ctypes.c_void_p
        lib.gvcpu_lpa.argtypes = [ctypes.c_int64, vp, vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp]
        lib.gvcpu_lpa.restype = ctypes.c_int
        lib.gvcpu_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().gvcpu_max_threads())


def lpa(g, tau: float = 0.05, max_iters: int = 20, prune: bool = True, strict: bool = True, threads: int = 0) -> dict:
    """Runs on host CSR ``g``; returns dict(labels, changed, processed,
    scanned (per sweep), iterations, converged, seconds, threads)."""
    lib = _load()
    n = int(g.n)
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.float32)
    labels = np.empty(max(n, 1), np.int32)
    k = max(max_iters, 1)
    changed, processed, scanned = (np.zeros(k, np.int64) for _ in range(3))
    it, conv, sec = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    p = lambda a: None if a is None else a.ctypes.data
    rc = lib.gvcpu_lpa(n, p(off), p(idx), p(w), float(tau), int(max_iters), int(bool(prune)), 0 if strict else 1,
                       int(threads), p(labels), p(changed), p(processed), p(scanned), ctypes.addressof(it),
                       ctypes.addressof(conv), ctypes.addressof(sec))
    if rc != 0:
        raise ValueError(f"gvcpu_lpa failed ({rc})")
    i = it.value
    return dict(labels=labels[:n], changed=changed[:i], processed=processed[:i], scanned=scanned[:i], iterations=i,
                converged=bool(conv.value), seconds=sec.value, threads=int(threads) if threads > 0 else max_threads())
