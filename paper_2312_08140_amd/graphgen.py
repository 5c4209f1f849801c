"""Seeded synthetic inputs: R-MAT, SBM, and a block-diagonal batch of uneven SBMs.

The generators live in their own host library (``lib/libgvelpa_gen.so``) and
hold none of the label-propagation arithmetic; the sequential oracle and the
GPU library both consume the CSR they return.  Every draw is counter based
(SplitMix64 output function), so a graph is a pure function of its
parameters and seed.

CSR layout: undirected with both directions stored, self-loops and duplicate
entries removed, rows sorted; ``offsets`` int64[n+1], ``indices`` int32[m],
``weights`` float32[m] holding small integers, or ``None`` for unit weights.

``rmat_device`` builds the same R-MAT graph in GPU memory
(``lib/libgvelpa_gen_gpu.so``, ``include/gvelpa_gen.h``): the CSR is
bit-identical to ``rmat``'s and lands in torch tensors on the device.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import _build

_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_int, ctypes.c_int64)
_lib = None
_gpu_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _build.GEN_LIB.exists():
            _build.build_gen()
        lib = ctypes.CDLL(str(_build.GEN_LIB))
        i64, u64, f64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int32
        p64 = ctypes.POINTER(ctypes.c_int64)
        pf64 = ctypes.POINTER(ctypes.c_double)
        lib.gg_rmat.argtypes = [ctypes.c_int, i64, f64, f64, f64, u64, ctypes.c_int, _ALLOC, p64, p64]
        lib.gg_sbm.argtypes = [i64, i64, f64, f64, u64, ctypes.c_int, ctypes.c_int, _ALLOC, p64]
        lib.gg_sbm_batch_params.argtypes = [i32, u64, f64, f64, f64, f64, f64, f64, p64, p64, pf64, pf64]
        lib.gg_sbm_batch.argtypes = [i32, p64, p64, pf64, pf64, u64, ctypes.c_int, _ALLOC, p64, p64, p64]
        lib.gg_grid.argtypes = [i64, i64, f64, u64, ctypes.c_int, _ALLOC, p64, p64]
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Host CSR graph.  ``weights is None`` means unit weights."""
    n: int
    offsets: np.ndarray
    indices: np.ndarray
    weights: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.indices.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)


class _Arrays:
    def __init__(self):
        self.arrays = {}
        self.cb = _ALLOC(self._alloc)

    def _alloc(self, kind, count):
        dtype = {0: np.int64, 1: np.int32, 2: np.float32}[kind]
        a = np.empty(max(int(count), 1), dtype=dtype)
        self.arrays[kind] = (a, int(count))
        return a.ctypes.data

    def get(self, kind):
        if kind not in self.arrays:
            return None
        a, c = self.arrays[kind]
        return a[:c]

    def take(self):
        """The three arrays (offsets, indices, weights); drops the holder's own
        references and its callback, which refers back to the holder, so the
        arrays are freed with their last user rather than at a later garbage
        collection."""
        out = (self.get(0), self.get(1), self.get(2))
        self.arrays = {}
        self.cb = None
        return out


def _weighted_code(weighted) -> int:
    # 1: weights 1..8 from a hash of the unordered pair; 0: an all-ones fp32 array; -1: None (unit)
    return {True: 1, False: -1, "ones": 0}[weighted]


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, weighted=True) -> CSR:
    lib = _load()
    arr = _Arrays()
    n = ctypes.c_int64()
    m = ctypes.c_int64()
    rc = lib.gg_rmat(scale, edge_factor, a, b, c, seed, _weighted_code(weighted), arr.cb,
                     ctypes.byref(n), ctypes.byref(m))
    if rc != 0:
        raise ValueError(f"gg_rmat failed ({rc})")
    return CSR(n.value, *arr.take(),
               name=f"rmat{scale}_ef{edge_factor}_s{seed}",
               meta=dict(kind="rmat", scale=scale, edge_factor=edge_factor, a=a, b=b, c=c, seed=seed))


def sbm(n: int, blocks: int, p_in: float, p_out: float, seed: int = 1, weighted=False,
        method: str = "auto") -> CSR:
    """Planted partition: ``blocks`` contiguous id ranges of near-equal size.

    method "direct" draws one Bernoulli per candidate pair (exact integer
    threshold); "skip" uses geometric skipping; "auto" is direct for n <= 20000.
    """
    lib = _load()
    direct = {"direct": 1, "skip": 0, "auto": 1 if n <= 20000 else 0}[method]
    arr = _Arrays()
    m = ctypes.c_int64()
    rc = lib.gg_sbm(n, blocks, p_in, p_out, seed, _weighted_code(weighted), direct, arr.cb, ctypes.byref(m))
    if rc != 0:
        raise ValueError(f"gg_sbm failed ({rc})")
    g = CSR(n, *arr.take(), name=f"sbm{n}_k{blocks}_s{seed}",
            meta=dict(kind="sbm", blocks=blocks, p_in=p_in, p_out=p_out, seed=seed))
    return g


def grid(rows: int, cols: int, p_keep: float = 0.55, seed: int = 1, weighted=False) -> CSR:
    """Low-degree road-like graph: the 4-neighbour lattice of rows x cols
    vertices with every lattice edge kept with probability p_keep (average
    degree about 4 p_keep)."""
    lib = _load()
    arr = _Arrays()
    n = ctypes.c_int64()
    m = ctypes.c_int64()
    rc = lib.gg_grid(rows, cols, p_keep, seed, _weighted_code(weighted), arr.cb, ctypes.byref(n), ctypes.byref(m))
    if rc != 0:
        raise ValueError(f"gg_grid failed ({rc})")
    return CSR(n.value, *arr.take(), name=f"grid{rows}x{cols}_p{p_keep}_s{seed}",
               meta=dict(kind="grid", rows=rows, cols=cols, p_keep=p_keep, seed=seed))


def sbm_truth(n: int, blocks: int) -> np.ndarray:
    """Planted block of every vertex (contiguous near-equal blocks)."""
    q, r = divmod(n, blocks)
    sizes = np.full(blocks, q, dtype=np.int64)
    sizes[:r] += 1
    return np.repeat(np.arange(blocks, dtype=np.int32), sizes)


def sbm_batch_params(count: int, master_seed: int = 7, n_range=(200, 50000), d_range=(8.0, 64.0),
                     mu_range=(0.1, 0.4)):
    lib = _load()
    n_g = np.zeros(count, np.int64)
    k_g = np.zeros(count, np.int64)
    p_in = np.zeros(count, np.float64)
    p_out = np.zeros(count, np.float64)
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    rc = lib.gg_sbm_batch_params(count, master_seed, float(n_range[0]), float(n_range[1]), d_range[0], d_range[1],
                                 mu_range[0], mu_range[1], P(n_g, ctypes.c_int64), P(k_g, ctypes.c_int64),
                                 P(p_in, ctypes.c_double), P(p_out, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"gg_sbm_batch_params failed ({rc})")
    return n_g, k_g, p_in, p_out


def sbm_batch(count: int = 4096, master_seed: int = 7, seed_base: int = 10000, n_range=(200, 50000),
              d_range=(8.0, 64.0), mu_range=(0.1, 0.4)):
    """``count`` independent SBMs as one block-diagonal CSR.

    Returns ``(csr, graph_vptr)``: graph g owns global ids
    ``[graph_vptr[g], graph_vptr[g+1])`` and uses seed ``seed_base + g``.
    """
    lib = _load()
    n_g, k_g, p_in, p_out = sbm_batch_params(count, master_seed, n_range, d_range, mu_range)
    vptr = np.zeros(count + 1, np.int64)
    arr = _Arrays()
    n = ctypes.c_int64()
    m = ctypes.c_int64()
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    rc = lib.gg_sbm_batch(count, P(n_g, ctypes.c_int64), P(k_g, ctypes.c_int64), P(p_in, ctypes.c_double),
                          P(p_out, ctypes.c_double), seed_base, -1, arr.cb, P(vptr, ctypes.c_int64),
                          ctypes.byref(n), ctypes.byref(m))
    if rc != 0:
        raise ValueError(f"gg_sbm_batch failed ({rc})")
    g = CSR(n.value, *arr.take(), name=f"sbmbatch{count}_s{master_seed}",
            meta=dict(kind="sbm_batch", count=count, master_seed=master_seed, k_g=k_g))
    return g, vptr


def from_edges(n: int, edges, weights=None, keep_self_loops: bool = False, symmetrize: bool = True) -> CSR:
    """CSR from an edge list (numpy; for small test graphs).

    Adds reverse edges when ``symmetrize``; drops self-loops unless asked to
    keep them; duplicate pairs are merged by keeping the first weight.
    """
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = None if weights is None else np.asarray(weights, dtype=np.float32).reshape(-1)
    if symmetrize:
        rev = e[:, ::-1]
        loops = e[:, 0] == e[:, 1]
        e = np.concatenate([e, rev[~loops]])
        if w is not None:
            w = np.concatenate([w, w[~loops]])
    if not keep_self_loops:
        keep = e[:, 0] != e[:, 1]
        e = e[keep]
        if w is not None:
            w = w[keep]
    key = e[:, 0] * max(n, 1) + e[:, 1]
    key_u, first = np.unique(key, return_index=True)
    e = e[first]
    if w is not None:
        w = w[first]
    order = np.lexsort((e[:, 1], e[:, 0]))
    e = e[order]
    if w is not None:
        w = w[order]
    counts = np.bincount(e[:, 0], minlength=n) if len(e) else np.zeros(n, np.int64)
    off = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    return CSR(n, off, e[:, 1].astype(np.int32), None if w is None else w.astype(np.float32))


@dataclass
class DeviceCSR:
    """CSR graph in device memory (torch tensors); ``weights is None`` means unit weights."""
    n: int
    offsets: object
    indices: object
    weights: object = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.indices.shape[0])

    def to_host(self) -> CSR:
        w = None if self.weights is None else self.weights.cpu().numpy()
        return CSR(self.n, self.offsets.cpu().numpy(), self.indices.cpu().numpy(), w, name=self.name,
                   meta=dict(self.meta))


def _load_gpu():
    global _gpu_lib
    if _gpu_lib is None:
        import torch  # noqa: F401  (binds the library to torch's HIP runtime)
        if not _build.GEN_GPU_LIB.exists():
            raise RuntimeError(f"GPU generator not built: {_build.GEN_GPU_LIB} (run __graft_entry__.build())")
        lib = ctypes.CDLL(str(_build.GEN_GPU_LIB))
        lib.gvgen_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, _ALLOC,
                                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        lib.gvgen_rmat.restype = ctypes.c_int
        lib.gvgen_status_string.argtypes = [ctypes.c_int]
        lib.gvgen_status_string.restype = ctypes.c_char_p
        _gpu_lib = lib
    return _gpu_lib


class _DeviceArrays:
    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.arrays = {}
        self.cb = _ALLOC(self._alloc)

    def _alloc(self, kind, count):
        t = self.torch
        dtype = {0: t.int64, 1: t.int32, 2: t.float32}[kind]
        a = t.empty(max(int(count), 1), dtype=dtype, device=self.device)
        self.arrays[kind] = (a, int(count))
        return a.data_ptr()

    def get(self, kind):
        if kind not in self.arrays:
            return None
        a, c = self.arrays[kind]
        return a[:c]

    def take(self):
        """The three arrays (offsets, indices, weights); drops the holder's own
        references and its callback, which refers back to the holder, so the
        arrays are freed with their last user rather than at a later garbage
        collection."""
        out = (self.get(0), self.get(1), self.get(2))
        self.arrays = {}
        self.cb = None
        return out


def rmat_device(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                seed: int = 1, weighted=True, device: int = 0) -> DeviceCSR:
    """``rmat`` generated and assembled on GPU ``device`` (same CSR, bit for bit)."""
    import torch
    lib = _load_gpu()
    arr = _DeviceArrays(device)
    n = ctypes.c_int64()
    m = ctypes.c_int64()
    stream = torch.cuda.current_stream(device).cuda_stream
    rc = lib.gvgen_rmat(scale, edge_factor, a, b, c, seed, _weighted_code(weighted), device, stream, arr.cb,
                        ctypes.byref(n), ctypes.byref(m))
    if rc != 0:
        raise RuntimeError(f"gvgen_rmat failed: {lib.gvgen_status_string(rc).decode()} ({rc})")
    return DeviceCSR(n.value, *arr.take(), name=f"rmat{scale}_ef{edge_factor}_s{seed}",
                     meta=dict(kind="rmat", scale=scale, edge_factor=edge_factor, a=a, b=b, c=c, seed=seed))


def rmat_expected_edges(scale: int, edge_factor: int) -> int:
    return edge_factor << scale


__all__ = ["CSR", "DeviceCSR", "rmat", "rmat_device", "sbm", "sbm_truth", "sbm_batch", "sbm_batch_params",
           "grid", "from_edges"]
