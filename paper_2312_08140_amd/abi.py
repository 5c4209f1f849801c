"""Thin ctypes binding of ``include/gvelpa.h`` (argument marshalling only).

Every function keeps the C name and signature; arrays may be numpy arrays
(host memory) or torch tensors (device memory, with ``LPA_FLAG_DEVICE_PTRS``).
``LPAGraph`` is a small owner of one handle.  The HIP library is required:
loading fails loudly when it is missing, and nothing here computes labels.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _build

try:  # load torch's HIP runtime first so that the library binds to the same one
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

LPA_OK = 0
LPA_ERR_INVALID_ARG = -1
LPA_ERR_INVALID_CSR = -2
LPA_ERR_WEIGHT_NOT_INTEGRAL = -3
LPA_ERR_TOO_LARGE = -4
LPA_ERR_OUT_OF_MEMORY = -5
LPA_ERR_DEVICE = -6
LPA_ERR_NO_GATE = -7
LPA_ERR_INTERNAL = -8

LPA_MODE_ASYNC = 0
LPA_MODE_DETERMINISTIC = 1

LPA_FLAG_DEVICE_PTRS = 1
LPA_FLAG_CHECK_SYMMETRIC = 2
LPA_FLAG_GATE = 4
LPA_FLAG_NO_GRAPH = 8
LPA_FLAG_KERNEL_TIMING = 16
LPA_FLAG_VERIFY = 32
LPA_FLAG_TRACE = 64
LPA_FLAG_EXACT_MARKS = 128
LPA_FLAG_ONE_LAUNCH = 256
LPA_FLAG_VERIFY_FULL = 512
LPA_FLAG_NO_REORDER = 1024
LPA_FLAG_NONSTRICT = 2048

GATE_PARAMS = 1377
GATE_FEATURES = 8
GATE_NOALLOC_MAX_SAMPLES = 262144

MAX_SWEEPS_RECORDED = 64
NUM_TIMED_KERNELS = 16
KERNEL_NAMES = ["compact", "bin0", "bin1", "bin2", "bin3", "bin4", "bin5", "hub_plan", "hub_chunk", "hub_finish",
                "end_sweep", "hub_part", "other", "gate_pass", "first", "k15"]


class lpa_stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("verified", ctypes.c_int32),
        ("num_colors", ctypes.c_int32),
        ("changed", ctypes.c_int64 * MAX_SWEEPS_RECORDED),
        ("frontier", ctypes.c_int64 * MAX_SWEEPS_RECORDED),
        ("edges_scanned", ctypes.c_int64 * MAX_SWEEPS_RECORDED),
        ("gated_out", ctypes.c_int64 * MAX_SWEEPS_RECORDED),
        ("ms", ctypes.c_float * MAX_SWEEPS_RECORDED),
        ("verify_changed", ctypes.c_int64),
        ("total_changed", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("setup_ms", ctypes.c_double),
        ("kernel_ms", ctypes.c_double * NUM_TIMED_KERNELS),
        ("kernel_launches", ctypes.c_int64 * NUM_TIMED_KERNELS),
        ("bin_vertices", ctypes.c_int64 * 8),
        ("bin_edges", ctypes.c_int64 * 8),
        ("bin_changed", ctypes.c_int64 * 8),
        ("bin_marks", ctypes.c_int64 * 8),
        ("compact_listed", ctypes.c_int64),
        ("compact_taken", ctypes.c_int64),
        ("weight_bytes", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("verify_edges_scanned", ctypes.c_int64),
        ("first_vertices", ctypes.c_int64),
        ("first_edges", ctypes.c_int64),
        ("first_changed", ctypes.c_int64),
        ("first_marks", ctypes.c_int64),
        ("first_reads", ctypes.c_int64),
    ]

    def to_dict(self) -> dict:
        k = min(self.iterations, MAX_SWEEPS_RECORDED)
        return dict(
            iterations=self.iterations, converged=bool(self.converged), verified=bool(self.verified),
            num_colors=self.num_colors, changed=list(self.changed[:k]), frontier=list(self.frontier[:k]),
            edges_scanned=list(self.edges_scanned[:k]), gated_out=list(self.gated_out[:k]), ms=list(self.ms[:k]),
            verify_changed=self.verify_changed, total_changed=self.total_changed, total_ms=self.total_ms,
            setup_ms=self.setup_ms,
            kernel_ms={KERNEL_NAMES[i]: self.kernel_ms[i] for i in range(NUM_TIMED_KERNELS) if self.kernel_launches[i]},
            kernel_launches={KERNEL_NAMES[i]: self.kernel_launches[i] for i in range(NUM_TIMED_KERNELS)
                             if self.kernel_launches[i]},
            bin_vertices=list(self.bin_vertices[:7]), bin_edges=list(self.bin_edges[:7]),
            bin_changed=list(self.bin_changed[:7]), bin_marks=list(self.bin_marks[:7]),
            compact_listed=self.compact_listed, compact_taken=self.compact_taken, weight_bytes=self.weight_bytes,
            verify_edges_scanned=self.verify_edges_scanned,
            first_vertices=self.first_vertices, first_edges=self.first_edges, first_changed=self.first_changed,
            first_marks=self.first_marks, first_reads=self.first_reads,
        )


_vp = ctypes.c_void_p
_i32, _i64, _u32, _u64, _f32, _f64 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                                      ctypes.c_float, ctypes.c_double)

# name -> (restype, argtypes); mirrors include/gvelpa.h
SIGNATURES = {
    "lpa_create": (ctypes.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_uint]),
    "lpa_run": (ctypes.c_int, [_vp, _f64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint, _vp, _vp, _vp,
                               ctypes.POINTER(lpa_stats)]),
    "lpa_get_flags": (ctypes.c_int, [_vp, _vp, ctypes.c_uint]),
    "lpa_modularity": (ctypes.c_int, [_vp, _vp, ctypes.c_uint, ctypes.POINTER(_f64)]),
    "lpa_color": (ctypes.c_int, [_vp, _u32, _vp, ctypes.c_uint, ctypes.POINTER(_i32)]),
    "lpa_set_bins": (ctypes.c_int, [_vp, _vp, _i32]),
    "lpa_set_async_phases": (ctypes.c_int, [_vp, _i32, _i32]),
    "lpa_set_async_schedule": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32]),
    "lpa_set_variants": (ctypes.c_int, [_vp, _vp, _i32]),
    "lpa_set_bin_order": (ctypes.c_int, [_vp, _i32]),
    "lpa_set_first_sweep": (ctypes.c_int, [_vp, _i32]),
    "lpa_get_schedule": (ctypes.c_int, [_vp, _vp]),
    "lpa_autotune": (ctypes.c_int, [_vp, _f64, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "lpa_batch_create": (ctypes.c_int, [_vp, _i32, _vp, _i64, _i64, _vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_uint]),
    "lpa_batch_stats": (ctypes.c_int, [_vp, _vp, _vp]),
    "lpa_batch_verify_stats": (ctypes.c_int, [_vp, _vp, _vp]),
    "lpa_gate_load": (ctypes.c_int, [_vp, _vp, _f32]),
    "lpa_set_trace": (ctypes.c_int, [_vp, _i64, _f64]),
    "lpa_gate_trace": (ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.POINTER(_i64), ctypes.c_uint]),
    "lpa_gate_forward": (ctypes.c_int, [_vp, _vp, _i64, _vp, ctypes.c_int, _vp, ctypes.c_uint]),
    "lpa_gate_backward": (ctypes.c_int, [_vp, _vp, _vp, _i64, _f32, _vp, ctypes.POINTER(_f32), ctypes.c_int, _vp,
                                         ctypes.c_uint]),
    "lpa_gate_backward_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i64, _f32, _vp, ctypes.POINTER(_f32), ctypes.c_int,
                                                 _vp]),
    "lpa_gate_train": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i32, _i32, _f32, _f32, _vp, ctypes.c_int, _vp,
                                      ctypes.c_uint]),
    "lpa_gate_threshold": (ctypes.c_int, [_vp, _vp, _vp, _i64, _f64, ctypes.POINTER(_f32), ctypes.c_int, _vp,
                                          ctypes.c_uint]),
    "lpa_nmi": (ctypes.c_int, [_vp, _vp, _i64, ctypes.POINTER(_f64), ctypes.c_int, _vp, ctypes.c_uint]),
    "lpa_destroy": (None, [_vp]),
    "lpa_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lpa_last_error_detail": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load ``lib/libgvelpa.so`` (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not _build.LPA_LIB.exists():
            raise RuntimeError(f"HIP library not built: {_build.LPA_LIB} (run __graft_entry__.build())")
        lib = ctypes.CDLL(str(_build.LPA_LIB))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class LPAError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        detail = ""
        if code == LPA_ERR_DEVICE:
            d = load().lpa_last_error_detail().decode()
            detail = f" [{d}]" if d else ""
        super().__init__(f"{what}: {status_string(code)} ({code}){detail}")


def status_string(code: int) -> str:
    return load().lpa_status_string(code).decode()


def _ptr(a) -> Optional[int]:
    """Address of a numpy array or torch tensor (None passes NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be contiguous")
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return a.data_ptr()
    raise TypeError(f"unsupported array type {type(a)}")


def _check(rc: int, what: str) -> None:
    if rc != LPA_OK:
        raise LPAError(rc, what)


def lpa_create(n, m, offsets, indices, weights=None, device=0, hip_stream=None, flags=0):
    h = ctypes.c_void_p()
    rc = load().lpa_create(ctypes.byref(h), n, m, _ptr(offsets), _ptr(indices), _ptr(weights), device, hip_stream,
                           flags)
    return rc, h


def lpa_run(handle, tolerance, max_iters, mode, prune, flags=0, init_labels=None, init_flags=None, labels_out=None,
            stats=None):
    return load().lpa_run(handle, tolerance, max_iters, mode, int(prune), flags, _ptr(init_labels), _ptr(init_flags),
                          _ptr(labels_out), ctypes.byref(stats) if stats is not None else None)


def lpa_get_flags(handle, flags_out, flags=0):
    return load().lpa_get_flags(handle, _ptr(flags_out), flags)


def lpa_modularity(handle, labels=None, flags=0):
    q = ctypes.c_double()
    rc = load().lpa_modularity(handle, _ptr(labels), flags, ctypes.byref(q))
    return rc, q.value


def lpa_color(handle, seed=0, colors_out=None, flags=0):
    nc = ctypes.c_int32()
    rc = load().lpa_color(handle, seed & 0xFFFFFFFF, _ptr(colors_out), flags, ctypes.byref(nc))
    return rc, nc.value


def lpa_set_bins(handle, max_degree=None):
    arr = None if max_degree is None else np.ascontiguousarray(max_degree, dtype=np.int32)
    return load().lpa_set_bins(handle, _ptr(arr), 0 if arr is None else len(arr))


def lpa_set_async_phases(handle, phases, by_colour=0):
    return load().lpa_set_async_phases(handle, phases, int(by_colour))


def lpa_set_async_schedule(handle, early_phases, early_sweeps, late_phases, by_colour=1):
    return load().lpa_set_async_schedule(handle, early_phases, early_sweeps, late_phases, int(by_colour))


def lpa_set_bin_order(handle, hubs_last):
    return load().lpa_set_bin_order(handle, int(hubs_last))


def lpa_set_first_sweep(handle, kernels):
    return load().lpa_set_first_sweep(handle, int(kernels))


def lpa_get_schedule(handle, out):
    return load().lpa_get_schedule(handle, _ptr(out))


def lpa_set_variants(handle, variant=None):
    arr = None if variant is None else np.ascontiguousarray(variant, dtype=np.int32)
    return load().lpa_set_variants(handle, _ptr(arr), 0 if arr is None else len(arr))


def lpa_autotune(handle, tolerance, max_iters, mode, variant_out=None, bin_ms_out=None, schedule_out=None,
                 bins_out=None):
    return load().lpa_autotune(handle, tolerance, max_iters, mode, _ptr(variant_out), _ptr(bin_ms_out),
                               _ptr(schedule_out), _ptr(bins_out))


def lpa_batch_create(n_graphs, graph_vptr, n, m, offsets, indices, weights=None, device=0, hip_stream=None, flags=0):
    h = ctypes.c_void_p()
    rc = load().lpa_batch_create(ctypes.byref(h), n_graphs, _ptr(graph_vptr), n, m, _ptr(offsets), _ptr(indices),
                                 _ptr(weights), device, hip_stream, flags)
    return rc, h


def lpa_batch_stats(handle, iterations=None, converged=None):
    return load().lpa_batch_stats(handle, _ptr(iterations), _ptr(converged))


def lpa_batch_verify_stats(handle, verified=None, verify_changed=None):
    return load().lpa_batch_verify_stats(handle, _ptr(verified), _ptr(verify_changed))


def lpa_destroy(handle):
    load().lpa_destroy(handle)


def lpa_nmi(a, b, n, device=0, hip_stream=None, flags=0):
    out = ctypes.c_double()
    rc = load().lpa_nmi(_ptr(a), _ptr(b), n, ctypes.byref(out), device, hip_stream, flags)
    return rc, out.value


def nmi(a, b, device=0) -> float:
    """NMI of two labelings (numpy arrays or device tensors of int32)."""
    dev = hasattr(a, "data_ptr")
    if dev != hasattr(b, "data_ptr"):
        raise ValueError("both labelings must be host arrays or both device tensors")
    if not dev:
        a = np.ascontiguousarray(a, dtype=np.int32)
        b = np.ascontiguousarray(b, dtype=np.int32)
    n = int(a.shape[0])
    if int(b.shape[0]) != n:
        raise ValueError("labelings differ in length")
    rc, v = lpa_nmi(a, b, n, device, _current_stream(device), LPA_FLAG_DEVICE_PTRS if dev else 0)
    _check(rc, "lpa_nmi")
    return v


def lpa_gate_load(handle, params, threshold):
    return load().lpa_gate_load(handle, _ptr(params), threshold)


def lpa_set_trace(handle, capacity, probability):
    return load().lpa_set_trace(handle, capacity, probability)


def lpa_gate_trace(handle, features=None, targets=None, capacity=0, flags=0):
    c = ctypes.c_int64()
    rc = load().lpa_gate_trace(handle, _ptr(features), _ptr(targets), capacity, ctypes.byref(c), flags)
    return rc, c.value


def lpa_gate_forward(params, features, count, probs, device=0, hip_stream=None, flags=0):
    return load().lpa_gate_forward(_ptr(params), _ptr(features), count, _ptr(probs), device, hip_stream, flags)


def lpa_gate_backward(params, features, targets, count, pos_weight, grad, device=0, hip_stream=None, flags=0):
    loss = ctypes.c_float()
    rc = load().lpa_gate_backward(_ptr(params), _ptr(features), _ptr(targets), count, pos_weight, _ptr(grad),
                                  ctypes.byref(loss), device, hip_stream, flags)
    return rc, loss.value


def lpa_gate_backward_noalloc(params, features, targets, count, pos_weight, grad, device=0, hip_stream=None):
    loss = ctypes.c_float()
    rc = load().lpa_gate_backward_noalloc(_ptr(params), _ptr(features), _ptr(targets), count, pos_weight, _ptr(grad),
                                          ctypes.byref(loss), device, hip_stream)
    return rc, loss.value


def lpa_gate_train(params, features, targets, count, order, epochs, batch, lr, pos_weight, epoch_loss=None,
                   device=0, hip_stream=None, flags=0):
    return load().lpa_gate_train(_ptr(params), _ptr(features), _ptr(targets), count, _ptr(order), epochs, batch, lr,
                                 pos_weight, _ptr(epoch_loss), device, hip_stream, flags)


def lpa_gate_threshold(params, features, targets, count, recall, device=0, hip_stream=None, flags=0):
    t = ctypes.c_float()
    rc = load().lpa_gate_threshold(_ptr(params), _ptr(features), _ptr(targets), count, recall, ctypes.byref(t),
                                   device, hip_stream, flags)
    return rc, t.value


def lpa_status_string(code):
    return status_string(code)


def _current_stream(device: int):
    if torch is None or not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream(device).cuda_stream


class LPAGraph:
    """Owns one library handle for a CSR graph (numpy host arrays or torch device tensors)."""

    def __init__(self, csr=None, *, n=None, offsets=None, indices=None, weights=None, device: int = 0,
                 stream=None, check_symmetric: bool = False, reorder: bool = True):
        if csr is not None:
            n, offsets, indices, weights = csr.n, csr.offsets, csr.indices, csr.weights
        self.n = int(n)
        self.device = device
        on_device = hasattr(offsets, "data_ptr")
        flags = (LPA_FLAG_DEVICE_PTRS if on_device else 0) | (LPA_FLAG_CHECK_SYMMETRIC if check_symmetric else 0)
        flags |= 0 if reorder else LPA_FLAG_NO_REORDER
        if not on_device:
            offsets = np.ascontiguousarray(offsets, dtype=np.int64)
            indices = np.ascontiguousarray(indices, dtype=np.int32)
            weights = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
        self._keep = (offsets, indices, weights) if on_device else None
        self.m = int(indices.shape[0])
        self.stream = _current_stream(device) if stream is None else stream
        rc, h = lpa_create(self.n, self.m, offsets, indices, weights, device, self.stream, flags)
        _check(rc, "lpa_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lpa_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, tolerance=0.05, max_iters=20, mode=LPA_MODE_ASYNC, prune=True, flags=0, init_labels=None,
            init_flags=None, labels_out=None):
        """Returns (labels, stats dict).  labels_out may be a device tensor."""
        st = lpa_stats()
        fl = flags
        if labels_out is None:
            labels_out = np.empty(self.n, np.int32)
        if hasattr(labels_out, "data_ptr"):
            fl |= LPA_FLAG_DEVICE_PTRS
            if init_labels is not None and not hasattr(init_labels, "data_ptr"):
                raise ValueError("init arrays must live where labels_out lives")
        else:
            if init_labels is not None:
                init_labels = np.ascontiguousarray(init_labels, dtype=np.int32)
            if init_flags is not None:
                init_flags = np.ascontiguousarray(init_flags, dtype=np.uint8)
        rc = lpa_run(self.handle, tolerance, max_iters, mode, prune, fl, init_labels, init_flags, labels_out, st)
        _check(rc, "lpa_run")
        return labels_out, st.to_dict()

    def flags(self):
        out = np.empty(self.n, np.uint8)
        _check(lpa_get_flags(self.handle, out), "lpa_get_flags")
        return out

    def modularity(self, labels=None) -> float:
        fl = LPA_FLAG_DEVICE_PTRS if hasattr(labels, "data_ptr") else 0
        if labels is not None and not fl:
            labels = np.ascontiguousarray(labels, dtype=np.int32)
        rc, q = lpa_modularity(self.handle, labels, fl)
        _check(rc, "lpa_modularity")
        return q

    def color(self, seed=0):
        out = np.empty(self.n, np.int32)
        rc, nc = lpa_color(self.handle, seed, out)
        _check(rc, "lpa_color")
        return out, nc

    def set_bins(self, max_degree=None):
        _check(lpa_set_bins(self.handle, max_degree), "lpa_set_bins")

    def set_async_phases(self, phases, by_colour=False):
        _check(lpa_set_async_phases(self.handle, phases, by_colour), "lpa_set_async_phases")

    def set_async_schedule(self, early_phases=16, early_sweeps=2, late_phases=4, by_colour=True):
        _check(lpa_set_async_schedule(self.handle, early_phases, early_sweeps, late_phases, by_colour),
               "lpa_set_async_schedule")

    def set_variants(self, variant=None):
        _check(lpa_set_variants(self.handle, variant), "lpa_set_variants")

    def set_bin_order(self, hubs_last):
        _check(lpa_set_bin_order(self.handle, hubs_last), "lpa_set_bin_order")

    def set_first_sweep(self, kernels):
        """Kernels of each step of the first sweep that read the initial labels (0-7)."""
        _check(lpa_set_first_sweep(self.handle, kernels), "lpa_set_first_sweep")

    def schedule(self):
        """(early steps, early sweeps, late steps, by colour, hubs last, snapshot kernels of the first sweep,
        rows allow it) of the handle."""
        out = np.zeros(7, np.int32)
        _check(lpa_get_schedule(self.handle, out), "lpa_get_schedule")
        return tuple(int(x) for x in out)

    def autotune(self, tolerance=0.05, max_iters=20, mode=LPA_MODE_ASYNC):
        """Returns (variant per bin, ms per run of each chosen bin kernel, schedule, bin degree limits)."""
        v = np.zeros(6, np.int32)
        ms = np.zeros(6, np.float64)
        sch = np.zeros(3, np.int32)
        lim = np.zeros(6, np.int32)
        _check(lpa_autotune(self.handle, tolerance, max_iters, mode, v, ms, sch, lim), "lpa_autotune")
        return v, ms, tuple(int(x) for x in sch), tuple(int(x) for x in lim)

    def gate_load(self, params, threshold):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (GATE_PARAMS,):
            raise ValueError(f"gate parameters must be {GATE_PARAMS} float32 values")
        _check(lpa_gate_load(self.handle, p, float(threshold)), "lpa_gate_load")

    def set_trace(self, capacity, probability=1.0):
        _check(lpa_set_trace(self.handle, int(capacity), float(probability)), "lpa_set_trace")

    def gate_trace(self):
        """(features float32[count][8], targets uint8[count]) recorded since set_trace."""
        rc, c = lpa_gate_trace(self.handle)
        _check(rc, "lpa_gate_trace")
        x = np.empty((c, GATE_FEATURES), np.float32)
        y = np.empty(c, np.uint8)
        if c:
            rc, c2 = lpa_gate_trace(self.handle, x, y, c)
            _check(rc, "lpa_gate_trace")
        return x, y


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _samples(features, targets):
    """Host or device sample arrays -> (features, targets, count, flags)."""
    if hasattr(features, "data_ptr"):
        if targets is not None and not hasattr(targets, "data_ptr"):
            raise ValueError("features and targets must both be host or both device arrays")
        return features, targets, int(features.shape[0]), LPA_FLAG_DEVICE_PTRS
    x = np.ascontiguousarray(features, dtype=np.float32).reshape(-1, GATE_FEATURES)
    y = None if targets is None else np.ascontiguousarray(targets, dtype=np.uint8)
    return x, y, int(x.shape[0]), 0


def gate_forward(params, features, device=0):
    """Gate probabilities of every sample (float32[count], where the features live)."""
    p = _f32(params, (GATE_PARAMS,))
    x, _, c, fl = _samples(features, None)
    out = (torch.empty(c, dtype=torch.float32, device=features.device) if fl else np.empty(c, np.float32))
    _check(lpa_gate_forward(p, x, c, out, device, _current_stream(device), fl), "lpa_gate_forward")
    return out


def gate_backward(params, features, targets, pos_weight=1.0, device=0):
    """(gradient float32[1377], loss) of the mean weighted BCE."""
    p = _f32(params, (GATE_PARAMS,))
    x, y, c, fl = _samples(features, targets)
    g = np.empty(GATE_PARAMS, np.float32)
    rc, loss = lpa_gate_backward(p, x, y, c, float(pos_weight), g, device, _current_stream(device), fl)
    _check(rc, "lpa_gate_backward")
    return g, loss


def gate_backward_noalloc(params, features, targets, pos_weight=1.0, device=0):
    """``gate_backward`` without any device allocation (device tensors only; at
    most GATE_NOALLOC_MAX_SAMPLES samples per call)."""
    if not (hasattr(features, "data_ptr") and hasattr(targets, "data_ptr")):
        raise ValueError("features and targets must be device tensors")
    p = _f32(params, (GATE_PARAMS,))
    g = np.empty(GATE_PARAMS, np.float32)
    rc, loss = lpa_gate_backward_noalloc(p, features, targets, int(features.shape[0]), float(pos_weight), g, device,
                                         _current_stream(device))
    _check(rc, "lpa_gate_backward_noalloc")
    return g, loss


def gate_train(params, features, targets, epochs, batch, lr=1e-3, pos_weight=1.0, order=None, device=0):
    """Adam training; returns (new parameters float32[1377], per-epoch loss float32[epochs])."""
    p = _f32(params, (GATE_PARAMS,)).copy()
    x, y, c, fl = _samples(features, targets)
    if order is not None:
        if fl:
            if not hasattr(order, "data_ptr"):
                raise ValueError("order must live where the samples live")
        else:
            order = np.ascontiguousarray(order, dtype=np.int64)
    losses = np.zeros(max(epochs, 1), np.float32)
    rc = lpa_gate_train(p, x, y, c, order, int(epochs), int(batch), float(lr), float(pos_weight), losses, device,
                        _current_stream(device), fl)
    _check(rc, "lpa_gate_train")
    return p, losses[:epochs]


def gate_threshold(params, features, targets, recall, device=0):
    p = _f32(params, (GATE_PARAMS,))
    x, y, c, fl = _samples(features, targets)
    rc, t = lpa_gate_threshold(p, x, y, c, float(recall), device, _current_stream(device), fl)
    _check(rc, "lpa_gate_threshold")
    return t


class LPABatch(LPAGraph):
    """Many independent graphs (block-diagonal CSR) in one handle; graph g owns
    vertices [graph_vptr[g], graph_vptr[g+1])."""

    def __init__(self, csr, graph_vptr, device: int = 0, stream=None, reorder: bool = True):
        self.n = int(csr.n)
        self.device = device
        self.vptr = np.ascontiguousarray(graph_vptr, dtype=np.int64)
        self.ngraphs = len(self.vptr) - 1
        off = np.ascontiguousarray(csr.offsets, dtype=np.int64)
        idx = np.ascontiguousarray(csr.indices, dtype=np.int32)
        w = None if csr.weights is None else np.ascontiguousarray(csr.weights, dtype=np.float32)
        self._keep = None
        self.m = int(idx.shape[0])
        self.stream = _current_stream(device) if stream is None else stream
        rc, h = lpa_batch_create(self.ngraphs, self.vptr, self.n, self.m, off, idx, w, device, self.stream,
                                 0 if reorder else LPA_FLAG_NO_REORDER)
        _check(rc, "lpa_batch_create")
        self.handle = h

    def graph_stats(self):
        it = np.zeros(self.ngraphs, np.int32)
        cv = np.zeros(self.ngraphs, np.int32)
        _check(lpa_batch_stats(self.handle, it, cv), "lpa_batch_stats")
        return it, cv.astype(bool)

    def verify_stats(self):
        """Per graph: verified (bool) and labels changed by its verification sweeps."""
        ok = np.zeros(self.ngraphs, np.int32)
        ch = np.zeros(self.ngraphs, np.int32)
        _check(lpa_batch_verify_stats(self.handle, ok, ch), "lpa_batch_verify_stats")
        return ok.astype(bool), ch
