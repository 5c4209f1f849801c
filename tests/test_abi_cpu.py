"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects invalid input before any device work."""
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2312_08140_amd import abi, graphgen as gg

HEADER = Path(__file__).resolve().parent.parent / "include" / "gvelpa.h"


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", HEADER.read_text(), flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(lpa_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    lib = abi.load()
    names = declared_functions()
    assert "lpa_create" in names and "lpa_run" in names and "lpa_modularity" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in abi.SIGNATURES, f"binding lacks {name}"


def test_status_strings():
    for code in range(-8, 1):
        assert abi.lpa_status_string(code)
    assert abi.lpa_status_string(-99) == "unknown status"


def _create(n, off, idx, w=None, flags=0):
    rc, h = abi.lpa_create(n, len(idx), np.asarray(off, np.int64), np.asarray(idx, np.int32),
                           None if w is None else np.asarray(w, np.float32), 0, None, flags)
    if rc == 0:
        abi.lpa_destroy(h)
    return rc


def test_invalid_csr_rejected_on_host():
    assert _create(3, [1, 1, 2, 2], [0, 1]) == abi.LPA_ERR_INVALID_CSR      # offsets[0] != 0
    assert _create(3, [0, 2, 1, 2], [1, 0]) == abi.LPA_ERR_INVALID_CSR      # decreasing
    assert _create(3, [0, 1, 2, 3], [1, 0]) == abi.LPA_ERR_INVALID_CSR      # offsets[n] != m
    assert _create(2, [0, 1, 2], [1, 5]) == abi.LPA_ERR_INVALID_CSR         # index out of range
    assert _create(2, [0, 1, 2], [1, -1]) == abi.LPA_ERR_INVALID_CSR


def test_bad_weights_rejected_on_host():
    off, idx = [0, 1, 2], [1, 0]
    assert _create(2, off, idx, [1.5, 1.5]) == abi.LPA_ERR_WEIGHT_NOT_INTEGRAL
    assert _create(2, off, idx, [-1, -1]) == abi.LPA_ERR_WEIGHT_NOT_INTEGRAL
    assert _create(2, off, idx, [np.nan, np.nan]) == abi.LPA_ERR_WEIGHT_NOT_INTEGRAL
    assert _create(2, off, idx, [np.inf, np.inf]) == abi.LPA_ERR_WEIGHT_NOT_INTEGRAL
    assert _create(2, off, idx, [2.0 ** 25, 2.0 ** 25]) == abi.LPA_ERR_WEIGHT_NOT_INTEGRAL


def test_weighted_degree_limit():
    # 300 entries of weight 2^24 in one row exceed 2^32
    k = 300
    off = [0, k] + [k + i + 1 for i in range(k)]
    idx = list(range(1, k + 1)) + [0] * k
    w = [2.0 ** 24] * (2 * k)
    assert _create(k + 1, off, idx, w) == abi.LPA_ERR_TOO_LARGE


def test_asymmetric_rejected_when_asked():
    assert _create(2, [0, 1, 1], [1], flags=abi.LPA_FLAG_CHECK_SYMMETRIC) == abi.LPA_ERR_INVALID_CSR
    g = gg.from_edges(3, [(0, 1), (1, 2)], [1, 2])
    w = g.weights.copy()
    w[0] = 3
    assert _create(3, g.offsets, g.indices, w, flags=abi.LPA_FLAG_CHECK_SYMMETRIC) == abi.LPA_ERR_INVALID_CSR


def test_argument_errors():
    rc, _ = abi.lpa_create(-1, 0, np.zeros(1, np.int64), None, None, 0, None, 0)
    assert rc == abi.LPA_ERR_INVALID_ARG
    rc, _ = abi.lpa_create(1 << 31, 0, np.zeros(2, np.int64), None, None, 0, None, 0)
    assert rc == abi.LPA_ERR_TOO_LARGE
    assert abi.lpa_run(None, 0.05, 20, 0, 1) == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_batch_stats(None) == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_batch_verify_stats(None) == abi.LPA_ERR_INVALID_ARG


def test_batch_ranges_checked_on_host():
    """The graph ranges of a batch are checked before any device work: at
    least one graph, starting at 0, non-decreasing, ending at n."""
    g = gg.from_edges(6, [(0, 1), (3, 4)])
    for vptr, ng in (([0], 0), ([1, 6], 1), ([0, 4, 3, 6], 3), ([0, 3, 5], 2)):
        rc, h = abi.lpa_batch_create(ng, np.array(vptr, np.int64), g.n, g.m, g.offsets, g.indices)
        assert rc == abi.LPA_ERR_INVALID_ARG, vptr
        assert not h.value


def test_no_device_reports_device_error():
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    g = gg.sbm(100, 2, 0.2, 0.01, seed=1)
    assert _create(g.n, g.offsets, g.indices) == abi.LPA_ERR_DEVICE


def test_gate_argument_errors_on_host():
    p = np.zeros(abi.GATE_PARAMS, np.float32)
    x = np.zeros((4, 8), np.float32)
    y = np.zeros(4, np.uint8)
    out = np.zeros(4, np.float32)
    g = np.zeros(abi.GATE_PARAMS, np.float32)
    assert abi.lpa_gate_forward(None, x, 4, out) == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_gate_forward(p, None, 4, out) == abi.LPA_ERR_INVALID_ARG
    bad = p.copy()
    bad[7] = np.nan
    assert abi.lpa_gate_forward(bad, x, 4, out) == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_gate_backward(p, x, y, 0, 1.0, g)[0] == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_gate_backward(p, x, y, 4, -1.0, g)[0] == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_gate_train(p, x, y, 4, None, 1, 0, 1e-3, 1.0) == abi.LPA_ERR_INVALID_ARG      # batch 0
    assert abi.lpa_gate_train(p, x, y, 4, None, 1, 2, 0.0, 1.0) == abi.LPA_ERR_INVALID_ARG      # lr 0
    order = np.array([0, 1, 2, 4], np.int64)                                                    # 4 out of range
    assert abi.lpa_gate_train(p, x, y, 4, order, 1, 2, 1e-3, 1.0) == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_gate_threshold(p, x, y, 4, 1.5)[0] == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_gate_load(None, p, 0.5) == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_set_trace(None, 10, 0.5) == abi.LPA_ERR_INVALID_ARG


def test_gate_no_device_reports_device_error():
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    p = np.zeros(abi.GATE_PARAMS, np.float32)
    x = np.zeros((4, 8), np.float32)
    assert abi.lpa_gate_forward(p, x, 4, np.zeros(4, np.float32)) == abi.LPA_ERR_DEVICE


def test_nmi_argument_errors_on_host():
    a = np.zeros(4, np.int32)
    assert abi.lpa_nmi(a, None, 4)[0] == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_nmi(a, a, -1)[0] == abi.LPA_ERR_INVALID_ARG
    assert abi.lpa_nmi(None, None, 0) == (abi.LPA_OK, 1.0)   # empty labelings need no device
