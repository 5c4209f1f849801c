"""The no-allocation gradient entry point (lpa_gate_backward_noalloc) against
lpa_gate_backward: the same gradient and loss bit for bit, on two calls in a
row (the second smaller, so stale scratch contents would show), at the
largest accepted size, and a clear error beyond it."""
import sys

import numpy as np
import pytest

from paper_2312_08140_amd import abi

pytestmark = pytest.mark.gpu


def _samples(count, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, (count, 8)).astype(np.float32)
    X[:, 0] = np.log2(1.0 + rng.integers(1, 5000, count)).astype(np.float32)
    y = (rng.uniform(size=count) < 0.3).astype(np.uint8)
    return X, y


def _params(seed):
    return (np.random.default_rng(seed).standard_normal(abi.GATE_PARAMS) * 0.3).astype(np.float32)


def test_noalloc_gradient_equals_allocating_entry_point():
    import torch
    for count, pw, seed in [(50_000, 2.5, 1), (777, 1.0, 2), (abi.GATE_NOALLOC_MAX_SAMPLES, 4.0, 3), (1, 0.5, 4)]:
        print(f"noalloc gradient count={count} pos_weight={pw}", flush=True)
        sys.stdout.flush()
        X, y = _samples(count, seed)
        p = _params(seed + 10)
        Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
        g_ref, l_ref = abi.gate_backward(p, Xd, yd, pos_weight=pw)
        g, l = abi.gate_backward_noalloc(p, Xd, yd, pos_weight=pw)
        assert np.array_equal(g, g_ref) and l == l_ref


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    count = abi.GATE_NOALLOC_MAX_SAMPLES + 1
    X, y = _samples(count, 5)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    g = np.empty(abi.GATE_PARAMS, np.float32)
    rc, _ = abi.lpa_gate_backward_noalloc(_params(6), Xd, yd, count, 1.0, g)
    assert rc == abi.LPA_ERR_TOO_LARGE
    rc, _ = abi.lpa_gate_backward_noalloc(_params(6), Xd, yd, 0, 1.0, g)
    assert rc == abi.LPA_ERR_INVALID_ARG
