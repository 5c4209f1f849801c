"""Seeded input generators: structure and determinism (CPU only)."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2312_08140_amd import graphgen as gg


def _check_csr(g):
    off, idx = g.offsets, g.indices
    assert off[0] == 0 and off[-1] == g.m and np.all(np.diff(off) >= 0)
    assert idx.min() >= 0 and idx.max() < g.n
    rows = np.repeat(np.arange(g.n), np.diff(off))
    assert not np.any(rows == idx)  # no self-loops
    key = rows.astype(np.int64) * g.n + idx
    assert np.all(np.diff(key) > 0)  # sorted rows, no duplicates
    rkey = idx.astype(np.int64) * g.n + rows
    order = np.argsort(rkey)
    assert np.array_equal(np.sort(rkey), key)  # symmetric structure
    if g.weights is not None:
        assert np.array_equal(g.weights[order], g.weights)  # w_ij = w_ji
        assert g.weights.min() >= 1 and g.weights.max() <= 8
        assert np.all(g.weights == np.round(g.weights))


def test_rmat_structure():
    g = gg.rmat(12, 16, seed=1)
    _check_csr(g)
    assert g.n == 4096 and 0 < g.m <= 2 * 16 * 4096
    d = g.degrees()
    assert d[0] == d.max()  # a = 0.57 puts the heaviest corner at vertex 0


def test_sbm_structure_and_density():
    g = gg.sbm(1000, 10, 0.1, 0.002, seed=1)
    _check_csr(g)
    assert g.weights is None
    truth = gg.sbm_truth(1000, 10)
    rows = np.repeat(np.arange(g.n), g.degrees())
    inside = truth[rows] == truth[g.indices]
    # expected directed counts: 2 * 10 * C(100,2) * 0.1 = 9900 inside, 2 * 45 * 1e4 * 0.002 = 1800 across
    assert 9000 < inside.sum() < 10800
    assert 1400 < (~inside).sum() < 2200


def test_sbm_skip_method_density():
    g = gg.sbm(20000, 20, 0.02, 0.0002, seed=3, method="skip")
    _check_csr(g)
    exp = 2 * (20 * 1000 * 999 / 2 * 0.02 + 190 * 1e6 * 0.0002)
    assert abs(g.m - exp) < 0.05 * exp


def test_batch_block_diagonal():
    g, vptr = gg.sbm_batch(count=12, master_seed=7, n_range=(200, 3000))
    _check_csr(g)
    assert vptr[0] == 0 and vptr[-1] == g.n and np.all(np.diff(vptr) >= 200 - 1)
    gid = np.searchsorted(vptr, np.arange(g.n), side="right") - 1
    rows = np.repeat(np.arange(g.n), g.degrees())
    assert np.array_equal(gid[rows], gid[g.indices])  # no cross-graph edges


def test_thread_count_independent():
    code = ("from paper_2312_08140_amd import graphgen as gg; import hashlib;"
            "g = gg.rmat(13, 8, seed=9); h = hashlib.sha256(g.offsets.tobytes() + g.indices.tobytes() + "
            "g.weights.tobytes()).hexdigest(); print(h)")
    outs = []
    for t in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env, text=True).strip())
    assert outs[0] == outs[1]


def test_grid_lattice_structure():
    """The low-degree lattice: every entry joins lattice neighbours, rows are
    sorted and symmetric, p_keep = 1 gives the full 4-neighbour lattice, and
    the average degree is about 4 p_keep; the graph is a function of the seed."""
    from paper_2312_08140_amd import graphgen as gg
    full = gg.grid(7, 9, 1.0)
    assert full.n == 63 and full.m == 2 * (7 * 8 + 6 * 9)
    for v in range(full.n):
        r, c = divmod(v, 9)
        want = sorted(u for u in (v - 9, v - 1, v + 1, v + 9)
                      if 0 <= u < 63 and (abs(u - v) == 9 or u // 9 == r))
        assert full.indices[full.offsets[v]:full.offsets[v + 1]].tolist() == want
    g = gg.grid(300, 400, 0.55, seed=5)
    assert abs(g.m / g.n - 4 * 0.55 * (1 - 0.5 / 300 - 0.5 / 400)) < 0.02
    h = gg.grid(300, 400, 0.55, seed=5)
    assert np.array_equal(g.indices, h.indices) and np.array_equal(g.offsets, h.offsets)
    lat = set()
    for v in range(g.n):
        for u in g.indices[g.offsets[v]:g.offsets[v + 1]]:
            assert abs(int(u) - v) in (1, 400) and (v, int(u)) not in lat
            lat.add((v, int(u)))
    assert all((u, v) in lat for v, u in lat)
