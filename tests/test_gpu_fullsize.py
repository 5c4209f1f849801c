"""Deterministic parity at the full sizes of the benchmark workloads.

* R-MAT scale 24, edge factor 16, weights 1..8 (16.8 M vertices, 0.52 G
  stored entries): labels, flags and per-sweep dN, processed and scanned
  counts equal the oracle run in (colour, id) order.
* The uneven batch of 4,096 SBMs (36.9 M vertices, 1.3 G entries) in one
  handle: every graph's labels, sweep count and convergence equal an
  independent oracle run of that graph (host threads, one graph each).
* More than 2^31 stored entries (513 disjoint 2,048-cliques, 2.15 G entries),
  the int64-offset path: labels equal the oracle and Appendix-style closed
  form (a clique ends with the smallest id other than its first-visited
  vertex), two sweeps.

Each case prints what it runs before every GPU step.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2312_08140_amd import abi, graphgen as gg

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]

DET = abi.LPA_MODE_DETERMINISTIC
THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_rmat24_deterministic_full_size():
    g = gg.rmat(24, 16, seed=1, weighted=True)
    say(f"R-MAT-24: n={g.n} m={g.m}; oracle colouring")
    ocol, onc = oracle.color(g, 0)
    say("GPU colouring and deterministic run")
    G = abi.LPAGraph(g)
    colors, nc = G.color(0)
    assert nc == onc and np.array_equal(colors, ocol), "colouring differs from the greedy oracle"
    labels, st = G.run(0.05, 20, DET, True)
    flags = G.flags()
    q = G.modularity()
    G.close()
    say(f"GPU: {st['iterations']} sweeps, dN {st['changed']}; oracle run")
    ref = oracle.lpa(g, order=oracle.color_order(ocol, onc), tau=0.05, max_iters=20)
    assert st["iterations"] == ref["iterations"] and st["converged"] == ref["converged"]
    assert st["changed"] == ref["changed"].tolist()
    assert st["frontier"] == ref["processed"].tolist()
    assert st["edges_scanned"] == ref["scanned"].tolist()
    assert np.array_equal(labels, ref["labels"])
    assert np.array_equal(flags, ref["flags"])
    assert q == oracle.modularity(g, ref["labels"])


def test_sbm_batch_4096_deterministic_full_size():
    g, vptr = gg.sbm_batch(4096, master_seed=7, seed_base=10000)
    say(f"batch of 4096 SBMs: n={g.n} m={g.m}; GPU run")
    B = abi.LPABatch(g, vptr)
    labels, st = B.run(0.05, 20, DET, True)
    it, cv = B.graph_stats()
    B.close()
    say(f"GPU: up to {st['iterations']} sweeps; oracle on {THREADS} threads")
    ref = oracle.lpa_batch(g, vptr, deterministic=True, tau=0.05, max_iters=20, threads=THREADS)
    bad = [k for k in range(4096)
           if not (np.array_equal(labels[vptr[k]:vptr[k + 1]], ref[k]["labels"]) and it[k] == ref[k]["iterations"]
                   and cv[k] == ref[k]["converged"])]
    assert not bad, f"{len(bad)} graphs differ, first {bad[:10]}"
    assert st["iterations"] == max(r["iterations"] for r in ref)


def _cliques_csr(c, k):
    """c disjoint unit-weight k-cliques, rows sorted, without self-loops."""
    n = c * k
    off = np.arange(n + 1, dtype=np.int64) * (k - 1)
    base = np.tile(np.arange(k, dtype=np.int32), (k, 1))
    pattern = base[~np.eye(k, dtype=bool)].reshape(k, k - 1)
    idx = np.empty(n * (k - 1), np.int32)
    for b in range(c):
        idx[b * k * (k - 1):(b + 1) * k * (k - 1)] = (pattern + b * k).ravel()
    return gg.CSR(n, off, idx, None, name=f"cliques{c}x{k}")


def test_more_than_2_31_entries_cliques():
    c, k = 513, 2048
    g = _cliques_csr(c, k)
    assert g.m > (1 << 31)
    vptr = np.arange(c + 1, dtype=np.int64) * k
    say(f"{c} cliques of {k}: n={g.n} m={g.m}; GPU colouring and deterministic run")
    G = abi.LPAGraph(g)
    colors, nc = G.color(0)
    labels, st = G.run(0.05, 20, DET, True)
    q = G.modularity()
    G.close()
    say(f"GPU: {st['iterations']} sweeps, dN {st['changed']}, scanned {st['edges_scanned']}; oracle")
    ocol, onc = oracle.color(g, 0)
    assert nc == onc == k and np.array_equal(colors, ocol)
    ref = oracle.lpa_batch(g, vptr, deterministic=True, tau=0.05, max_iters=20, threads=THREADS)
    for b in range(c):
        lo, hi = b * k, (b + 1) * k
        assert np.array_equal(labels[lo:hi], ref[b]["labels"]), f"clique {b}"
        first = lo + int(np.argmin(ocol[lo:hi]))          # colour 0 of the clique: visited first
        want = lo if first != lo else lo + 1              # smallest id of the clique other than it
        assert np.all(labels[lo:hi] == want), f"clique {b}"
    # sweep 1 re-processes the vertices marked after their turn in sweep 0 (the
    # last-visited vertex of a clique is not, nor its predecessor when the last
    # one kept its label): compare the per-sweep counts with the oracle's sums
    assert st["iterations"] == 2 and all(r["iterations"] == 2 for r in ref)
    assert st["changed"] == [c * (k - 1), 0]
    assert st["changed"] == [sum(int(r["changed"][s]) for r in ref) for s in range(2)]
    assert st["frontier"] == [sum(int(r["processed"][s]) for r in ref) for s in range(2)]
    assert st["edges_scanned"] == [sum(int(r["scanned"][s]) for r in ref) for s in range(2)]
    assert st["edges_scanned"][0] == g.m
    assert q == pytest.approx(1.0 - 1.0 / c, abs=1e-12)
