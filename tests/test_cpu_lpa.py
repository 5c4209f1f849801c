"""The multicore CPU comparator (the paper's design on OpenMP threads).

With one thread its dynamic schedule visits the vertices in id order, so the
run is the sequential method: it must equal the oracle in id order label for
label, sweep for sweep (strict and non-strict).  With several threads any
interleaving is a valid asynchronous run: checked through invariants, a
verified fixed point and modularity within 0.01 of the sequential run."""
import numpy as np
import pytest

import oracle
from paper_2312_08140_amd import cpu_lpa, graphgen as gg


@pytest.mark.parametrize("strict", [True, False])
@pytest.mark.parametrize("kind", ["sbm", "rmat", "weighted", "degenerate"])
def test_one_thread_equals_oracle(kind, strict):
    g = {"sbm": lambda: gg.sbm(1000, 10, 0.1, 0.002, seed=1),
         "rmat": lambda: gg.rmat(13, 16, seed=2, weighted=False),
         "weighted": lambda: gg.rmat(12, 8, seed=3, weighted=True),
         "degenerate": lambda: gg.from_edges(7, [(0, 0), (1, 2), (2, 3), (5, 6)], [4, 0, 2, 1],
                                             keep_self_loops=True)}[kind]()
    for tau, it, prune in ((0.05, 20, True), (0.0, 7, True), (0.0, 5, False)):
        a = cpu_lpa.lpa(g, tau=tau, max_iters=it, prune=prune, strict=strict, threads=1)
        r = oracle.lpa(g, tau=tau, max_iters=it, prune=prune, strict=strict)
        assert np.array_equal(a["labels"], r["labels"])
        assert a["iterations"] == r["iterations"] and a["converged"] == r["converged"]
        assert a["changed"].tolist() == r["changed"].tolist()
        assert a["processed"].tolist() == r["processed"].tolist()
        assert a["scanned"].tolist() == r["scanned"].tolist()


def _components(g):
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg
    a = sp.csr_matrix((np.ones(g.m), g.indices, g.offsets), shape=(g.n, g.n))
    return cg.connected_components(a, directed=False)[1]


@pytest.mark.parametrize("seed", [1, 2])
def test_many_threads_quality_and_fixed_point(seed):
    g = gg.sbm(50_000, 50, 0.01, 0.0001, seed=seed, method="skip")
    a = cpu_lpa.lpa(g, tau=0.05, max_iters=20, threads=4)
    assert a["converged"]
    comp = _components(g)
    assert np.array_equal(comp[a["labels"]], comp)
    q_par = oracle.modularity(g, a["labels"])
    q_seq = oracle.modularity(g, oracle.lpa(g, tau=0.05, max_iters=20)["labels"])
    assert abs(q_par - q_seq) <= 0.01
    # verified fixed point: one more full sweep from these labels changes <= tau * n
    v = oracle.lpa(g, tau=-1.0, max_iters=1, prune=False, init_labels=a["labels"])
    assert v["changed"][0] <= 0.05 * g.n


def test_rejects_invalid_input():
    g = gg.from_edges(3, [(0, 1)])
    bad = gg.CSR(3, g.offsets, np.array([1, 7], np.int32))
    with pytest.raises(ValueError):
        cpu_lpa.lpa(bad)
    badw = gg.CSR(3, g.offsets, g.indices, np.array([0.5, 0.5], np.float32))
    with pytest.raises(ValueError):
        cpu_lpa.lpa(badw)
