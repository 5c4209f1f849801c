"""GPU parity of the learned active-set gate.

* the network's forward pass, gradient and Adam steps against the FP64
  oracle of ``oracle/mlp.py`` evaluated at the same bf16-rounded weights;
* the traced samples of a deterministic run against the sequential trace
  oracle (same vertex order, so the same sample multiset);
* gated runs: threshold 0 is the plain method followed by the verification
  sweep, bit for bit in deterministic mode; threshold 1 skips every flagged
  vertex and the verification sweep's fallback still reaches the plain
  quality; a trained gate keeps modularity within 0.01 of the plain run.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp
from oracle.gate_trace import lpa_trace
from paper_2312_08140_amd import abi, gate, graphgen as gg

pytestmark = pytest.mark.gpu

DET, ASYNC = abi.LPA_MODE_DETERMINISTIC, abi.LPA_MODE_ASYNC


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_order(G, g, seed=0):
    """The deterministic mode's vertex order from the oracle's greedy colouring
    (checked equal to the library's colouring first)."""
    colors, nc = G.color(seed)
    ocol, onc = oracle.color(g, seed)
    assert nc == onc and np.array_equal(colors, ocol), "colouring differs from the greedy oracle"
    return oracle.color_order(ocol, onc)


def _same_samples(X, y, ref, decimals=4):
    """Trace samples equal the oracle's as a multiset of whole rows (features
    and target together): both sides sorted lexicographically by (target,
    features rounded to a few decimals), then compared row by row."""
    assert len(y) == len(ref["y"])
    a = np.column_stack([y.astype(np.float64), X.astype(np.float64)])
    b = np.column_stack([ref["y"].astype(np.float64), ref["X"]])
    ka, kb = np.round(a, decimals), np.round(b, decimals)
    a = a[np.lexsort(ka.T[::-1])]
    b = b[np.lexsort(kb.T[::-1])]
    assert np.array_equal(a[:, 0], b[:, 0])
    assert np.allclose(a[:, 1:], b[:, 1:], rtol=1e-6, atol=1e-5)


def random_samples(count, seed):
    """Features in the ranges the sweep produces: f0 = log2(1 + deg), f3 0/1, the rest in [0, 1]."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, (count, 8)).astype(np.float32)
    X[:, 0] = np.log2(1.0 + rng.integers(1, 5000, count)).astype(np.float32)
    X[:, 3] = rng.integers(0, 2, count).astype(np.float32)
    y = (rng.uniform(size=count) < 0.3).astype(np.uint8)
    return X, y


def random_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(mlp.NPARAMS) * scale).astype(np.float32)


def normwise(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("count", [1, 127, 10_000])
def test_forward_matches_oracle(count):
    say(f"gate forward count={count}")
    X, _ = random_samples(count, 1)
    p32 = random_params(2)
    p = abi.gate_forward(p32, X)
    ref, _ = mlp.forward(mlp.bf16_round(p32), X.astype(np.float64))
    assert np.max(np.abs(p - ref) / np.maximum(ref, 1e-30)) <= 1e-5


def test_forward_device_pointers():
    import torch
    X, _ = random_samples(3000, 3)
    p32 = random_params(4)
    host = abi.gate_forward(p32, X)
    dev = abi.gate_forward(p32, torch.from_numpy(X).cuda())
    assert np.array_equal(dev.cpu().numpy(), host)


@pytest.mark.parametrize("count,pw", [(1, 1.0), (3000, 2.5), ((1 << 22) + 777, 4.0)])
def test_backward_matches_oracle(count, pw):
    """Gradient per tensor within 1e-3 normwise of the FP64 gradient at the
    same bf16 weights; the loss within 1e-5.  The largest case spans two of
    the library's 4 Mi-sample slices."""
    say(f"gate backward count={count} pos_weight={pw}")
    X, y = random_samples(count, 5)
    p32 = random_params(6)
    g, loss = abi.gate_backward(p32, X, y, pos_weight=pw)
    pb = mlp.bf16_round(p32)
    gref = mlp.backward(pb, X.astype(np.float64), y, pos_weight=pw)
    lref = mlp.loss(pb, X.astype(np.float64), y, pos_weight=pw)
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    gd, rd = mlp.unpack(g), mlp.unpack(gref)
    for name, _ in mlp.SHAPES:
        assert normwise(gd[name], rd[name]) <= 1e-3, name


def test_train_matches_oracle_adam():
    """Two epochs of mini-batch Adam (ragged last batch, shuffled order)
    against the same steps in FP64 at the bf16 rounding of an FP32 master."""
    count, batch, epochs, lr, pw = 1000, 256, 2, 1e-3, 2.0
    X, y = random_samples(count, 7)
    p32 = random_params(8)
    rng = np.random.default_rng(9)
    order = np.concatenate([rng.permutation(count) for _ in range(epochs)]).astype(np.int64)
    got, losses = abi.gate_train(p32, X, y, epochs, batch, lr=lr, pos_weight=pw, order=order)
    theta = p32.astype(np.float32)
    m = np.zeros(mlp.NPARAMS)
    v = np.zeros(mlp.NPARAMS)
    t = 0
    ref_losses = []
    for e in range(epochs):
        acc = 0.0
        for b in range(0, count, batch):
            sel = order[e * count + b:e * count + min(b + batch, count)]
            pb = mlp.bf16_round(theta)
            acc += mlp.loss(pb, X[sel].astype(np.float64), y[sel], pw) * len(sel) / count
            gr = mlp.backward(pb, X[sel].astype(np.float64), y[sel], pos_weight=pw)
            t += 1
            th64, m, v = mlp.adam_step(theta.astype(np.float64), gr, m, v, t, lr=lr)
            theta = th64.astype(np.float32)
        ref_losses.append(acc)
    assert np.allclose(losses, ref_losses, rtol=1e-4)
    d_gpu = got.astype(np.float64) - p32
    d_ref = theta.astype(np.float64) - p32
    # Adam moves each weight by about lr per step; only a gradient within
    # rounding of zero can flip a step's sign
    assert normwise(d_gpu, d_ref) <= 2e-2
    assert np.mean(np.abs(d_gpu - d_ref) > 1e-5) <= 0.01


def test_train_learns_a_rule():
    """A label that is a threshold rule of two features becomes predictable."""
    X, _ = random_samples(20_000, 10)
    y = ((X[:, 1] < 0.3) & (X[:, 3] > 0.5)).astype(np.uint8)
    info = gate.train(X, y, epochs=20, batch=512, lr=3e-3, recall=0.98, seed=1)
    assert info["losses"][-1] < 0.25 * info["losses"][0]
    assert info["holdout_recall"] >= 0.98
    # the positives are 15 % of the samples; a useful gate skips most of the rest
    assert info["holdout_skip"] >= 0.7


def test_threshold_keeps_recall():
    X, y = random_samples(5000, 11)
    p32 = random_params(12)
    for r in (0.5, 0.9, 1.0):
        t = abi.gate_threshold(p32, X, y, r)
        p = abi.gate_forward(p32, X)
        pos = p[y == 1]
        assert np.mean(pos >= t) >= r
        assert np.any(pos == t)        # the largest such threshold is a positive's probability


# ---------------------------------------------------------------- traces

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_trace_matches_oracle(seed):
    """Deterministic run, every re-processing traced: the samples equal the
    trace oracle's in (colour, id) order as a multiset of whole rows (the
    sweep is feature 4), so no feature can move between samples unnoticed."""
    g = gg.sbm(400 * seed, 4, 0.08, 0.01, seed=seed, weighted=seed == 2)
    say(f"trace parity n={g.n} m={g.m} seed={seed}")
    G = abi.LPAGraph(g)
    order = _oracle_order(G, g)
    G.set_trace(1 << 20, 1.0)
    labels, st = G.run(0.0, 12, DET, True, flags=abi.LPA_FLAG_TRACE)
    X, y = G.gate_trace()
    G.close()
    ref = lpa_trace(g, order=order, tau=0.0, max_iters=12)
    assert np.array_equal(labels, ref["labels"])
    assert len(y) == len(ref["y"])
    _same_samples(X, y, ref)


def test_trace_hub_path_matches_oracle():
    """Every vertex a hub (all bin limits 0): the features the hub path writes
    (from its label partitions' statistics) equal the trace oracle's."""
    g = gg.sbm(800, 4, 0.08, 0.01, seed=2, weighted=True)
    G = abi.LPAGraph(g)
    G.set_bins([0, 0, 0, 0, 0, 0])
    order = _oracle_order(G, g)
    G.set_trace(1 << 20, 1.0)
    labels, st = G.run(0.0, 12, DET, True, flags=abi.LPA_FLAG_TRACE)
    X, y = G.gate_trace()
    G.close()
    ref = lpa_trace(g, order=order, tau=0.0, max_iters=12)
    assert np.array_equal(labels, ref["labels"])
    assert len(y) == len(ref["y"])
    _same_samples(X, y, ref)


def test_trace_sampling_and_capacity():
    g = gg.sbm(20_000, 20, 0.01, 0.0005, seed=4)
    G = abi.LPAGraph(g)
    G.set_trace(1 << 22, 1.0)
    _, st = G.run(0.05, 20, ASYNC, True, flags=abi.LPA_FLAG_TRACE)
    X, y = G.gate_trace()
    full = len(y)
    assert full == sum(st["frontier"][1:]) and int(y.sum()) == sum(st["changed"][1:])
    G.set_trace(1 << 22, 0.25)
    G.run(0.05, 20, ASYNC, True, flags=abi.LPA_FLAG_TRACE)
    _, y25 = G.gate_trace()
    assert 0.15 * full <= len(y25) <= 0.35 * full
    G.set_trace(100, 1.0)
    G.run(0.05, 20, ASYNC, True, flags=abi.LPA_FLAG_TRACE)
    _, y100 = G.gate_trace()
    assert len(y100) == 100
    G.close()


# ---------------------------------------------------------------- gated runs

@pytest.mark.parametrize("kind", ["sbm", "rmat"])
def test_threshold_zero_is_plain_with_verification(kind):
    """Threshold 0 processes every flagged vertex: the gated deterministic run
    equals the plain run with LPA_FLAG_VERIFY label for label, and both equal
    the oracle's run followed by one unpruned sweep (and, if that sweep
    changes more than tau * n labels, by plain pruning from its state)."""
    g = gg.sbm(1000, 10, 0.1, 0.002, seed=3) if kind == "sbm" else gg.rmat(12, 8, seed=2, weighted=True)
    say(f"gate threshold 0 {kind} n={g.n} m={g.m}")
    G = abi.LPAGraph(g)
    G.gate_load(random_params(13), 0.0)
    a, sa = G.run(0.05, 20, DET, True, flags=abi.LPA_FLAG_GATE)
    b, sb = G.run(0.05, 20, DET, True, flags=abi.LPA_FLAG_VERIFY)
    assert np.array_equal(a, b)
    assert sa["changed"] == sb["changed"] and sa["verify_changed"] == sb["verify_changed"]
    assert sa["verified"] == sb["verified"] and sum(sa["gated_out"]) == 0
    order = _oracle_order(G, g)
    r1 = oracle.lpa(g, order=order, tau=0.05, max_iters=20)
    r2 = oracle.lpa(g, order=order, tau=0.05, max_iters=1, prune=False, init_labels=r1["labels"])
    assert sa["verify_changed"] == int(r2["changed"][0])
    if r2["changed"][0] <= 0.05 * g.n:
        assert sa["verified"] and np.array_equal(a, r2["labels"])
    G.close()


@pytest.mark.parametrize("kind", ["sbm", "rmat"])
def test_pruned_verification_equals_full(kind):
    """The verification sweep over the flagged vertices gives the labels and
    dN of the sweep over every vertex (deterministic mode, from the state a
    gated run leaves, with many vertices still flagged)."""
    g = gg.sbm(2000, 20, 0.05, 0.002, seed=6) if kind == "sbm" else gg.rmat(12, 8, seed=3, weighted=True)
    G = abi.LPAGraph(g)
    G.gate_load(random_params(15), 0.5)
    a, sa = G.run(0.05, 20, DET, True, flags=abi.LPA_FLAG_GATE)
    b, sb = G.run(0.05, 20, DET, True, flags=abi.LPA_FLAG_GATE | abi.LPA_FLAG_VERIFY_FULL)
    say(f"verify {kind}: gated_out {sum(sa['gated_out'])} verify_changed {sa['verify_changed']} "
        f"edges {sa['verify_edges_scanned']} vs full {sb['verify_edges_scanned']}")
    assert np.array_equal(a, b)
    assert sa["changed"] == sb["changed"] and sa["verify_changed"] == sb["verify_changed"]
    assert sa["verified"] == sb["verified"]
    assert sb["verify_edges_scanned"] >= sa["verify_edges_scanned"]
    G.close()


def test_threshold_one_falls_back():
    """Threshold 1 gates out every re-processing: the run stalls after sweep 0,
    the verification sweep sees the stall and plain pruning finishes the job."""
    g = gg.sbm(20_000, 20, 0.01, 0.0005, seed=5)
    G = abi.LPAGraph(g)
    plain, sp = G.run(0.05, 20, ASYNC, True)
    q_plain = G.modularity(plain)
    G.gate_load(random_params(14), 1.0)
    lab, st = G.run(0.05, 20, ASYNC, True, flags=abi.LPA_FLAG_GATE)
    assert sum(st["gated_out"]) > 0 and st["frontier"][1] == 0
    assert st["verified"]
    assert G.modularity(lab) >= q_plain - 0.01
    G.close()


def test_trained_gate_quality():
    """A gate trained on traces of other SBMs keeps modularity within 0.01
    of the plain run on a fresh SBM, verified, with fewer vertices processed
    after sweep 0."""
    train_graphs = [gg.sbm(100_000, 100, 32 * (1 - mu) / 999, 32 * mu / (100_000 - 1000), seed=100 + i)
                    for i, mu in enumerate((0.1, 0.2, 0.3, 0.4))]
    X, y = gate.collect(train_graphs, probability=0.5)
    say(f"gate samples {len(y)} positives {int(y.sum())}")
    info = gate.train(X, y, epochs=4, batch=4096, lr=1e-3, recall=0.98, seed=0)
    assert info["holdout_recall"] >= 0.98
    for mu in (0.2, 0.3):
        g = gg.sbm(200_000, 200, 32 * (1 - mu) / 999, 32 * mu / (200_000 - 1000), seed=1)
        G = abi.LPAGraph(g)
        plain, sp = G.run(0.05, 20, ASYNC, True)
        qp = G.modularity(plain)
        G.gate_load(info["params"], info["threshold"])
        lab, sg = G.run(0.05, 20, ASYNC, True, flags=abi.LPA_FLAG_GATE)
        qg = G.modularity(lab)
        say(f"mu={mu} plain Q={qp:.4f} frontier={sum(sp['frontier'][1:])} gated Q={qg:.4f} "
            f"frontier={sum(sg['frontier'][1:])} gated_out={sum(sg['gated_out'])} verified={sg['verified']}")
        assert sg["verified"] and qg >= qp - 0.01
        assert sum(sg["gated_out"]) > 0
        G.close()


def test_trained_gate_saves_work_on_rmat():
    """What the trained network gains: on R-MAT under the one-step schedule,
    a gate trained on traces of smaller R-MAT graphs (same schedule) reaches
    a verified fixed point scanning fewer stored entries than plain pruning
    does to reach one (its verification sweep included on both sides), at the
    same modularity (within 0.01).  Asynchronous runs differ from run to run
    (a plain run may stop a sweep early), so the entry counts are medians of
    three runs."""
    sched = (1, 0, 1)
    train_graphs = [gg.rmat(19, 16, seed=100 + i, weighted=True) for i in range(4)]
    X, y = gate.collect(train_graphs, probability=0.5, schedule=sched)
    info = gate.train(X, y, epochs=4, batch=4096, lr=1e-3, recall=0.98, seed=0)
    g = gg.rmat(20, 16, seed=1, weighted=True)
    G = abi.LPAGraph(g)
    G.set_async_schedule(*sched)
    ep, eg = [], []
    for _ in range(3):
        plain, sp = G.run(0.05, 20, ASYNC, True, flags=abi.LPA_FLAG_VERIFY)
        assert sp["verified"]
        ep.append(sum(sp["edges_scanned"]) + sp["verify_edges_scanned"])
    qp = G.modularity(plain)
    G.gate_load(info["params"], info["threshold"])
    for _ in range(3):
        lab, sg = G.run(0.05, 20, ASYNC, True, flags=abi.LPA_FLAG_GATE)
        assert sg["verified"]
        eg.append(sum(sg["edges_scanned"]) + sg["verify_edges_scanned"])
    qg = G.modularity(lab)
    say(f"verified plain entries {ep} Q={qp:.6f}; gated entries {eg} Q={qg:.6f} skipped={sum(sg['gated_out'])} "
        f"verify_changed={sg['verify_changed']}")
    assert qg >= qp - 0.01
    assert abi.nmi(plain, lab) >= 0.99
    assert np.median(eg) < 0.95 * np.median(ep)
    G.close()


# ---------------------------------------------------------------- the gate inside the sweep

def _pick_gate(g, order, seeds=(21, 22, 23, 24), tau=0.05, max_iters=20, min_margin=1e-3):
    """Parameters and a threshold in (0, 1) for which the gated oracle takes
    no decision within ``min_margin`` of the threshold's logit and skips at
    least one flagged vertex.  Candidate logit thresholds are midpoints of the
    widest gaps between the decision logits of the plain trace (middle half of
    their range); all of it runs on the oracle side."""
    from oracle.gate_trace import _logit_fp64, lpa_gated, lpa_trace
    trace = lpa_trace(g, order=order, tau=tau, max_iters=max_iters)
    for seed in seeds:
        theta = random_params(seed)
        z = np.sort(np.unique(_logit_fp64(mlp.bf16_round(theta), trace["X"])))
        if len(z) < 8:
            continue
        lo, hi = len(z) // 4, 3 * len(z) // 4
        gaps = np.diff(z[lo:hi + 1])
        for k in np.argsort(gaps)[::-1][:6]:
            zc = 0.5 * (z[lo + k] + z[lo + k + 1])
            thr = float(np.float32(1.0 / (1.0 + np.exp(-zc))))
            if not 0.0 < thr < 1.0:
                continue
            ref = lpa_gated(g, theta, thr, order=order, tau=tau, max_iters=max_iters)
            if ref["margin"] >= min_margin and ref["gated"].sum() > 0:
                return theta, thr, ref
    raise AssertionError("no gate with a safe margin found")


@pytest.mark.parametrize("kind", ["sbm", "rmat", "all_hubs", "lds_table"])
def test_gated_deterministic_equals_gated_oracle(kind):
    """The network evaluated inside the sweep (decision pass + compaction)
    against the gated method's oracle at a threshold strictly inside (0, 1):
    deterministic mode, so labels, per-sweep dN, processed vertices, scanned
    entries, gated-out vertices and the verification outcome must all be equal.
    The threshold is chosen (on the oracle side) so that no decision lies
    within 1e-3 of it in logit, beyond any fp32-vs-fp64 difference."""
    if kind in ("rmat", "lds_table"):
        g = gg.rmat(11, 8, seed=5, weighted=True)
    else:
        g = gg.sbm(1200 if kind == "sbm" else 800, 6 if kind == "sbm" else 4, 0.05, 0.006, seed=11,
                   weighted=True)
    G = abi.LPAGraph(g)
    if kind == "all_hubs":
        G.set_bins([0, 0, 0, 0, 0, 0])  # every vertex through the hub kernels (their feature writes)
    if kind == "lds_table":
        G.set_variants([1, 0, 0, 0, 0, 0])  # the lowest bin's LDS table (the default is its register table)
    order = _oracle_order(G, g)
    theta, thr, ref = _pick_gate(g, order)
    say(f"gated {kind}: n={g.n} m={g.m} threshold={thr:.6f} margin={ref['margin']:.2e} "
        f"gated={ref['gated'].tolist()} changed={ref['changed'].tolist()} verified={ref['verified']}")
    G.gate_load(theta, thr)
    lab, st = G.run(0.05, 20, DET, True, flags=abi.LPA_FLAG_GATE)
    G.close()
    assert np.array_equal(lab, ref["labels"])
    assert st["iterations"] == ref["iterations"] and st["converged"] == ref["converged"]
    assert st["changed"] == ref["changed"].tolist()
    assert st["frontier"] == ref["processed"].tolist()
    assert st["edges_scanned"] == ref["scanned"].tolist()
    assert st["gated_out"] == ref["gated"].tolist()
    assert st["verify_changed"] == ref["verify_changed"]
    assert st["verify_edges_scanned"] == ref["verify_scanned"]
    assert st["verified"] == ref["verified"]


# ---------------------------------------------------------------- gated and verified batches

def _batch_parts(g, vptr, B, seed=0):
    """Per graph of a batch: its vertex range, its subgraph and the
    deterministic mode's order restricted to it (the greedy colouring of the
    whole block-diagonal graph, checked equal to the library's)."""
    colors, nc = B.color(seed)
    ocol, onc = oracle.color(g, seed)
    assert nc == onc and np.array_equal(colors, ocol), "colouring differs from the greedy oracle"
    parts = []
    for k in range(len(vptr) - 1):
        lo, hi = int(vptr[k]), int(vptr[k + 1])
        order = np.lexsort((np.arange(hi - lo), ocol[lo:hi])).astype(np.int32)
        parts.append((lo, hi, oracle.subgraph(g, lo, hi), order))
    return parts


def _gated_refs(parts, theta, thr, tau, max_iters):
    from oracle.gate_trace import lpa_gated
    return [lpa_gated(sub, theta, thr, order=order, tau=tau, max_iters=max_iters) for _, _, sub, order in parts]


def _check_batch(B, parts, refs, lab, st):
    """Every graph of the batch against its own gated-method oracle run:
    labels, counted sweeps, convergence, verification outcome and the labels
    its verification sweeps changed; the run's totals follow."""
    it, cv = B.graph_stats()
    ok, vch = B.verify_stats()
    for k, ((lo, hi, _, _), r) in enumerate(zip(parts, refs)):
        assert np.array_equal(lab[lo:hi], r["labels"] + lo), f"graph {k}"
        assert it[k] == r["iterations"] and cv[k] == r["converged"], f"graph {k}: {it[k]} {cv[k]}"
        assert ok[k] == r["verified"] and vch[k] == r["verify_changed"], f"graph {k}: {ok[k]} {vch[k]}"
    assert st["verified"] == all(r["verified"] for r in refs)
    assert st["converged"] == all(r["converged"] for r in refs)
    assert st["verify_changed"] == sum(r["verify_changed"] for r in refs)


def _gate_batch(count=6, seed=3, n_range=(60, 300)):
    return gg.sbm_batch(count=count, master_seed=seed, seed_base=700 + seed, n_range=n_range)


@pytest.mark.parametrize("tau,max_iters,full", [(0.05, 20, False), (0.05, 20, True), (0.01, 2, False),
                                                (0.01, 2, True), (0.0, 1, False)])
def test_batch_verified_equals_oracle(tau, max_iters, full):
    """A verified batch (gate off): each graph runs the method, its own
    verification sweep and, where that fails (max_iters = 2 stops graphs
    early), its fallback sweeps and last verification - the gated oracle at
    threshold 0, graph by graph.  A full verification processes every vertex
    and gives the same outcome.  tau = 0 with one sweep leaves graphs
    unconverged and unverified at the end of their fallback."""
    g, vptr = _gate_batch(12, 5)
    B = abi.LPABatch(g, vptr)
    parts = _batch_parts(g, vptr, B)
    refs = _gated_refs(parts, random_params(1), 0.0, tau, max_iters)
    say(f"verified batch: n={g.n} m={g.m} tau={tau} max_iters={max_iters} full={full} "
        f"verified={[r['verified'] for r in refs]} iterations={[r['iterations'] for r in refs]}")
    fl = abi.LPA_FLAG_VERIFY_FULL if full else abi.LPA_FLAG_VERIFY
    lab, st = B.run(tau, max_iters, DET, True, flags=fl)
    _check_batch(B, parts, refs, lab, st)
    if max_iters <= 2:
        assert any(r["verify_changed"] > 0 for r in refs)  # some graph's first verification found work
    if max_iters == 1:
        assert not all(r["verified"] for r in refs)
    B.close()


def _pick_batch_gate(parts, seeds=(21, 22, 23, 24, 25, 26), tau=0.05, max_iters=20, min_margin=1e-3):
    """Gate parameters and a threshold in (0, 1) for which no decision of any
    graph's gated oracle run lies within ``min_margin`` of the threshold's
    logit and some flagged vertex is skipped; candidates are midpoints of the
    widest gaps between the decision logits of the graphs' plain traces."""
    from oracle.gate_trace import _logit_fp64
    X = np.concatenate([lpa_trace(sub, order=order, tau=tau, max_iters=max_iters)["X"]
                        for _, _, sub, order in parts])
    for seed in seeds:
        theta = random_params(seed)
        z = np.sort(np.unique(_logit_fp64(mlp.bf16_round(theta), X)))
        if len(z) < 8:
            continue
        lo, hi = len(z) // 4, 3 * len(z) // 4
        gaps = np.diff(z[lo:hi + 1])
        for k in np.argsort(gaps)[::-1][:6]:
            zc = 0.5 * (z[lo + k] + z[lo + k + 1])
            thr = float(np.float32(1.0 / (1.0 + np.exp(-zc))))
            if not 0.0 < thr < 1.0:
                continue
            refs = _gated_refs(parts, theta, thr, tau, max_iters)
            if min(r["margin"] for r in refs) >= min_margin and sum(int(r["gated"].sum()) for r in refs) > 0:
                return theta, thr, refs
    raise AssertionError("no gate with a safe margin found")


def test_batch_gated_equals_gated_oracle():
    """A gated batch in deterministic mode: the in-sweep network gates only the
    graphs still in their gated sweeps, and every graph matches its own gated
    oracle run (threshold chosen on the oracle side with a 1e-3 logit margin)."""
    g, vptr = _gate_batch(6, 3)
    B = abi.LPABatch(g, vptr)
    parts = _batch_parts(g, vptr, B)
    theta, thr, refs = _pick_batch_gate(parts)
    say(f"gated batch: n={g.n} m={g.m} threshold={thr:.6f} gated={[int(r['gated'].sum()) for r in refs]} "
        f"verified={[r['verified'] for r in refs]}")
    B.gate_load(theta, thr)
    lab, st = B.run(0.05, 20, DET, True, flags=abi.LPA_FLAG_GATE)
    _check_batch(B, parts, refs, lab, st)
    assert sum(st["gated_out"]) == sum(int(r["gated"].sum()) for r in refs)
    B.close()


@pytest.mark.parametrize("max_iters", [20, 5])
def test_batch_gate_skipping_everything_falls_back(max_iters):
    """Threshold 1 skips every flagged vertex after the first sweep: graphs
    fail verification and recover through their fallback sweeps, each as its
    gated oracle run says; a plain run on the same handle afterwards equals
    the plain oracle again."""
    g, vptr = _gate_batch(10, 4)
    B = abi.LPABatch(g, vptr)
    parts = _batch_parts(g, vptr, B)
    theta = random_params(31)
    refs = _gated_refs(parts, theta, 1.0, 0.05, max_iters)
    say(f"threshold-1 batch: n={g.n} m={g.m} verified={[r['verified'] for r in refs]} "
        f"iterations={[r['iterations'] for r in refs]} verify_changed={[r['verify_changed'] for r in refs]}")
    assert any(r["verify_changed"] > 0 for r in refs)
    B.gate_load(theta, 1.0)
    lab, st = B.run(0.05, max_iters, DET, True, flags=abi.LPA_FLAG_GATE)
    _check_batch(B, parts, refs, lab, st)
    lab, st = B.run(0.05, 20, DET, True)
    plain = oracle.lpa_batch(g, vptr, deterministic=True, tau=0.05, max_iters=20)
    it, cv = B.graph_stats()
    for k, (lo, hi, _, _) in enumerate(parts):
        assert np.array_equal(lab[lo:hi], plain[k]["labels"]), f"graph {k}"
        assert it[k] == plain[k]["iterations"] and cv[k] == plain[k]["converged"]
    B.close()


def test_batch_gated_async():
    """Asynchronous gated batch: labels stay inside their graph, every graph
    ends verified, and modularity stays within 0.01 of the plain batch run."""
    g, vptr = gg.sbm_batch(count=200, master_seed=9, seed_base=900, n_range=(100, 3000))
    B = abi.LPABatch(g, vptr)
    plain, sp = B.run(0.05, 20, ASYNC, True)
    qp = B.modularity(plain)
    B.gate_load(random_params(22), 0.5)
    lab, st = B.run(0.05, 20, ASYNC, True, flags=abi.LPA_FLAG_GATE)
    ok, vch = B.verify_stats()
    gid = np.searchsorted(vptr, np.arange(g.n), side="right") - 1
    qg = B.modularity(lab)
    say(f"async gated batch: n={g.n} m={g.m} Q plain {qp:.5f} gated {qg:.5f} skipped={sum(st['gated_out'])} "
        f"verify_changed={st['verify_changed']} sweeps={st['iterations']}")
    assert np.array_equal(gid[lab], gid)
    assert ok.all() and st["verified"] and st["converged"]
    assert sum(st["gated_out"]) > 0
    assert abs(qg - qp) <= 0.01
    B.close()
