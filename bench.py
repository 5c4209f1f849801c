"""Benchmark: strict label propagation on R-MAT graphs, one MI355X.

Headline workload (default): R-MAT scale 26, edge factor 32, (a, b, c, d) =
(0.57, 0.19, 0.19, 0.05), symmetrised, self-loops and duplicates removed,
integer weights 1..8 stored as fp32, seed 1 (67.1 M vertices, 4.16 G stored
entries), generated and assembled on the GPU; tau = 0.05, at most 20 sweeps,
vertex pruning on.  A step is one whole run of the method (every sweep to
convergence) in the asynchronous mode, with the graph already resident in HBM.

Printed: one JSON line.  ``value`` is edges scanned per second over the timed
runs (the per-sweep rate, weighted by the work of each sweep); the line also
carries the sweep-0 rate, time to converge, modularity, the deterministic
mode's figures, the roofline of the dominant kernel (HIP events on the
library's stream), the same figures on R-MAT scale 24 (edge factor 16), the
batch of 4,096 uneven SBMs, plain-vs-gated comparisons, and the sequential CPU
oracle timed on bounded samples of these workloads.
"""
import argparse
import json
import os
import subprocess
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0


def library_digest():
    """sha256[:16] of the HIP library sources (the state byte counters were taken on)."""
    import hashlib
    h = hashlib.sha256()
    src = ROOT / "paper_2312_08140_amd" / "csrc" / "lpa"
    for f in sorted(list(src.glob("*.hip")) + list(src.glob("*.hpp")), key=lambda p: str(p)):
        h.update(f.read_bytes())
    return h.hexdigest()[:16]


DEFAULT_BINS = [4, 16, 64, 256, 1024, 4096]  # the library's default degree limits of bins 0-5
DEFAULT_CONFIG = {"variants": [0] * 6, "schedule": [16, 2, 4], "bins": DEFAULT_BINS, "hubs_last": 0, "snapshot": 0}


def profiled_config(workload):
    """The configuration (variants, schedule, bins, hubs_last, snapshot) the committed byte
    counters were taken with, when the library sources still match them; else None."""
    try:
        for line in (ROOT / "profiles" / f"{workload}_async_hbm_traffic.md").read_text().splitlines():
            if line.startswith("machine-readable: "):
                d = json.loads(line[len("machine-readable: "):])
                if d.get("sources") == library_digest():
                    return {"variants": d["variants"], "schedule": d["schedule"], "bins": d.get("bins", DEFAULT_BINS),
                            "hubs_last": d.get("hubs_last", 0), "snapshot": d.get("snapshot", 0)}
    except OSError:
        pass
    return None


CONFIG_KEYS = ("variants", "schedule", "bins", "hubs_last", "snapshot")


def same_config(a, b):
    return all(a.get(k, DEFAULT_CONFIG[k]) == b.get(k, DEFAULT_CONFIG[k]) for k in CONFIG_KEYS)


def measured_traffic(kernel, tuned, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None when the kernels or their configuration changed since the counters were taken."""
    try:
        for line in (ROOT / "profiles" / f"{workload}_async_hbm_traffic.md").read_text().splitlines():
            if line.startswith("machine-readable: "):
                d = json.loads(line[len("machine-readable: "):])
                if d.get("sources") != library_digest():
                    return None
                if tuned is None or not same_config(d, tuned):
                    return None
                return d["bytes_per_launch"].get(kernel)
    except OSError:
        return None
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(st):
    """Algorithmic bytes each kernel kind moved over a run.

    Scan kernels, per processed vertex: frontier entry 4 + row offset 8 +
    own label 4; per stored entry: index 4 + weight (packed size) + gathered
    neighbour label 4; per changed vertex: label write 4; per neighbour mark 1.
    Compaction: list entry 4 + flag 1 per listed vertex, flag clear 1 +
    frontier write 4 per taken vertex.  Snapshot first sweep ("first"): as a
    scan kernel, except that a neighbour id (4) is read only where the kernel
    read one.
    """
    wb = st["weight_bytes"]
    out = {}
    for b in range(7):
        byt = (st["bin_vertices"][b] * 16 + st["bin_edges"][b] * (8 + wb) + st["bin_changed"][b] * 4 +
               st["bin_marks"][b])
        out["hub_chunk" if b == 6 else f"bin{b}"] = byt
    out["compact"] = st["compact_listed"] * 5 + st["compact_taken"] * 5
    out["first"] = (st.get("first_vertices", 0) * 16 + st.get("first_edges", 0) * (4 + wb) +
                    st.get("first_reads", 0) * 4 + st.get("first_changed", 0) * 4 + st.get("first_marks", 0))
    return out


def _sbm1m(mu, seed, n=1_000_000, k=1000, d=32.0):
    from paper_2312_08140_amd import graphgen
    return graphgen.sbm(n, k, d * (1 - mu) / (n // k - 1), d * mu / (n - n // k), seed=seed)


def _median_runs(G, tau, max_iters, flags, out, k):
    from paper_2312_08140_amd import abi
    G.run(tau, max_iters, abi.LPA_MODE_ASYNC, True, flags=flags, labels_out=out)
    ms, st = [], None
    for _ in range(k):
        _, st = G.run(tau, max_iters, abi.LPA_MODE_ASYNC, True, flags=flags, labels_out=out)
        ms.append(st["total_ms"])
    return float(np.median(ms)), st


def _compare(G, gate_info, tau, max_iters, out, truth=None, plain=None):
    """Plain vs gated time-to-converge (median of 5 runs each) on one handle.
    A gated run ends with its verification sweep; the plain run is reported
    as is and also with that verification sweep (a verified fixed point,
    which the asynchronous mode must reach as well)."""
    import torch
    from paper_2312_08140_amd import abi
    if plain is None:
        p_ms, sp = _median_runs(G, tau, max_iters, 0, out, 5)
        lp = out.clone()
        qp = G.modularity(lp)
    else:
        p_ms, sp, lp, qp = plain
    pv_ms, spv = _median_runs(G, tau, max_iters, abi.LPA_FLAG_VERIFY, out, 5)
    G.gate_load(gate_info["params"], gate_info["threshold"])
    snap = G.schedule()[5]
    G.set_first_sweep(0)  # gated runs: the first sweep the gate was traced with
    g_ms, sg = _median_runs(G, tau, max_iters, abi.LPA_FLAG_GATE, out, 5)
    G.set_first_sweep(snap)
    lg = out.clone()
    qg = G.modularity(lg)
    r = {"plain_ms": round(p_ms, 3), "plain_verified_ms": round(pv_ms, 3), "gated_ms": round(g_ms, 3),
         "speedup": round(p_ms / g_ms, 3), "speedup_vs_verified_plain": round(pv_ms / g_ms, 3),
         "q_plain": round(qp, 6), "q_gated": round(qg, 6), "q_loss": round(qp - qg, 6),
         "nmi_plain_vs_gated": round(abi.nmi(lp, lg), 6), "verified": bool(sg["verified"]),
         "plain_verified": bool(spv["verified"]),
         "sweeps_plain": sp["iterations"], "sweeps_gated": sg["iterations"],
         "processed_plain": int(sum(sp["frontier"])),
         "processed_gated": int(sum(sg["frontier"])), "gated_out": int(sum(sg["gated_out"])),
         "verify_changed": int(sg["verify_changed"]),
         "entries_plain": int(sum(sp["edges_scanned"])),
         "entries_plain_verified": int(sum(spv["edges_scanned"]) + spv["verify_edges_scanned"]),
         "entries_gated": int(sum(sg["edges_scanned"]) + sg["verify_edges_scanned"])}
    if truth is not None:
        t = torch.from_numpy(truth.astype(np.int32)).cuda()
        r["nmi_truth_plain"] = round(abi.nmi(lp, t), 6)
        r["nmi_truth_gated"] = round(abi.nmi(lg, t), 6)
    return r


def _traces(graphs, cfg, probability, tau, max_iters):
    """(features, targets) of traced plain runs, every handle configured like
    the ones the gate serves (the schedule shapes the label dynamics)."""
    from paper_2312_08140_amd import abi
    xs, ys = [], []
    for make in graphs:
        g = make()
        if hasattr(g.offsets, "data_ptr"):
            H = abi.LPAGraph(n=g.n, offsets=g.offsets, indices=g.indices, weights=g.weights)
        else:
            H = abi.LPAGraph(g)
        if cfg == "tune":
            H.autotune(tau, max_iters, abi.LPA_MODE_ASYNC)
        elif cfg is not None:
            _apply(H, cfg)
        H.set_first_sweep(0)  # see gate_comparison
        H.set_trace(1 << 24, probability)
        H.run(tau, max_iters, abi.LPA_MODE_ASYNC, True, flags=abi.LPA_FLAG_TRACE)
        x, y = H.gate_trace()
        H.close()
        del g, H
        _release_cached()
        xs.append(x)
        ys.append(y)
    return np.concatenate(xs), np.concatenate(ys)


def _release_cached():
    """Device memory torch keeps cached goes back to the driver, where the
    library's own allocations can use it."""
    import torch
    torch.cuda.empty_cache()


def gate_comparison(args, G, runs, out, tuned, sec=None):
    """Learned active-set gate vs plain pruning.  The gate is trained on traces
    of 64 seeded plain runs - 32 SBM-1M graphs (seeds 100-131, mixing cycling
    0.1-0.4) for the SBM network and 32 R-MAT scale-24 graphs (seeds 100-131)
    for each R-MAT network (one per configuration it gates, traced under that
    configuration) - disjoint from the evaluation graphs; it is then
    compared with plain runs on SBM-1M (seed 1, mixing 0.1-0.4), on R-MAT-24
    (seed 1) and on the headline graph.  Training is outside every timed run.
    Traces and gated runs leave the snapshot first sweep off (every first-sweep
    kernel reads the labels as the schedule delivers them): after a snapshot
    sweep most labels still change in the next sweep, which leaves the gate
    little to skip; plain runs keep their tuned configuration."""
    import torch
    from paper_2312_08140_amd import abi, gate, graphgen
    res = {}
    # every SBM handle is tuned on its own graph (the quality guard of the
    # autotuner then holds per mixing level), training handles included
    sbm_cfg = None if args.no_tune else "tune"
    t = time.time()
    X, y = _traces([lambda i=i, mu=mu: _sbm1m(mu, 100 + i) for i, mu in enumerate((0.1, 0.2, 0.3, 0.4) * 8)],
                   sbm_cfg, 0.1, args.tau, args.max_iters)
    t_tr = time.time() - t
    info = sbm_info = gate.train(X, y, epochs=4, batch=4096, lr=1e-3, recall=0.98, seed=0)
    res["sbm_gate"] = {"train_runs": 32, "trace_config": "each handle autotuned" if sbm_cfg else "default",
                       "samples": int(len(y)),
                       "positive_share": round(float(y.mean()), 4), "threshold": round(info["threshold"], 6),
                       "holdout_recall": round(info["holdout_recall"], 4),
                       "holdout_skip": round(info["holdout_skip"], 4),
                       "loss": [round(float(v), 5) for v in info["losses"]], "trace_seconds": round(t_tr, 2),
                       "seconds": round(time.time() - t, 2)}
    log(f"sbm gate: {res['sbm_gate']}")
    rows = []
    for mu in (0.1, 0.2, 0.3, 0.4):
        s = _sbm1m(mu, 1)
        H = abi.LPAGraph(s)
        o = torch.empty(s.n, dtype=torch.int32, device="cuda:0")
        if sbm_cfg is not None:
            H.autotune(args.tau, args.max_iters, abi.LPA_MODE_ASYNC)
        r = _compare(H, info, args.tau, args.max_iters, o, truth=graphgen.sbm_truth(s.n, 1000))
        r["mu"] = mu
        r["schedule"] = list(H.schedule())
        rows.append(r)
        log(f"sbm1m mu={mu}: {r}")
        H.close()
    res["sbm1m"] = rows
    # one R-MAT network per configuration it is deployed with: the traces are
    # recorded under the configuration (bins, bin order, snapshot first sweep)
    # of the runs it will gate, since those set the label dynamics it learns
    rmat_cfgs = [("head", tuned)]
    if sec is not None:
        rmat_cfgs.insert(0, ("secondary", sec["tuning"]))
    gates = {}
    for name, cfg in rmat_cfgs:
        same = next((k for k, (c, _) in gates.items() if c is not None and cfg is not None and same_config(c, cfg)),
                    None)
        if same is not None or (cfg is None and gates):
            gates[name] = gates[same if same is not None else next(iter(gates))]
            continue
        t = time.time()
        X, y = _traces([lambda i=i: graphgen.rmat_device(24, 16, seed=100 + i, weighted=True) for i in range(32)],
                       cfg, 0.05, args.tau, args.max_iters)
        t_tr = time.time() - t
        info = gate.train(X, y, epochs=4, batch=4096, lr=1e-3, recall=0.98, seed=0)
        res[f"rmat_gate_{name}"] = {"train_runs": "32 R-MAT scale 24 edge factor 16, seeds 100-131",
                                    "trace_config": cfg, "samples": int(len(y)),
                                    "positive_share": round(float(y.mean()), 4),
                                    "threshold": round(info["threshold"], 6),
                                    "holdout_recall": round(info["holdout_recall"], 4),
                                    "holdout_skip": round(info["holdout_skip"], 4), "trace_seconds": round(t_tr, 2),
                                    "seconds": round(time.time() - t, 2)}
        log(f"rmat gate ({name} configuration): {res[f'rmat_gate_{name}']}")
        gates[name] = (cfg, info)
    if sec is not None:
        d = graphgen.rmat_device(args.secondary_scale, args.secondary_edge_factor, seed=args.seed, weighted=True)
        H = abi.LPAGraph(n=d.n, offsets=d.offsets, indices=d.indices, weights=d.weights)
        _apply(H, sec["tuning"])
        o = torch.empty(d.n, dtype=torch.int32, device="cuda:0")
        r = _compare(H, gates["secondary"][1], args.tau, args.max_iters, o)
        res[f"rmat{args.secondary_scale}"] = r
        log(f"rmat{args.secondary_scale} gated: {r}")
        H.close()
        del d
    info = gates["head"][1]
    p_ms = float(np.median([r["total_ms"] for r in runs]))
    lp = out.clone()
    G.run(args.tau, args.max_iters, abi.LPA_MODE_ASYNC, True, labels_out=lp)
    r = _compare(G, info, args.tau, args.max_iters, out, plain=(p_ms, runs[-1], lp, G.modularity(lp)))
    res[f"rmat{args.scale}"] = r
    log(f"rmat{args.scale} gated: {r}")
    return res, sbm_info


def batch_workload(args, gate_info=None):
    """Many independent SBMs of uneven size in one handle (block-diagonal CSR,
    each graph with its own stop test, every run one HIP graph launch):
    default tuning vs autotuned, asynchronous and deterministic; with a gate
    (the SBM network of gate_comparison, trained on SBM-1M traces), plain vs
    gated, every graph verified on its own."""
    import torch
    from paper_2312_08140_amd import abi, graphgen
    t = time.time()
    csr, vptr = graphgen.sbm_batch(args.batch, master_seed=7, seed_base=10000)
    log(f"batch of {args.batch} SBMs: n={csr.n} m={csr.m} in {time.time() - t:.1f}s")
    B = abi.LPABatch(csr, vptr)
    out = torch.empty(csr.n, dtype=torch.int32, device="cuda:0")
    res = {"workload": f"sbm_batch{args.batch}_seed7", "graphs": args.batch, "n": csr.n, "m": csr.m}

    def timed(mode, label):
        B.run(args.tau, args.max_iters, mode, True, labels_out=out)
        ms, st = [], None
        for _ in range(5):
            _, st = B.run(args.tau, args.max_iters, mode, True, labels_out=out)
            ms.append(st["total_ms"])
        it, conv = B.graph_stats()
        med = float(np.median(ms))
        r = {"time_ms": round(med, 3), "entries_per_s": round(sum(st["edges_scanned"]) / (med * 1e-3), 1),
             "m_over_time": round(csr.m / (med * 1e-3), 1), "sweeps_max": int(it.max()),
             "sweeps_mean": round(float(it.mean()), 3), "graphs_converged": int(conv.sum()),
             "modularity_union": round(B.modularity(out), 6)}
        log(f"batch {label}: {r}")
        return r
    res["async_default"] = timed(abi.LPA_MODE_ASYNC, "async default")
    res["det_default"] = timed(abi.LPA_MODE_DETERMINISTIC, "det default")
    if not args.no_tune:
        t = time.time()
        v, _, sch, lim = B.autotune(args.tau, args.max_iters, abi.LPA_MODE_ASYNC)
        res["tuning"] = {"variants": [int(x) for x in v], "schedule": list(sch), "bins": list(lim),
                         "seconds": round(time.time() - t, 2)}
        res["async_tuned"] = timed(abi.LPA_MODE_ASYNC, "async tuned")
    if gate_info is not None:
        r = _compare(B, gate_info, args.tau, args.max_iters, out)
        ok, vch = B.verify_stats()
        it, conv = B.graph_stats()
        r.update({"graphs_verified": int(ok.sum()), "graphs_converged": int(conv.sum()),
                  "graph_sweeps_mean": round(float(it.mean()), 3)})
        res["gated"] = r
        log(f"batch gated: {r}")
    if not args.no_tune:
        t = time.time()
        dv, _, _, dlim = B.autotune(args.tau, args.max_iters, abi.LPA_MODE_DETERMINISTIC)
        res["det_tuning"] = {"variants": [int(x) for x in dv], "bins": list(dlim), "seconds": round(time.time() - t, 2)}
        res["det_tuned"] = timed(abi.LPA_MODE_DETERMINISTIC, "det tuned")
    B.close()
    return res, (csr, vptr)


def _stats_summary(runs, m):
    ttc = [r["total_ms"] for r in runs]
    sweep0 = [r["ms"][0] for r in runs if r["iterations"] > 0]
    return {"time_to_converge_ms": {"median": round(float(np.median(ttc)), 3), "min": round(float(np.min(ttc)), 3)},
            "sweeps": runs[0]["iterations"],
            "sweep0_edges_per_s": round(m / (np.median(sweep0) * 1e-3), 1) if sweep0 else None,
            "m_over_time_to_converge": round(m / (np.median(ttc) * 1e-3), 1)}


def _apply(G, cfg):
    G.set_variants(cfg["variants"])
    G.set_async_schedule(*cfg["schedule"])
    G.set_bins(cfg["bins"])
    G.set_bin_order(cfg.get("hubs_last", 0))
    G.set_first_sweep(cfg.get("snapshot", 0))


def tune_async(args, G, workload):
    """Autotuned asynchronous configuration of handle G (or the one given on
    the command line); when the autotuner's near-tie pick differs from the
    configuration the committed byte counters of this workload were taken
    with, that one is timed instead so the counters apply."""
    from paper_2312_08140_amd import abi
    if args.variants or args.schedule or args.bins or args.hubs_last or args.snapshot:
        v = [int(x) for x in args.variants.split(",")] if args.variants else [0] * 6
        s = [int(x) for x in args.schedule.split(",")] if args.schedule else [16, 2, 4]
        lim = [int(x) for x in args.bins.split(",")] if args.bins else list(DEFAULT_BINS)
        tuned = {"variants": v, "schedule": s, "bins": lim, "hubs_last": int(args.hubs_last),
                 "snapshot": int(args.snapshot), "seconds": 0.0,
                 "given": True}
        _apply(G, tuned)
        return tuned
    if args.no_tune:
        return None
    t = time.time()
    variants, bin_ms, sched, lim = G.autotune(args.tau, args.max_iters, abi.LPA_MODE_ASYNC)
    tuned = {"variants": [int(v) for v in variants], "schedule": list(sched), "bins": list(lim),
             "hubs_last": G.schedule()[4], "snapshot": G.schedule()[5], "seconds": round(time.time() - t, 2),
             "source": "autotune"}
    prof = profiled_config(workload)
    if prof is not None and not same_config(prof, tuned):
        tuned["autotune_pick"] = {k: tuned[k] for k in CONFIG_KEYS}
        tuned.update(prof, source="autotune pick recorded with the profile")
        _apply(G, tuned)
    return tuned


def roofline_of(G, args, out, tuned, workload):
    """Per-kernel HIP-event timing run (eager launches on the library's stream)
    and the roofline of the dominant kernel on algorithmic bytes."""
    from paper_2312_08140_amd import abi
    _, kt = G.run(args.tau, args.max_iters, abi.LPA_MODE_ASYNC, True, flags=abi.LPA_FLAG_KERNEL_TIMING,
                  labels_out=out)
    kb = kernel_bytes(kt)
    kms = dict(kt["kernel_ms"])
    hub_ms = sum(kms.get(k, 0) for k in ("hub_plan", "hub_chunk", "hub_part", "hub_finish"))
    dominant = max(kms, key=lambda k: kms[k])
    per_kernel = {}
    for k, ms in kms.items():
        byt = kb.get(k, 0)
        ms_eff = hub_ms if k == "hub_chunk" else ms
        per_kernel[k] = dict(ms=round(ms, 4), launches=kt["kernel_launches"][k], bytes=int(byt),
                             gbs=round(byt / (ms_eff * 1e-3) / 1e9, 1) if byt and ms_eff > 0 else None)
    dom_bytes = kb.get(dominant, 0)
    dom_launches = kt["kernel_launches"][dominant]
    dom_ms = kms[dominant] / dom_launches
    achieved = (dom_bytes / dom_launches) / (dom_ms * 1e-3) / 1e9
    total_bytes = sum(kb.values())
    sweep_ms = sum(kt["ms"])
    return {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "bytes_per_launch": int(dom_bytes / dom_launches), "avg_launch_ms": round(dom_ms, 5),
            "traffic": measured_traffic(dominant, tuned, workload),
            "whole_sweep": {"bytes": int(total_bytes), "ms": round(sweep_ms, 3),
                            "achieved": round(total_bytes / (sweep_ms * 1e-3) / 1e9, 1),
                            "frac": round(total_bytes / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "per_kernel": per_kernel}


def storage_order_indices(d, with_offsets=False):
    """The neighbour indices as the library stores them: vertices renumbered
    in decreasing degree order (ties by id) and every row sorted by neighbour
    position.  Built with torch in chunks of at most 2^28 entries."""
    import torch
    n, m = d.n, d.m
    off = d.offsets.long()
    deg = off[1:] - off[:-1]
    order = torch.argsort(-deg, stable=True)
    rank = torch.empty(n, dtype=torch.int64, device=off.device)
    rank[order] = torch.arange(n, device=off.device)
    ndeg = deg[order]
    noff = torch.zeros(n + 1, dtype=torch.int64, device=off.device)
    noff[1:] = torch.cumsum(ndeg, 0)
    shift = max(1, (n - 1).bit_length())
    new_idx = torch.empty(m, dtype=torch.int32, device=off.device)
    hoff = noff.cpu().numpy()
    p = 0
    while p < n:
        q = max(p + 1, int(np.searchsorted(hoff, hoff[p] + (1 << 28), side="right")) - 1)
        q = min(q, n)
        e0, e1 = int(hoff[p]), int(hoff[q])
        if e1 > e0:
            row_of = torch.repeat_interleave(torch.arange(p, q, device=off.device), ndeg[p:q])
            src = off[order[row_of]] + (torch.arange(e1 - e0, device=off.device) - (noff[row_of] - e0))
            key = ((row_of - p) << shift) | rank[d.indices[src].long()]
            del row_of, src
            key = torch.sort(key)[0]
            new_idx[e0:e1] = (key & ((1 << shift) - 1)).to(torch.int32)
            del key
        p = q
    del rank, order, deg
    if with_offsets:
        return new_idx, noff, ndeg
    return new_idx


def gather_ceiling(d, reps=3, bins=None):
    """What a label gather alone costs on this graph: torch's index_select of a
    label array by the neighbour indices (4 B index read, 4 B label gather,
    4 B output write per entry) - in the generator's CSR order, in the order
    the library stores the graph (decreasing degree, sorted rows: the order its
    kernels gather in), and, where it fits, with all indices sorted (every
    gather then walks the label array in order).  A ceiling for any kernel
    that gathers one label per entry in that order.  With the bin degree limits,
    also the storage-order gather of each bin's entries on its own (the bins
    are contiguous ranges of that order)."""
    import torch
    C = torch.arange(d.n, dtype=torch.int32, device="cuda:0")
    res = {}

    def timed(idx, count=None):
        count = d.m if count is None else count
        out = torch.index_select(C, 0, idx)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            torch.index_select(C, 0, idx, out=out)
        e1.record()
        torch.cuda.synchronize()
        del out
        ms = e0.elapsed_time(e1) / reps
        return {"ms": round(ms, 3), "entries_per_s": round(count / (ms * 1e-3), 1),
                "gb_per_s_12B_per_entry": round(12 * count / (ms * 1e-3) / 1e9, 1)}
    res["csr_order"] = timed(d.indices)
    si, noff, ndeg = storage_order_indices(d, with_offsets=True)
    res["storage_order"] = timed(si)
    if bins is not None:
        # vertices of bin b: degree in (bins[b-1], bins[b]] (bin 0 from 1), hubs above bins[5]
        lims = [0] + list(bins)
        per = {}
        for name, lo, hi in [("hubs", lims[-1], None)] + [(f"bin{b}", lims[b], lims[b + 1]) for b in range(5, -1, -1)]:
            sel = (ndeg > lo) if hi is None else ((ndeg > lo) & (ndeg <= hi))
            nz = torch.nonzero(sel).flatten()
            if nz.numel() == 0:
                continue
            e0, e1 = int(noff[int(nz[0])]), int(noff[int(nz[-1]) + 1])
            if e1 > e0:
                per[name] = timed(si[e0:e1].contiguous(), e1 - e0)
                per[name]["entries"] = e1 - e0
        res["storage_order_by_bin"] = per
    del si, noff, ndeg
    torch.cuda.empty_cache()
    if d.m <= (1 << 30):
        srt = torch.sort(d.indices)[0]
        res["sorted_indices"] = timed(srt)
        del srt
    torch.cuda.empty_cache()
    return res


def deterministic_of(G, args, out, m, tuned):
    """The deterministic mode on its own tuning (colour class by colour class
    it prefers other bin limits and shapes; results do not depend on them)."""
    from paper_2312_08140_amd import abi
    t = time.time()
    det_tuning = None
    if tuned is not None and not tuned.get("given"):
        dv, _, _, dlim = G.autotune(args.tau, args.max_iters, abi.LPA_MODE_DETERMINISTIC)
        det_tuning = {"variants": [int(x) for x in dv], "bins": list(dlim), "seconds": round(time.time() - t, 2)}
    _, sd = G.run(args.tau, args.max_iters, abi.LPA_MODE_DETERMINISTIC, True, labels_out=out)
    q_det = G.modularity(out)
    runs = []
    for _ in range(3):
        _, sd2 = G.run(args.tau, args.max_iters, abi.LPA_MODE_DETERMINISTIC, True, labels_out=out)
        runs.append(sd2)
    det = dict(colouring_and_capture_ms=round(sd["setup_ms"], 1), colours=sd["num_colors"],
               modularity=round(q_det, 6), tuning=det_tuning, **_stats_summary(runs, m))
    det["edges_per_s"] = round(sum(runs[-1]["edges_scanned"]) / (runs[-1]["total_ms"] * 1e-3), 1)
    if tuned is not None:  # back to the asynchronous tuning
        _apply(G, tuned)
    return det, q_det


def timed_async(G, args, out, steps, warmup):
    from paper_2312_08140_amd import abi
    import torch
    for _ in range(warmup):
        G.run(args.tau, args.max_iters, abi.LPA_MODE_ASYNC, True, labels_out=out)
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = G.run(args.tau, args.max_iters, abi.LPA_MODE_ASYNC, True, labels_out=out)
        runs.append(st)
    torch.cuda.synchronize()
    return runs, time.perf_counter() - t0


def secondary_rmat(args):
    """R-MAT scale 24, edge factor 16 (the mid-size configuration): asynchronous
    and deterministic figures, tuned like the headline."""
    import torch
    from paper_2312_08140_amd import abi, graphgen
    t = time.time()
    d = graphgen.rmat_device(args.secondary_scale, args.secondary_edge_factor, seed=args.seed, weighted=True)
    G = abi.LPAGraph(n=d.n, offsets=d.offsets, indices=d.indices, weights=d.weights)
    torch.cuda.synchronize()
    wl = f"rmat{args.secondary_scale}"
    res = {"workload": f"rmat{args.secondary_scale}_ef{args.secondary_edge_factor}_w1-8_seed{args.seed}", "n": d.n,
           "m": d.m, "generate_and_create_s": round(time.time() - t, 2)}
    sub = argparse.Namespace(**{**vars(args), "variants": None, "schedule": None, "bins": None, "hubs_last": 0,
                                "snapshot": 0})
    tuned = tune_async(sub, G, wl)
    out = torch.empty(d.n, dtype=torch.int32, device="cuda:0")
    runs, wall = timed_async(G, args, out, 10, 2)
    res.update(value=round(sum(sum(r["edges_scanned"]) for r in runs) / wall, 1),
               ms_per_run=round(wall * 1e3 / len(runs), 3), modularity=round(G.modularity(out), 6), tuning=tuned,
               **_stats_summary(runs, d.m))
    lab_a = out.clone()
    _, sv = G.run(args.tau, args.max_iters, abi.LPA_MODE_ASYNC, True, flags=abi.LPA_FLAG_VERIFY, labels_out=out)
    res["verified"] = bool(sv["verified"])
    res["verify_changed"] = int(sv["verify_changed"])
    res["roofline"] = roofline_of(G, args, out, tuned, wl)
    res["roofline"]["gather_ceiling"] = gather_ceiling(d, bins=tuned["bins"] if tuned else None)
    if not args.no_det:
        res["deterministic"], q_det = deterministic_of(G, args, out, d.m, tuned)
        res["q_async_minus_det"] = round(res["modularity"] - q_det, 6)
    log(f"{res['workload']}: {res['value'] / 1e9:.1f} G edges/s, {res['ms_per_run']} ms/run")
    G.close()
    return res, d, lab_a


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return None


def cpu_baselines(args, head_host, sec_host, batch_in):
    """The sequential C oracle (one core; it is sequential by definition) on
    bounded samples: sweep 0 of the headline graph over a seeded quarter of
    its vertices (the others start unflagged and come first in the order, so
    the marks the quarter writes land on vertices the sweep has passed and the
    sweep processes the quarter alone), the
    mid-size R-MAT to convergence in id order and in (colour, id) order, and
    the 4,096-graph batch to convergence spread over every host core (one
    graph per thread).  Then the multicore comparator in the paper's design
    (OpenMP, every host core) to convergence on both R-MAT graphs, strict and
    non-strict."""
    import oracle
    from paper_2312_08140_amd import cpu_lpa
    res = {"cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if head_host is not None:
        fl = (np.random.default_rng(12345).random(head_host.n) < 0.25).astype(np.uint8)
        order = np.concatenate([np.flatnonzero(fl == 0), np.flatnonzero(fl == 1)]).astype(np.int32)
        t = time.perf_counter()
        r = oracle.lpa(head_host, order=order, tau=args.tau, max_iters=1, prune=True, init_flags=fl)
        dt = time.perf_counter() - t
        res["headline_sweep0"] = {"value": round(float(r["scanned"].sum()) / dt, 1), "unit": "edges/s", "cores": 1,
                                  "seconds": round(dt, 2), "entries": int(r["scanned"].sum()),
                                  "vertices": int(r["processed"].sum()),
                                  "sample": "sweep 0 of the headline graph over a seeded random quarter of the "
                                            "vertices in id order, placed after the other (unflagged) vertices"}
        log(f"cpu oracle headline sweep 0: {res['headline_sweep0']}")
    if sec_host is not None:
        rows = {}
        t = time.perf_counter()
        r = oracle.lpa(sec_host, tau=args.tau, max_iters=args.max_iters, prune=True)
        dt = time.perf_counter() - t
        rows["id_order"] = {"seconds": round(dt, 2), "sweeps": r["iterations"], "entries": int(r["scanned"].sum()),
                            "edges_per_s": round(float(r["scanned"].sum()) / dt, 1),
                            "m_over_time_to_converge": round(sec_host.m / dt, 1)}
        t = time.perf_counter()
        col, nc = oracle.color(sec_host, 0)
        order = oracle.color_order(col, nc)
        tc = time.perf_counter() - t
        t = time.perf_counter()
        r = oracle.lpa(sec_host, order=order, tau=args.tau, max_iters=args.max_iters, prune=True)
        dt = time.perf_counter() - t
        rows["colour_order"] = {"seconds": round(dt, 2), "colouring_s": round(tc, 2), "sweeps": r["iterations"],
                                "entries": int(r["scanned"].sum()),
                                "edges_per_s": round(float(r["scanned"].sum()) / dt, 1),
                                "m_over_time_to_converge": round(sec_host.m / dt, 1)}
        res["secondary_to_convergence"] = rows
        log(f"cpu oracle secondary: {rows}")
    if batch_in is not None:
        g, vptr = batch_in
        threads = os.cpu_count() or 1
        t = time.perf_counter()
        ref = oracle.lpa_batch(g, vptr, deterministic=False, tau=args.tau, max_iters=args.max_iters, threads=threads)
        dt = time.perf_counter() - t
        ent = int(sum(int(r["scanned"].sum()) for r in ref))
        res["batch_to_convergence"] = {"seconds": round(dt, 2), "cores": threads, "entries": ent,
                                       "edges_per_s": round(ent / dt, 1), "m_over_time": round(g.m / dt, 1),
                                       "sample": f"{len(vptr) - 1} graphs, id order, one graph per thread"}
        log(f"cpu oracle batch: {res['batch_to_convergence']}")
    comp = {}
    for name, g in (("headline", head_host), ("secondary", sec_host)):
        if g is None:
            continue
        for strict in (True, False):
            r = cpu_lpa.lpa(g, tau=args.tau, max_iters=args.max_iters, prune=True, strict=strict, threads=0)
            ent = int(r["scanned"].sum())
            comp[f"{name}_{'strict' if strict else 'non_strict'}"] = {
                "seconds": round(r["seconds"], 3), "threads": r["threads"], "sweeps": r["iterations"],
                "converged": r["converged"], "entries": ent, "edges_per_s": round(ent / r["seconds"], 1),
                "m_over_time_to_converge": round(g.m / r["seconds"], 1),
                "modularity": round(oracle.modularity(g, r["labels"]), 6)}
            log(f"cpu comparator {name} strict={strict}: {comp[f'{name}_' + ('strict' if strict else 'non_strict')]}")
    res["multicore_comparator"] = comp
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--edge-factor", type=int, default=32)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tau", type=float, default=0.05)
    ap.add_argument("--max-iters", type=int, default=20)
    ap.add_argument("--secondary-scale", type=int, default=24, help="mid-size R-MAT scale (0: skip)")
    ap.add_argument("--secondary-edge-factor", type=int, default=16)
    ap.add_argument("--no-det", action="store_true", help="skip the deterministic-mode figures")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for hardware byte counters)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default schedule and kernel shapes")
    ap.add_argument("--variants", default=None,
                    help="kernel shape per degree bin of the headline graph, e.g. 2,1,1,2,2,1 (instead of autotuning)")
    ap.add_argument("--bins", default=None,
                    help="degree limits of bins 0-5, e.g. 4,16,64,256,1024,4096 (instead of autotuning)")
    ap.add_argument("--schedule", default=None,
                    help="asynchronous schedule early_steps,early_sweeps,late_steps (instead of autotuning)")
    ap.add_argument("--hubs-last", type=int, default=0, help="with the options above: the hub bin runs last (1)")
    ap.add_argument("--snapshot", type=int, default=0,
                    help="with the options above: the first sweep reads a snapshot of the initial labels (1)")
    ap.add_argument("--no-gate", action="store_true", help="skip the plain-vs-gated comparison")
    ap.add_argument("--batch", type=int, default=4096,
                    help="batched workload of this many uneven SBMs (4096 = the benchmark batch; 0: skip)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2312_08140_amd import abi, graphgen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_start = time.time()
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t = time.time()
    d = graphgen.rmat_device(args.scale, args.edge_factor, seed=args.seed, weighted=True)
    gen_s = time.time() - t
    n_head, m_head = d.n, d.m
    log(f"generated R-MAT scale {args.scale} on the GPU: n={d.n} m={d.m} in {gen_s:.1f}s")
    t = time.time()
    G = abi.LPAGraph(n=d.n, offsets=d.offsets, indices=d.indices, weights=d.weights)
    torch.cuda.synchronize()
    create_s = time.time() - t
    log(f"lpa_create in {create_s:.1f}s")
    workload = f"rmat{args.scale}"
    A = abi.LPA_MODE_ASYNC
    out = torch.empty(d.n, dtype=torch.int32, device="cuda:0")
    tuned = tune_async(args, G, workload)
    log(f"autotune: {tuned}")

    runs, wall = timed_async(G, args, out, args.steps, args.warmup)
    scanned = sum(sum(r["edges_scanned"]) for r in runs)
    value = scanned / wall
    ms_per_step = wall * 1000.0 / args.steps
    q_async = G.modularity(out)
    log(f"async: {value / 1e9:.2f} G edges/s, {ms_per_step:.2f} ms/run, sweeps {runs[0]['iterations']}, Q {q_async:.6f}")
    lab_async = out.clone()
    _, sv = G.run(args.tau, args.max_iters, A, True, flags=abi.LPA_FLAG_VERIFY, labels_out=out)
    verify = {"verified": bool(sv["verified"]), "verify_changed": int(sv["verify_changed"]),
              "modularity": round(G.modularity(out), 6)}
    roofline = roofline_of(G, args, out, tuned, workload)
    log(f"dominant kernel {roofline['kernel']}: {roofline['achieved']:.0f} GB/s ({roofline['frac'] * 100:.1f}% of peak)")
    roofline["gather_ceiling"] = gather_ceiling(d, bins=tuned["bins"] if tuned else None)
    log(f"gather ceiling: {roofline['gather_ceiling']}")

    det, q_det = (None, None)
    if not args.no_det:
        det, q_det = deterministic_of(G, args, out, d.m, tuned)
        log(f"det: {det}")

    secondary, sec_dev = None, None
    if args.secondary_scale:
        secondary, sec_dev, _ = secondary_rmat(args)

    gated, sbm_info = None, None
    if not args.no_gate:
        gated, sbm_info = gate_comparison(args, G, runs, out, tuned, secondary)

    batch, batch_in = None, None
    if args.batch:
        batch, batch_in = batch_workload(args, sbm_info)

    head_host = None
    if not args.no_cpu:
        G.close()
        G = None
        head_host = d.to_host()
    del d
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        sec_host = sec_dev.to_host() if sec_dev is not None else None
        del sec_dev
        extra = cpu_baselines(args, head_host, sec_host, batch_in)
        hs = extra.get("headline_sweep0")
        cpu = {"value": hs["value"] if hs else None, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "sequential C oracle (one thread), sweep 0 of the headline graph over a seeded random "
                         "quarter of its vertices", **extra}

    res = {
        "metric": "LPA edges/s per sweep + time-to-converge at equal modularity, plain vs gated",
        "value": round(value, 1), "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_ef{args.edge_factor}_w1-8_seed{args.seed}", "n": n_head,
                   "m": m_head, "mode": "async", "prune": True, "tau": args.tau, "max_iters": args.max_iters},
        "modularity": round(q_async, 6), "verification": verify,
        "q_async_minus_det": round(q_async - q_det, 6) if q_det is not None else None,
        **_stats_summary(runs, m_head),
        "generate_s": round(gen_s, 2), "create_s": round(create_s, 2),
        "deterministic": det, "tuning": tuned, "gated": gated, "secondary": secondary, "batch": batch,
        "roofline": roofline, "cpu_baseline": cpu, "bench_seconds": round(time.time() - t_start, 1),
    }
    print(json.dumps(res), flush=True)
    if G is not None:
        G.close()


if __name__ == "__main__":
    main()
