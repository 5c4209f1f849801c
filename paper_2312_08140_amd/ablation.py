"""Parameter ablation of the method on one MI355X, with a low-degree workload.

The paper measures its optimisations one at a time over its 13 graphs
(Section 4.1, Figure rak-opt): the tolerance (4.1.3), the iteration cap
(4.1.2), vertex pruning (4.1.4) and strict against non-strict LPA (4.1.5),
and it reports that low-degree graphs cost more time per edge (Section 5.2).
This module runs the same study on synthetic stand-ins, on the GPU library
and on the multicore CPU comparator:

* ``rmat24``   R-MAT scale 24, edge factor 16, weights 1..8 (web-graph stand-in);
* ``sbm1m``    SBM, 10^6 vertices in 1,000 blocks, average degree 32, mixing 0.2
               (community-structured social-graph stand-in);
* ``road``     the 8192 x 6144 lattice with every edge kept with probability
               0.55: 50.3 M vertices, average degree 2.2 (stand-in for the
               road and k-mer graphs, e.g. europe_osm: 50.9 M vertices, 108 M
               edges, average degree 2.1).

Every row is the median of three runs to convergence (asynchronous mode, the
handle tuned once by ``lpa_autotune`` at the base setting) with its sweeps,
entries scanned, modularity and time per scanned entry.  Usage:
``python -m paper_2312_08140_amd.ablation [--out FILE]`` (one JSON document).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


BASE = dict(tau=0.05, max_iters=20, prune=True, strict=True)
VARIANTS = [
    ("base", {}),
    ("tau_0.1", dict(tau=0.1)),
    ("tau_0.01", dict(tau=0.01)),
    ("tau_1e-5", dict(tau=1e-5)),
    ("max_iters_5", dict(max_iters=5)),
    ("max_iters_10", dict(max_iters=10)),
    ("max_iters_50", dict(max_iters=50)),
    ("no_pruning", dict(prune=False)),
    ("non_strict", dict(strict=False)),
]


def _graphs(which):
    from paper_2312_08140_amd import graphgen as gg
    out = {}
    if "rmat24" in which:
        out["rmat24"] = gg.rmat_device(24, 16, seed=1, weighted=True)
    if "sbm1m" in which:
        n, k, d, mu = 1_000_000, 1000, 32.0, 0.2
        out["sbm1m"] = gg.sbm(n, k, d * (1 - mu) / (n // k - 1), d * mu / (n - n // k), seed=1)
    if "road" in which:
        out["road"] = gg.grid(8192, 6144, 0.55, seed=1)
    return out


def gpu_rows(name, g, reps=3):
    import torch
    from paper_2312_08140_amd import abi
    if hasattr(g.offsets, "data_ptr"):
        G = abi.LPAGraph(n=g.n, offsets=g.offsets, indices=g.indices, weights=g.weights)
    else:
        G = abi.LPAGraph(g)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    t = time.time()
    v, _, sch, lim = G.autotune(BASE["tau"], BASE["max_iters"], abi.LPA_MODE_ASYNC)
    full = G.schedule()
    tuning = {"variants": [int(x) for x in v], "schedule": list(sch), "bins": list(lim), "hubs_last": full[4],
              "snapshot": full[5], "seconds": round(time.time() - t, 2)}
    rows = {}
    for label, change in VARIANTS + [("untuned_defaults", {}), ("deterministic", {})]:
        p = dict(BASE, **change)
        mode = abi.LPA_MODE_DETERMINISTIC if label == "deterministic" else abi.LPA_MODE_ASYNC
        if label == "untuned_defaults":
            G.set_variants(None)
            G.set_bins(None)
            G.set_async_schedule()
            G.set_bin_order(0)
            G.set_first_sweep(0)
        flags = 0 if p["strict"] else abi.LPA_FLAG_NONSTRICT
        G.run(p["tau"], p["max_iters"], mode, p["prune"], flags=flags, labels_out=out)  # warm-up
        ms, st = [], None
        for _ in range(reps):
            _, st = G.run(p["tau"], p["max_iters"], mode, p["prune"], flags=flags, labels_out=out)
            ms.append(st["total_ms"])
        t_ms = float(np.median(ms))
        ent = int(sum(st["edges_scanned"]))
        rows[label] = {"time_ms": round(t_ms, 3), "sweeps": st["iterations"], "converged": st["converged"],
                       "entries_scanned": ent, "ns_per_entry": round(t_ms * 1e6 / max(ent, 1), 4),
                       "m_over_time": round(g.m / (t_ms * 1e-3), 1), "modularity": round(G.modularity(out), 6),
                       "communities": int(torch.unique(out).numel())}
        log(f"gpu {name} {label}: {rows[label]}")
    G.close()
    return {"n": g.n, "m": g.m, "tuning": tuning, "rows": rows}


def cpu_rows(name, g, threads=0):
    import oracle
    from paper_2312_08140_amd import cpu_lpa
    rows = {}
    for label, change in [("base", {}), ("no_pruning", dict(prune=False)), ("non_strict", dict(strict=False))]:
        p = dict(BASE, **change)
        r = cpu_lpa.lpa(g, tau=p["tau"], max_iters=p["max_iters"], prune=p["prune"], strict=p["strict"],
                        threads=threads)
        ent = int(r["scanned"].sum())
        rows[label] = {"seconds": round(r["seconds"], 3), "sweeps": r["iterations"], "entries_scanned": ent,
                       "ns_per_entry": round(r["seconds"] * 1e9 / max(ent, 1), 3),
                       "m_over_time": round(g.m / r["seconds"], 1), "threads": r["threads"],
                       "modularity": round(oracle.modularity(g, r["labels"]), 6)}
        log(f"cpu {name} {label}: {rows[label]}")
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", default="rmat24,sbm1m,road")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--threads", type=int, default=0, help="CPU comparator threads (0: OpenMP default)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available(), "the ablation needs a GPU"
    res = {"settings": {"base": BASE, "variants": [v[0] for v in VARIANTS] + ["untuned_defaults", "deterministic"]},
           "gpu": {}, "cpu": {}}
    graphs = _graphs(args.graphs.split(","))
    for name, g in graphs.items():
        log(f"{name}: n={g.n} m={g.m}")
        res["gpu"][name] = gpu_rows(name, g)
        if not args.no_cpu:
            host = g.to_host() if hasattr(g, "to_host") else g
            res["cpu"][name] = cpu_rows(name, host, args.threads)
    txt = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(txt + "\n")
    print(txt, flush=True)


if __name__ == "__main__":
    main()
