"""Host logic of bench.py (no GPU): the one-GPU guard, the byte model of the
roofline, and the rule that measured traffic is reported only for the library
sources and tuned configuration the committed byte counters were taken with."""
import json
import subprocess
import sys

import pytest

import bench

ROOT = bench.ROOT


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _stats(weight_bytes=1):
    z = [0] * 7
    st = dict(weight_bytes=weight_bytes, bin_vertices=list(z), bin_edges=list(z), bin_changed=list(z),
              bin_marks=list(z), compact_listed=0, compact_taken=0)
    return st


def test_kernel_bytes_model():
    """Per processed vertex 16 B, per scanned entry 8 B + the packed weight,
    per change 4 B, per mark 1 B; compaction 5 B per listed and per taken
    vertex; bin 6 is reported as the hub scan; the snapshot first sweep
    counts 4 B + the weight per entry and 4 B per neighbour id it read."""
    st = _stats(weight_bytes=1)
    st["bin_vertices"][2] = 10
    st["bin_edges"][2] = 100
    st["bin_changed"][2] = 3
    st["bin_marks"][2] = 7
    st["bin_vertices"][6] = 1
    st["bin_edges"][6] = 5000
    st["compact_listed"] = 11
    st["compact_taken"] = 4
    b = bench.kernel_bytes(st)
    assert b["bin2"] == 10 * 16 + 100 * 9 + 3 * 4 + 7
    assert b["hub_chunk"] == 16 + 5000 * 9
    assert b["bin0"] == 0
    assert b["compact"] == 11 * 5 + 4 * 5
    assert bench.kernel_bytes(_stats(weight_bytes=0))["bin3"] == 0
    assert b["first"] == 0
    st["first_vertices"], st["first_edges"], st["first_reads"], st["first_changed"], st["first_marks"] = 3, 40, 6, 2, 5
    assert bench.kernel_bytes(st)["first"] == 3 * 16 + 40 * 5 + 6 * 4 + 2 * 4 + 5
    st4 = _stats(weight_bytes=4)
    st4["bin_edges"][4] = 10
    assert bench.kernel_bytes(st4)["bin4"] == 10 * 12


def _write_profile(tmp_path, sources, variants, schedule, bins=None, bytes_per_launch=None):
    prof = tmp_path / "profiles"
    prof.mkdir(exist_ok=True)
    d = {"sources": sources, "variants": variants, "schedule": schedule,
         "bytes_per_launch": bytes_per_launch or {"bin5": 123456}}
    if bins is not None:
        d["bins"] = bins
    (prof / "rmat24_async_hbm_traffic.md").write_text("# summary\n\nmachine-readable: " + json.dumps(d) + "\n")


@pytest.fixture
def fake_root(tmp_path, monkeypatch):
    digest = bench.library_digest()
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    monkeypatch.setattr(bench, "library_digest", lambda: digest)
    return tmp_path, digest


def test_profiled_config_needs_matching_sources(fake_root):
    root, digest = fake_root
    _write_profile(root, digest, [0, 2, 2, 2, 2, 1], [1, 0, 1], [7, 31, 127, 511, 2047, 8191])
    assert bench.profiled_config("rmat24") == {"variants": [0, 2, 2, 2, 2, 1], "schedule": [1, 0, 1],
                                               "bins": [7, 31, 127, 511, 2047, 8191], "hubs_last": 0,
                                               "snapshot": 0}
    _write_profile(root, "0" * 16, [0, 2, 2, 2, 2, 1], [1, 0, 1])
    assert bench.profiled_config("rmat24") is None
    assert bench.profiled_config("rmat26") is None  # no summary at all


def test_profile_without_bins_means_default_bins(fake_root):
    root, digest = fake_root
    _write_profile(root, digest, [0] * 6, [16, 2, 4])
    assert bench.profiled_config("rmat24")["bins"] == bench.DEFAULT_BINS


def test_measured_traffic_only_for_the_profiled_configuration(fake_root):
    root, digest = fake_root
    cfg = dict(variants=[0, 2, 2, 2, 2, 1], schedule=[1, 0, 1], bins=[7, 31, 127, 511, 2047, 8191])
    _write_profile(root, digest, cfg["variants"], cfg["schedule"], cfg["bins"], {"bin5": 3896665165})
    assert bench.measured_traffic("bin5", dict(cfg), "rmat24") == 3896665165
    assert bench.measured_traffic("bin4", dict(cfg), "rmat24") is None       # kernel not in the summary
    assert bench.measured_traffic("bin5", None, "rmat24") is None            # untuned run
    for key, other in (("variants", [1] * 6), ("schedule", [16, 2, 4]), ("bins", bench.DEFAULT_BINS),
                       ("hubs_last", 1), ("snapshot", 1)):
        changed = dict(cfg)
        changed[key] = other
        assert bench.measured_traffic("bin5", changed, "rmat24") is None
    _write_profile(root, "f" * 16, cfg["variants"], cfg["schedule"], cfg["bins"], {"bin5": 1})
    assert bench.measured_traffic("bin5", dict(cfg), "rmat24") is None       # sources changed since


def test_committed_profiles_name_their_configuration():
    """Every committed counter summary carries the machine-readable line the
    bench reads, with sources, kernel shapes, schedule and bin limits."""
    for name in ("rmat24_async_hbm_traffic.md", "rmat26_async_hbm_traffic.md"):
        lines = [ln for ln in (ROOT / "profiles" / name).read_text().splitlines()
                 if ln.startswith("machine-readable: ")]
        assert len(lines) == 1, name
        d = json.loads(lines[0][len("machine-readable: "):])
        assert len(d["sources"]) == 16 and len(d["variants"]) == 6 and len(d["schedule"]) == 3
        assert len(d["bins"]) == 6 and d["bytes_per_launch"]


def test_storage_order_indices_match_the_library_layout():
    """The gather ceiling's index order: vertices in decreasing degree (ties
    by id), each row's neighbours renamed to positions and sorted - checked
    against a plain numpy construction (torch on the CPU)."""
    import types
    import numpy as np
    import torch
    from paper_2312_08140_amd import graphgen as gg
    g = gg.rmat(10, 8, seed=3, weighted=False)
    d = types.SimpleNamespace(n=g.n, m=g.m, offsets=torch.from_numpy(g.offsets.astype(np.int64)),
                              indices=torch.from_numpy(g.indices.astype(np.int32)))
    got = bench.storage_order_indices(d).numpy()
    deg = np.diff(g.offsets)
    order = np.argsort(-deg, kind="stable")
    pos = np.empty(g.n, np.int64)
    pos[order] = np.arange(g.n)
    want = np.concatenate([np.sort(pos[g.indices[g.offsets[v]:g.offsets[v + 1]]]) for v in order])
    assert np.array_equal(got, want.astype(np.int32))
