"""Host logic of the benchmark report (CPU only): the interaction rate and
FLOP/s at the stated flop counts, the tree build's algorithmic HBM rate, the
walk rates, the HBM traffic record that is used only while the kernel sources
still hash to the digest it was taken for, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _rec(n_pp, n_pc, ms_force, **extra):
    r = dict(n_pp=n_pp, n_pc=n_pc, n_pp_near=n_pp // 10, ms_force=ms_force, ms_build=1.0,
             ms_walk=0.4, n_nodes=1000, ms_neighbors=0.1, n_cell_entries=10, n_part_entries=20,
             n_near_entries=5, walk_fixed_stride=1, n_groups=7, nnz=4)
    r.update(extra)
    return r


def test_summarize_rates_and_flops():
    rec = [_rec(1000, 2000, 2.0), _rec(3000, 4000, 4.0)]
    s = bench.summarize(rec, seconds=0.5, steps=2, quad=True)
    assert s["interactions_per_step"] == (1000 + 2000 + 3000 + 4000) / 2
    assert s["interactions_per_s"] == 10000 / 0.5
    assert s["ms_per_step"] == 250.0
    flops = ((1000 * bench.F_PP + 2000 * bench.F_PC_QUAD) + (3000 * bench.F_PP + 4000 * bench.F_PC_QUAD)) / 2
    assert s["flops_per_launch"] == flops
    assert s["force_tflops"] == pytest.approx(flops / 3e-3 / 1e12)
    survey = ((1000 * 37 + 2000 * 75) + (3000 * 37 + 4000 * 75)) / 2
    assert s["force_tflops_survey"] == pytest.approx(survey / 3e-3 / 1e12)
    mono = bench.summarize(rec, seconds=0.5, steps=2, quad=False)
    assert mono["flops_per_launch"] < flops      # the monopole cell term counts fewer flops


def test_build_roofline_and_walk_rates():
    head = dict(build_ms=1.0, walk_ms=0.4, n_nodes=1000, n_groups=50.0,
                list_entries={"cell": 100.0, "part": 200.0, "near": 50.0})
    b = bench.build_roofline(head, n=1 << 20)
    byts = (1 << 20) * sum(bench.BUILD_BYTES_PER_PARTICLE.values()) + \
        1000 * sum(bench.BUILD_BYTES_PER_NODE.values())
    assert b["algorithmic_bytes"] == byts
    assert b["tree_ms"] == pytest.approx(0.6)
    assert b["achieved_GBps"] == pytest.approx(byts / 0.6e-3 / 1e9)
    assert b["frac"] == pytest.approx(b["achieved_GBps"] / bench.HBM_PEAK_GBPS)
    w = bench.walk_rates(head)
    assert w["groups_per_s"] == pytest.approx(50 / 0.4e-3)
    assert w["list_entries"] == 350.0
    assert w["list_bytes"] == 4 * 350 + 3 * 16 * 50


def test_traffic_record_follows_the_kernel_sources(tmp_path, monkeypatch):
    digest = bench.kernel_sources_digest()
    rec = {"kernel": "k", "workload": "w", "precision": "mixed", "sources_sha256": digest,
           "fetch_bytes": 10, "write_bytes": 2}
    f = tmp_path / "traffic.md"
    f.write_text("# summary\n\ntraffic: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic("w", "mixed") == rec
    assert bench.recorded_traffic("w", "fp64") is None
    assert bench.recorded_traffic("other", "mixed") is None
    f.write_text("traffic: " + json.dumps(dict(rec, sources_sha256="0" * 64)) + "\n")
    assert bench.recorded_traffic("w", "mixed") is None     # taken for other sources
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.recorded_traffic("w", "mixed") is None


def test_committed_traffic_record_is_well_formed():
    """The committed record names the interaction kernel, its workload, and
    read and write bytes per launch (it is used only while its digest holds)."""
    lines = [ln for ln in open(bench.TRAFFIC_FILE) if ln.startswith("traffic: ")]
    assert len(lines) == 1
    rec = json.loads(lines[0][len("traffic: "):])
    assert rec["kernel"].startswith("k_force") and rec["workload"] == "king9_1m"
    assert rec["fetch_bytes"] > 0 and rec["write_bytes"] > 0
    assert len(rec["sources_sha256"]) == 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr
