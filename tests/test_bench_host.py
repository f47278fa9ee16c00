"""Host-side contract of bench.py (no GPU): the one-GPU refusal, the traffic record's
source digest, and the per-model flop count the roofline objects use."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_sources_and_box_it_was_measured_on(tmp_path, monkeypatch):
    rec = {"kernel": "k_force", "bytes_per_launch": 123.0, "sources_sha256": bench.force_sources_digest(),
           "n_atoms": 4 * 200 ** 3}
    summary = tmp_path / "traffic.md"
    summary.write_text("# summary\n\ntraffic-json: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "traffic_summary_path", lambda cells: str(summary))
    assert bench.force_traffic(200) == 123.0
    assert bench.force_traffic(100) is None          # counters of another box
    rec["sources_sha256"] = "0" * 64  # counters taken on other sources
    summary.write_text("traffic-json: " + json.dumps(rec) + "\n")
    assert bench.force_traffic(200) is None
    monkeypatch.setattr(bench, "traffic_summary_path", lambda cells: str(tmp_path / "missing.md"))
    assert bench.force_traffic(200) is None


def test_summary_names_follow_the_box():
    assert bench.traffic_summary_path(200).endswith("k_force_fcc32m_fp32_hbm_traffic.md")
    assert bench.traffic_summary_path(100).endswith("k_force_fcc4m_fp32_hbm_traffic.md")


def test_flop_counts_scale_with_each_models_own_pairs():
    d_full, f_full = bench.flops_per_atom(74.6, 44.7, 122.0, "full")
    assert abs(f_full - (346 * 74.6 + 1222 * 44.7)) < 1e-6
    # the surrogate at its own (shorter) cutoffs does less work per atom than at the
    # full model's pair counts, which an MTS run's last evaluation would report
    _, f_own = bench.flops_per_atom(18.5, 12.0, 122.0, "surrogate")
    _, f_full_pairs = bench.flops_per_atom(74.6, 44.7, 122.0, "surrogate")
    assert f_own < 0.3 * f_full_pairs
    assert d_full > 0
