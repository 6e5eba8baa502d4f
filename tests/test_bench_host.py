"""Host logic of bench.py (no GPU): the one-GPU guard, the two-axis roofline choice, and
that a profile summary is used only on the source it was taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_roofline_names_the_binding_axis():
    ctr = {"salu_insts_per_launch": "7e7", "l2_hit_rate": "0.5"}
    launch_s = 1e-3
    # HBM: 400 GB/s of 8 TB/s = 5 %; VALU: 30 % of the issue peak -> bound by issue
    valu = 0.3 * bench.VALU_ISSUE_PEAK * launch_s
    r = bench.roofline_block(400.0, 2.0e9, valu, 0.3, launch_s, ctr)
    assert r["bound"] == "alu" and r["frac"] == pytest.approx(0.3)
    assert r["hbm"]["frac"] == pytest.approx(400.0 / bench.HBM_PEAK_GBS)
    assert r["alu"]["achieved"] == pytest.approx(valu / launch_s / 1e9)
    # traffic over the algorithmic bytes of the launch (400 GB/s for 1 ms = 0.4 GB)
    assert r["traffic_over_algorithmic"] == pytest.approx(2.0e9 / 0.4e9)
    # without counters only the HBM axis is known
    r = bench.roofline_block(400.0, None, None, None, launch_s, {})
    assert r["bound"] == "hbm" and r["alu"] is None and r["traffic_over_algorithmic"] is None
    # an HBM fraction above the issue fraction binds
    r = bench.roofline_block(4000.0, None, valu, 0.3, launch_s, ctr)
    assert r["bound"] == "hbm" and r["frac"] == pytest.approx(0.5)


def test_profile_is_used_only_on_its_source(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel v1\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.txt").write_text("# header\nk_average_us = 12.5\n"
                                f"kernel_source_sha256_16 = {bench.source_hash(str(src))}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    kv = bench.read_profile("k.txt", str(src))
    assert kv is not None and bench.read_float(kv, "k_average_us") == pytest.approx(12.5)
    src.write_text("// kernel v2\n")
    assert bench.read_profile("k.txt", str(src)) is None
