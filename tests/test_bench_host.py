"""Host logic of bench.py (no GPU): the one-GPU guard, the HBM counter
summary and its calibration by a plain copy, the source digest that keeps a
stored summary tied to the kernels it was taken on, and the roofline
classification of the force kernel."""
import csv
import os
import shutil
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counter_csv(folder, rows):
    """rows: (kernel name as rocprofv3 prints it, counter, value per dispatch)."""
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (k, c, v) in enumerate(rows):
            w.writerow([i, k, c, v])


def test_traffic_summary_scales_counters_by_the_copy(tmp_path):
    gib_kib = float(1 << 20)
    # the copy of 1 GiB: FETCH_SIZE reads half its bytes, WRITE_SIZE all of them
    _counter_csv(tmp_path / "cf", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", gib_kib / 2)] * 5)
    _counter_csv(tmp_path / "cw", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", gib_kib)] * 5)
    force = "void mdlg::k_force<2, 256>(mdlg::ForceArgs)"
    nl = "void mdlg::k_nlist_narrow<2, 256>(mdlg::NlistArgs)"
    _counter_csv(tmp_path / "f", [(force, "FETCH_SIZE", 100.0), (force, "FETCH_SIZE", 200.0),
                                  (nl, "FETCH_SIZE", 10.0), (force, "WRITE_SIZE", 1e9)])
    _counter_csv(tmp_path / "w", [(force, "WRITE_SIZE", 40.0), (nl, "WRITE_SIZE", 30.0)])
    out = bench.summarize_traffic("unit", str(tmp_path / "f"), str(tmp_path / "w"),
                                  str(tmp_path / "cf"), str(tmp_path / "cw"), out_dir=str(tmp_path))
    assert out["copy_calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert out["copy_calibration"]["write_factor"] == pytest.approx(1.0)
    k = out["kernels"]
    # mean over dispatches of the named counter only, by kernel class
    assert k["force"]["fetch_kib"] == pytest.approx(150.0)
    assert k["force"]["write_kib"] == pytest.approx(40.0)
    assert k["force"]["bytes_per_launch"] == pytest.approx((150.0 * 2 + 40.0) * 1024)
    assert k["nlist"]["bytes_per_launch"] == pytest.approx((10.0 * 2 + 30.0) * 1024)
    assert os.path.exists(tmp_path / "traffic_unit.json")


def _tree_with_sources(tmp_path):
    src = os.path.join(ROOT, "paper_1705_04368_amd", "csrc")
    dst = tmp_path / "paper_1705_04368_amd" / "csrc"
    os.makedirs(dst)
    for f in ("mdlg_kernels.hip", "mdlg_force_block.inc", "mdlg_args.h", "mdlg_device.h"):
        shutil.copy(os.path.join(src, f), dst / f)
    return dst


def test_source_digest_ignores_comments_and_follows_code(tmp_path, monkeypatch):
    dst = _tree_with_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.source_digest()
    k = dst / "mdlg_kernels.hip"
    text = k.read_text()
    k.write_text("// a new comment\n/* and a\n   block comment */\n" + text.replace("\n", "\n\n", 3))
    assert bench.source_digest() == d0
    k.write_text(text.replace("constexpr int kSentinel = 1 << 30;", "constexpr int kSentinel = 1 << 29;"))
    assert bench.source_digest() != d0
    # the force block's body, pasted into the kernels, counts as kernel source
    k.write_text(text)
    assert bench.source_digest() == d0
    f = dst / "mdlg_force_block.inc"
    body = f.read_text()
    assert "const bool interact = !P.forces_off;" in body
    f.write_text(body.replace("const bool interact = !P.forces_off;", "const bool interact = true;"))
    assert bench.source_digest() != d0


def test_stored_traffic_is_used_only_on_matching_sources(tmp_path, monkeypatch):
    _tree_with_sources(tmp_path)
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    import json
    rec = {"source_digest": bench.source_digest(), "kernels": {"force": {"bytes_per_launch": 123.0}}}
    (tmp_path / "profiles" / "traffic_w.json").write_text(json.dumps(rec))
    assert bench.load_traffic("w", "force") == 123.0
    assert bench.load_traffic("w", "nlist") is None
    rec["source_digest"] = "0" * 16
    (tmp_path / "profiles" / "traffic_w.json").write_text(json.dumps(rec))
    assert bench.load_traffic("w", "force") is None


def test_kernel_table_grades_forces_on_fp32_and_sort_on_hbm():
    # the force kernel on the FP32 vector units with the FLOPs of the
    # interacting pairs (9.82 per particle in 2D at rho = 0.5, 18 FLOP each);
    # the rebuild as one unit on HBM with 104 B per particle (2D) + 12 B per cell
    n, rho = 262144, 0.5
    lay = {"n_velocities": 49, "n_moments": 7, "margin": 0.4, "skin": 0.25, "pair_slots": 48,
           "n_cells": 32761}
    tim = {"force": (0.1, 10), "count": (0.02, 2), "scan": (0.01, 2), "scatter": (0.02, 2),
           "bin": (0.015, 1), "nlist": (0.0, 0)}
    k, sort = bench.kernel_table(tim, 2, n, rho, lay, 32761)
    f = k["force"]
    flops = n * 3.14159265 * 2.5 ** 2 * 0.5 * 18
    assert f["bound"] == "alu" and f["unit"] == "TFLOP/s" and f["peak"] == 157.3
    assert f["work_per_launch"] == pytest.approx(flops, rel=1e-6)
    assert f["achieved"] == pytest.approx(flops / 1e-5 / 1e12, rel=1e-6)
    assert f["frac"] == pytest.approx(f["achieved"] / 157.3)
    assert "nlist" not in k
    assert k["bin"]["bound"] == "hbm"
    # 52 B per particle (offset, image, cell, snapshot read and written) and
    # the per-site counters (2 x 4 x 49 + 2 x 8 x 7 B) shared by 8 particles
    assert bench.bin_bytes_per_particle(2, 49, 7, 8.0) == pytest.approx(52 + 504 / 8)
    assert sort["avg_ms"] == pytest.approx(0.025)
    assert sort["work_per_launch"] == n * 104 + 12 * 32761
    assert bench.sort_bytes(3, 1, 0) == 144
    # the force kernel's arithmetic intensity is below the ridge point on
    # HBM bytes too, but the FP32 bound is the one graded
    ridge = bench.PEAK_FP32_TFLOPS * 1e12 / (bench.PEAK_HBM_GBS * 1e9)
    assert bench.force_bytes_per_particle(2) == 32
    ai = bench.pairs_per_particle(2, rho) * 18 / bench.force_bytes_per_particle(2, rho, 3.3)
    assert 1.0 < ai < ridge


def test_event_pair_offset_is_removed_from_the_averages():
    # mdlg_timing_offset reads the clock wait's excess over its span; the
    # 0.6 us of the wait's own dispatch stays in every kernel's duration
    class FakeSystem:
        def __init__(self, ms):
            self.ms = ms

        def timing_offset(self):
            return self.ms

    assert bench.event_pair_offset(FakeSystem(0.0046)) == pytest.approx(0.004)
    assert bench.event_pair_offset(FakeSystem(0.0003)) == 0.0
    lay = {"n_velocities": 49, "n_moments": 7, "margin": 0.4, "skin": 0.25, "pair_slots": 48,
           "n_cells": 100}
    # 10 launches of 0.2 ms by their events, 2 of 0.003 ms
    tim = {"force": (2.0, 10), "scan": (0.006, 2)}
    k, _ = bench.kernel_table(tim, 2, 800, 0.5, lay, 100, offset_ms=0.004)
    assert k["force"]["event_ms"] == pytest.approx(0.2)
    assert k["force"]["avg_ms"] == pytest.approx(0.196)
    # graded on the corrected time
    assert k["force"]["achieved"] == pytest.approx(k["force"]["work_per_launch"] / 0.196e-3 / 1e12)
    # an average at or below the offset is left as measured
    assert k["scan"]["avg_ms"] == pytest.approx(0.003)
    assert k["scan"]["achieved"] > 0.0


def test_ensemble_statistics():
    import numpy as np
    rng = np.random.default_rng(3)
    fr = rng.normal(1.0, 0.1, size=(512, 4))
    w = rng.integers(10, 100, size=512)
    mean, se = bench.ensemble_mean_se(fr, w)
    assert mean == pytest.approx((w[:, None] * fr).sum(0) / w.sum())
    # equal weights: the plain standard error of the mean
    m2, se2 = bench.ensemble_mean_se(fr, np.ones(512))
    assert se2 == pytest.approx(fr.std(axis=0, ddof=1) / np.sqrt(512))
    c = bench.compare_fi(mean, se, mean + 0.5 * se, se, np.full(4, 1e6))
    assert c["agree"] and c["bins_tested"] == 4 and c["max_abs_z"] == pytest.approx(0.5 / np.sqrt(2))
    c = bench.compare_fi(mean, se, mean + 10 * se, se, np.full(4, 1e6))
    assert not c["agree"]
    # per-replica f_i from per-site averages
    m_r = np.array([2, 3])
    f_site = np.arange(13 * 2, dtype=float).reshape(13, 2)
    fr, sites = bench.replica_fi(f_site, m_r)
    assert list(sites) == [4, 9]
    assert fr[0] == pytest.approx(f_site[:4].mean(0)) and fr[1] == pytest.approx(f_site[4:].mean(0))
