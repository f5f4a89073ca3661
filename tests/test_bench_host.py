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
    for f in ("mdlg_kernels.hip", "mdlg_args.h", "mdlg_device.h"):
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


def test_force_kernel_is_hbm_bound_on_the_benchmarked_workloads():
    # algorithmic bytes: state read and written (16 d), reference offset (4 d)
    # and 2 bytes per neighbour within the list radius; FLOPs of the
    # interacting pairs within r_c.  Both workloads sit far below the ridge
    # point of the FP32 peak over the HBM bandwidth.
    ridge = bench.PEAK_FP32_TFLOPS * 1e12 / (bench.PEAK_HBM_GBS * 1e9)
    assert bench.force_bytes_per_particle(2, 0.5) == 32
    assert bench.force_bytes_per_particle(2, 0.5, 3.3) == pytest.approx(40 + 3.14159265 * 3.3 ** 2,
                                                                        rel=1e-6)
    for dim, rho, margin in ((2, 0.5, 0.4), (3, 4194304 / 192.0 ** 3, 0.392)):
        rl = 2.5 + 2 * margin
        ai = (bench.pairs_per_particle(dim, rho) * bench.FLOP_PER_PAIR[dim]
              / bench.force_bytes_per_particle(dim, rho, rl))
        assert 1.0 < ai < ridge / 4
    # the adjoint's reverse step likewise
    ai = (bench.pairs_per_particle(2, 0.5) * bench.ADJ_FLOP_PER_PAIR[2]
          / bench.adjoint_bytes_per_particle(2))
    assert ai < ridge
