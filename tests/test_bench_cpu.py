"""Host logic of bench.py on the CPU: the one-GPU contract, the algorithmic bytes per
element-step behind the roofline figure, and the PMC traffic parser (counter scaling by the copy
calibration, FP32 step-kernel launches only, the source-hash gate)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bytes_per_element_step_n4():
    # q read + write 8 Np, ring 12 Np, traces 16 Nfp, geometry / ids / flags 29 (words of 4 B)
    Np, Nfp = 35, 15
    assert bench.bytes_per_element_step(Np, Nfp, 0) == 3876
    assert bench.bytes_per_element_step(Np, Nfp, 1) == 3876 + 8 * Np
    assert bench.bytes_per_element_step(Np, Nfp, 2) == 3876 + 32 * Np


def _counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_from_pmc(tmp_path):
    d = str(tmp_path)
    gib = 2 ** 30
    # the calibration copy: FETCH_SIZE reads half of the bytes, WRITE_SIZE all of them (KiB)
    _counters(f"{d}/cf", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", gib / 2048), ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 8)])
    _counters(f"{d}/cw", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", gib / 1024)])
    fp32 = "void dgrtm::step_kernel_dma<4, 0, 0>(dgrtm::StepArgs)"
    bf16 = "void dgrtm::step_kernel_dma<4, 0, 1>(dgrtm::StepArgs)"
    img = "void dgrtm::step_kernel_dma<4, 2, 0>(dgrtm::StepArgs)"
    # the N >= 5 kernel: <N, MODE, OPS_LDS, PREC>
    lr32 = "void dgrtm::step_kernel_lowreg<5, 1, true, 0>(dgrtm::StepArgs)"
    lr16 = "void dgrtm::step_kernel_lowreg<5, 1, true, 1>(dgrtm::StepArgs)"
    _counters(f"{d}/sf", [(fp32, "FETCH_SIZE", 100.0), (fp32, "FETCH_SIZE", 300.0), (bf16, "FETCH_SIZE", 9999.0),
                          (img, "FETCH_SIZE", 50.0), ("dgrtm::record_kernel", "FETCH_SIZE", 7.0),
                          (lr32, "FETCH_SIZE", 70.0), (lr16, "FETCH_SIZE", 9999.0)])
    _counters(f"{d}/sw", [(fp32, "WRITE_SIZE", 10.0), (fp32, "WRITE_SIZE", 30.0), (bf16, "WRITE_SIZE", 9999.0),
                          (img, "WRITE_SIZE", 5.0), (lr32, "WRITE_SIZE", 7.0), (lr16, "WRITE_SIZE", 9999.0)])
    out = bench.traffic_from_pmc("toy", f"{d}/sf", f"{d}/sw", f"{d}/cf", f"{d}/cw", "cmd", profiles_dir=d)
    t = json.load(open(out))
    assert t["copy_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert t["copy_calibration"]["write_scale"] == pytest.approx(1.0)
    fwd = t["modes"]["forward_step"]
    assert fwd["launches"] == 2                                    # the split-BF16 launch is left out
    assert fwd["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2)
    assert fwd["write_bytes_per_launch"] == pytest.approx(20.0 * 1024)
    assert t["modes"]["image_step"]["bytes_per_launch"] == pytest.approx((50.0 * 2 + 5.0) * 1024)
    assert t["modes"]["recompute_step"]["launches"] == 1
    assert t["modes"]["recompute_step"]["bytes_per_launch"] == pytest.approx((70.0 * 2 + 7.0) * 1024)
    assert bench.load_traffic("toy", "forward_step", profiles_dir=d) == pytest.approx((400 + 20) * 1024, abs=0.1)
    # taken on another kernel source: no traffic figure
    t["kernel_source_sha256_16"] = "0" * 16
    json.dump(t, open(out, "w"))
    assert bench.load_traffic("toy", "forward_step", profiles_dir=d) is None


def test_column_sample_spans_the_depth():
    import numpy as np
    from paper_1506_00907_amd import inputs as I
    m = I.two_layer_mesh(10, 8, 5, seed=1)
    el = bench.column_elements(m, 3)
    assert el.size == 3 * 3 * 5 * 6 and np.all(np.diff(el) > 0)
    cells = el // 6
    assert set((cells // (10 * 8)).tolist()) == set(range(5))            # every layer
    assert set((cells % 10).tolist()) == {3, 4, 5} and set(((cells // 10) % 8).tolist()) == {2, 3, 4}


def test_kernel_trace_summary_classifies_launches_by_local_step(tmp_path):
    # two global steps of a 3-level schedule: local steps 0..3 activate 3, 1, 2, 1 levels
    d = tmp_path / "trace" / "host" / "1"
    d.mkdir(parents=True)
    rows = ["Kind,Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp"]
    dur = {3: 30000, 1: 10000, 2: 20000}
    t = 0
    for i in range(8):
        a = (3, 1, 2, 1)[i % 4]
        rows.append(f'KERNEL_DISPATCH,{2 * i + 1},"void dgrtm::step_kernel_dma<4, 0, 0>(dgrtm::StepArgs)",{t},{t + dur[a]}')
        rows.append(f'KERNEL_DISPATCH,{2 * i + 2},"dgrtm::record_kernel(float const*)",{t},{t + 1000}')
        t += 100000
    (d / "run_kernel_trace.csv").write_text("\n".join(rows) + "\n")
    out = bench.kernel_trace_summary(str(tmp_path / "trace"), 3)
    assert "mean 17.5  1:10.0 2:20.0 3:30.0" in out
    assert "dgrtm::record_kernel(float const*)" in out
