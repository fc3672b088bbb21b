"""Host-side logic of bench.py (no GPU): the one-GPU guard and the arithmetic
that turns rocprofv3 counter files into HBM bytes per launch."""
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
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def write_counters(d, counter, rows):
    os.makedirs(d)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, value) in enumerate(rows):
            w.writerow([i, name, counter, value])


def test_counter_calibration(tmp_path):
    """FETCH_SIZE of the copy kernel reads half of the bytes it moves and WRITE_SIZE
    all of them (the factors measured on MI355X): the step kernel's counts are
    scaled by the same factors, per launch, averaged over dispatches; other
    materials' launches and other kernels are ignored."""
    kib = bench.COPY_BYTES / 1024
    step = "void mclbm::march_kernel<1, 0, 6, 2>(mclbm::StepArgs, int, int, int)"
    other = "void mclbm::march_kernel<1, 1, 6, 2>(mclbm::StepArgs, int, int, int)"
    copy = "mclbm::copy_kernel(float const*, float*, unsigned long)"
    write_counters(tmp_path / "fetch", "FETCH_SIZE",
                   [(copy, kib / 2), (copy, kib / 2), (step, 1000.0), (step, 3000.0), (other, 9e9),
                    ("void at::native::foo", 7e9)])
    write_counters(tmp_path / "write", "WRITE_SIZE", [(copy, kib), (step, 1500.0), (other, 9e9)])
    out_file = tmp_path / "traffic.json"
    out = bench.ingest_counters(str(tmp_path / "fetch"), str(tmp_path / "write"), 64, str(out_file))
    assert out["fetch_factor"] == pytest.approx(2.0) and out["write_factor"] == pytest.approx(1.0)
    f32 = out["f32"]
    assert f32["read_bytes"] == pytest.approx(2 * 2000.0 * 1024)
    assert f32["written_bytes"] == pytest.approx(1500.0 * 1024)
    # the method's state per update (populations, u and j read and written),
    # and what the kernel must move without a stored j
    assert f32["algorithmic_bytes"] == 120 * 64 * 64 and f32["compulsory_bytes"] == 104 * 64 * 64
    assert f32["ratio"] == pytest.approx((4000.0 + 1500.0) * 1024 / (120 * 64 * 64))
    assert f32["ratio_compulsory"] == pytest.approx((4000.0 + 1500.0) * 1024 / (104 * 64 * 64))
    assert "f64" not in out and out["kernel_hash"] == bench.kernel_hash()
    assert json.loads(out_file.read_text())["f32"]["read_bytes"] == f32["read_bytes"]


def test_bytes_per_update():
    """Algorithmic bytes per lattice update by storage: 9 populations, u in FP64
    and j, each read and written once; the compulsory bytes leave out j."""
    assert bench.BYTES_PER_LUP == {"f32": 120, "f64": 208, "f16": 84, "bf16": 84}
    assert bench.COMPULSORY_BYTES_PER_LUP == {"f32": 104, "f64": 176, "f16": 68, "bf16": 68}


def test_counter_calibration_needs_the_copy(tmp_path):
    step = "void mclbm::march_kernel<1, 0, 6, 2>(mclbm::StepArgs, int, int, int)"
    write_counters(tmp_path / "fetch", "FETCH_SIZE", [(step, 1000.0)])
    write_counters(tmp_path / "write", "WRITE_SIZE", [(step, 1000.0)])
    with pytest.raises(SystemExit):
        bench.ingest_counters(str(tmp_path / "fetch"), str(tmp_path / "write"), 64, str(tmp_path / "t.json"))
