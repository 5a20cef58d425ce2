"""bench.py's contract on the CPU: one GPU only, and the roofline arithmetic."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_spmv_roofline_bytes_and_traffic():
    import bench
    # 9 FP64 values and one int32 column per block, int32 row pointers over
    # floor(n/3) slots, x read once and y written once (FP64)
    n = 1 << 10
    assert bench.spmv_bytes(100, n) == 76 * 100 + 4 * (n // 3 + 1) + 16 * n
    t = bench.spmv_traffic("hopper")
    c = bench.SPMV_COUNTERS["hopper"]
    fetch = c["fetch_kib"] * c["copy_kib"] / c["copy_fetch_kib"]
    write = c["write_kib"] * c["copy_kib"] / c["copy_write_kib"]
    assert abs(t - 1024.0 * (fetch + write)) < 1e-6 * t
    assert bench.spmv_traffic("no_such_scene") is None


def test_qtt_apply_work():
    import bench
    flops, nbytes = bench.qtt_apply_work([1, 2, 2, 1], 8, "f32")
    assert flops == 4.0 * 8 * (2 + 4 + 2)
    assert nbytes == 16.0 * 8 + 4 * (2 + 4 + 2) * 4
