"""Host-side parts of the benchmark contract (no GPU): the one-GPU refusal and the
arithmetic of the committed HBM-traffic summaries that bench.py reports as
roofline.traffic."""
import glob
import json
import os
import subprocess
import sys

import pytest

from paper_1803_02156_amd import traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))))
def test_traffic_summary_arithmetic(path):
    """HBM bytes = FETCH_SIZE x read factor + WRITE_SIZE x write factor (KiB), the
    factors from the copy kernel of the same run (it reads and writes known byte
    counts), and the algorithmic bytes are the Eq. 2 model of one fused step."""
    with open(path) as f:
        t = json.load(f)
    cal = t["copy_kernel_calibration"]
    nbytes = cal["bytes_read_and_written_each"]
    assert abs(cal["fetch_kib"] * 1024 * cal["read_factor"] / nbytes - 1) < 0.01
    assert abs(cal["write_kib"] * 1024 * cal["write_factor"] / nbytes - 1) < 0.01
    rd = t["fetch_size_kib_per_dispatch"] * 1024 * cal["read_factor"]
    wr = t["write_size_kib_per_dispatch"] * 1024 * cal["write_factor"]
    assert abs(rd - t["hbm_read_bytes_per_launch"]) <= 1e-6 * rd + 1024
    assert abs(wr - t["hbm_write_bytes_per_launch"]) <= 1e-6 * wr + 1024
    assert t["hbm_bytes_per_launch"] == t["hbm_read_bytes_per_launch"] + t["hbm_write_bytes_per_launch"]
    w = t["workload"]
    n = int(w.split("n=")[1].split(",")[0])
    nnz = int(w.split("nnz=")[1].split(",")[0])
    prec = 0 if "FP64" in w else 1
    n_b = int(w.split("n_b=")[1].split(",")[0])
    r_alg, w_alg = traffic.step_bytes(n, nnz, n_b, prec)
    assert t["algorithmic_bytes_per_launch"] == r_alg + w_alg
    assert t["algorithmic_read_bytes_per_launch"] == r_alg
    assert abs(t["traffic_over_algorithmic"] - t["hbm_bytes_per_launch"] / (r_alg + w_alg)) < 6e-4
    assert abs(t["reads_over_algorithmic"] - t["hbm_read_bytes_per_launch"] / r_alg) < 6e-4
