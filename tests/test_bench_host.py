"""Host logic of bench.py on the CPU: the committed counter summaries are
parsed and used only while the kernel source they were taken on is the
current one, the multi-GPU request is refused with a message, and the
algorithmic operation count is a plain weighted sum of the oracle's work
counters."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_profiles_parse_and_gate_on_source_hash():
    h = bench.source_hash()
    assert len(h) == 16
    t = bench.traffic_from_profile(h)
    v = bench.valu_from_profile(h)
    # the committed summaries were taken on the committed kernel sources
    assert t is not None and v is not None
    assert 5e7 < t["bytes"] < 2e8
    assert t["fetch_kib"] > 0 and t["write_kib"] > 0
    assert 0 < v["valu_busy_pct"] <= 100 and 0 < v["valu_utilization_pct"] <= 100
    assert v["valu_insts_per_launch"] > 1e6
    g = bench.grid_kernels_from_profile(1 << 20, 1 << 21, 0.05)
    assert g["kernels"] and set(g["kernels"]) >= {"k_cell_count", "k_scatter"}
    # any other source hash turns both off
    assert bench.traffic_from_profile("0" * 16) is None
    assert bench.valu_from_profile("0" * 16) is None


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_ops_is_weighted_work():
    w = np.zeros((3, len(bench.OP_COST)), np.int64)
    w[0, 0] = 10   # candidates examined
    w[1, 2] = 4    # neighbours used
    w[2, 3] = 7    # LP2 lines checked
    expect = 10 * bench.OP_COST[0] + 4 * bench.OP_COST[2] + 7 * bench.OP_COST[3]
    assert bench.algorithmic_ops(w) == expect


def test_roofline_object():
    r = bench.alu_roofline(3.9e9, 0.5, 1 << 20, bench.STEP_BYTES_PER_AGENT, "k")
    assert r["bound"] == "alu" and r["unit"] == "Top/s"
    np.testing.assert_allclose(r["achieved"], 3.9e9 / 0.5e-3 / 1e12)
    np.testing.assert_allclose(r["frac"], r["achieved"] / r["peak"])
    np.testing.assert_allclose(r["hbm_frac"], 49 * (1 << 20) / 0.5e-3 / 1e9 / 8000.0)


def test_grid_kernel_bytes():
    g = bench.grid_kernels_from_profile(1000, 500, 0.01)
    assert g["algorithmic_bytes"] == (8 * 1000 + 4 * 500) + (16 * 1000 + 8 * 500) + 4 * 500 \
        + 8 * 500 + 65 * 1000
    assert 0 < g["hbm_frac_whole_build"] < 1
