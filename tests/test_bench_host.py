"""Host logic of bench.py (CPU): the algorithmic-byte model of the V-cycle, the
flop counts, the traffic guard and the one-GPU contract."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_vcycle_bytes_by_hand():
    # 8^3 elements: levels of 8 and 4 elements per side (9^3 and 5^3 nodes);
    # top level 32 + 35.5 s bytes per node, coarsest 5 s
    assert bench.vcycle_bytes(3, 8, 4) == (32 + 35.5 * 4) * 729 + 5 * 4 * 125
    # 16^3: one intermediate level at 37.5 s per node
    assert bench.vcycle_bytes(3, 16, 8) == (32 + 35.5 * 8) * 17 ** 3 + 37.5 * 8 * 9 ** 3 + 5 * 8 * 125
    # an odd side stops the coarsening at once: split, coarse solve, merge
    assert bench.vcycle_bytes(2, 7, 4) == (32 + 9 * 4) * 64
    # the 256^3 figure quoted with the measurements
    assert abs(bench.vcycle_bytes(3, 256, 4) - 3.323e9) < 1e6


def test_flop_counts():
    # source-level count of the plain 3-D residual (no preconditioner
    # coefficient); the counter value of the compiled kernel is 63 below it
    assert bench.flops_per_element(3) == 2976
    assert bench.FLOPS_PER_ELEM[3] == bench.KERNEL_FLOPS_PER_ELEM_3D["residual"] == 2913
    assert bench.flops_per_element(3) - bench.FLOPS_PER_ELEM[3] == 63
    assert bench.FLOPS_PER_ELEM[2] == bench.flops_per_element(2) == 751


def test_traffic_figure_is_tied_to_the_sources():
    assert bench.residual_traffic("seeds3d_256") in (None, bench.RESIDUAL_TRAFFIC["bytes"])
    assert bench.residual_traffic("another_workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
