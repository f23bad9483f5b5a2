"""Host-side checks of the benchmark script (no GPU): the committed counter
figures belong to the committed kernel sources, and a multi-GPU request is
refused before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_counter_figures_belong_to_the_committed_kernels():
    """The traffic figure the roofline reports belongs to the kernel sources and
    launch plan it was measured on (profiles/hydro_fp64_256_counters.md), and
    is null for any other sources."""
    for f in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, f)), f
    # figures taken on other sources are reported as null, never as measured
    want = bench.STAGE_TRAFFIC["bytes_per_launch"] if bench.counters_valid() else None
    assert bench.measured_traffic() == want
    assert 0.0 < bench.STAGE_VALU_ISSUE_FRAC < 1.0


def test_flop_and_byte_counts_per_cell():
    assert bench.HYDRO_FLOPS_PER_CELL_STAGE == 45 * 15 + 106 * 3 + 13 + 57.5 + 11
    assert bench.HYDRO_BYTES_PER_CELL_STEP == 200.0
    # a radiation substep: stage 1 reads and writes (E_r, F); stage 2 with the
    # coupling also reads the stage buffer and the gas and writes m, E
    assert (bench.RAD_BYTES_STAGE1, bench.RAD_BYTES_STAGE2) == (64.0, 168.0)


def test_more_than_one_gpu_is_refused_without_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
