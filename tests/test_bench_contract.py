"""Host-side contract of bench.py (no GPU needed): the benchmark is a one-GPU program, so
--gpus N with N > 1 exits with status 2 and a message saying so, before any device work;
the algorithmic byte counts per node update match the state each form keeps."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bytes_per_node_update():
    # population form: 2 (NS Q + (Q - 1) + NS + 2 d) b
    assert bench.algorithmic_bytes_per_node(3, 19, 3, 8) == 1344      # 256^3 N = 4 FP64
    assert bench.algorithmic_bytes_per_node(3, 19, 3, 4) == 672
    assert bench.algorithmic_bytes_per_node(2, 9, 4, 4) == 416        # 2048^2 N = 5 FP32
    assert bench.algorithmic_bytes_per_node(2, 9, 3, 8) == 672        # 512^2 N = 4 FP64
    # moment form: 2 (NS (1 + 2d [+1 FP32]) + (Q - 1) + 2 d) b, moments buffer 2 NS (4 [+1]) b
    assert bench.algorithmic_bytes_per_node_moment_form(3, 19, 3, 8) == 720
    assert bench.algorithmic_bytes_per_node_moment_form(3, 19, 3, 4) == 384
    assert bench.moments_buffer_bytes_per_node(3, 8) == 192
    assert bench.moments_buffer_bytes_per_node(3, 4) == 120


def test_kernel_hash_covers_every_step_unit():
    """The traffic counters are used only while the sources they were taken with are
    unchanged: every step translation unit the build compiles, the headers they include and
    the host code that launches them enter the hash."""
    from paper_2306_06983_amd import build
    step_units = {s for s in build.SOURCES if s.startswith("kernels_")} | {"nphase_lbm.hip"}
    assert step_units <= set(bench.STEP_SOURCES)
    csrc = os.path.join(ROOT, "paper_2306_06983_amd", "csrc")
    for inc in ("kernels_tu.inc", "dispatch.hpp", "step_kernel.hpp", "step3d_kernel.hpp",
                "lattice.hpp", "aux_kernels.hpp"):
        assert os.path.exists(os.path.join(csrc, inc))
        assert inc in bench.STEP_SOURCES
