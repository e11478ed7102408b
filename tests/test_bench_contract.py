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
