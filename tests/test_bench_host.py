"""Host-side logic of bench.py (no GPU): the one-GPU refusal and the
algorithmic byte counts of the FFT stages used for the roofline."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_fft_stage_bytes_read_input_and_write_output_once():
    """each coil FFT pass reads its input array once and writes its output
    once; the first forward pass reads the image and C coil maps (complex64)
    and the last adjoint pass writes the coil-combined image"""
    n = (4, 6, 10)
    G = (8, 12, 20)
    C, es = 3, 8
    N = 4 * 6 * 10
    a = 4 * 6 * 20 * C * es      # after the axis-2 pass: n0 x n1 x G2 per coil
    b = 4 * 12 * 20 * C * es     # after the axis-1 pass: n0 x G1 x G2 per coil
    full = 8 * 12 * 20 * C * es  # the oversampled coil grids
    assert bench.stage_bytes("fft_coil_fwd_last", n, G, C, es) == N * 8 * (1 + C) + a
    assert bench.stage_bytes("fft_coil_fwd_ax1", n, G, C, es) == a + b
    assert bench.stage_bytes("fft_coil_fwd_ax0", n, G, C, es) == b + full
    assert bench.stage_bytes("fft_coil_adj_ax0", n, G, C, es) == full + b
    assert bench.stage_bytes("fft_coil_adj_ax1", n, G, C, es) == b + a
    assert bench.stage_bytes("fft_coil_adj_last", n, G, C, es) == a + N * 8 * (C + 1)
    # half-precision grids halve the grid terms only
    h = bench.stage_bytes("fft_coil_adj_ax0", n, G, C, 4)
    assert h * 2 == bench.stage_bytes("fft_coil_adj_ax0", n, G, C, 8)
    assert bench.stage_bytes("no_such_stage", n, G, C, es) is None
