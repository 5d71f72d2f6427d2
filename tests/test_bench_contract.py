"""Host-side checks of bench.py (CPU): the one-GPU rule and the algorithmic
byte and flop counts that the roofline fields divide by."""

import os
import subprocess
import sys

import numpy as np

import bench
from paper_2306_12739_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_plane_kernel_bytes_are_the_stage_fields_of_the_interior_planes():
    # 5 spectral fields in, 3 out, complex FP32 (8 B) per kept mode, on the Ny - 2
    # interior planes of every member, plus the two plane means per plane in FP64
    w = inputs.WORKLOADS["channel-re4200-64x97x64-e16"]
    K = (w["Nx"] // 2) * (w["Nz"] - 1)
    planes = w["Ny"] - 2
    E = 16
    nbytes, _ = bench.kernel_model(w, E, "mixed")["plane"]
    assert nbytes == 8 * planes * E * K * 8 + 2 * planes * E * 8
    nbytes64, _ = bench.kernel_model(w, E, "fp64")["plane"]
    assert nbytes64 == 8 * planes * E * K * 16 + 2 * planes * E * 8


def test_mode_kernel_flops_count_every_half_size_product():
    # MACs per real column: the two [A B] solves on each parity half, F from
    # D1 (odd <- even, even <- odd), dv/dy from D1c, du/dy and dw/dy from D1
    w = inputs.WORKLOADS["channel-re4200-64x97x64-e16"]
    N = w["Ny"] - 2
    He, Ho = (N + 1) // 2, N // 2
    Fe, Fo = He + 1, Ho + 1
    K = (w["Nx"] // 2) * (w["Nz"] - 1)
    E = 16
    macs = (2 * (2 * He * He + 2 * Ho * Ho) + (Ho * Fe + He * Fo) + (Fo * He + Fe * Ho)
            + 2 * (Fo * Fe + Fe * Fo))
    _, flops = bench.kernel_model(w, E, "mixed")["mode"]
    assert flops == 2 * K * E * 2 * macs
    # the full-size (unsplit) products would cost about twice as much
    full = 2 * (N * 2 * N) + N * w["Ny"] + w["Ny"] * N + 2 * w["Ny"] * w["Ny"]
    assert 1.9 < full / macs < 2.1


def test_source_hash_is_stable_and_vector_peak_is_the_unpacked_rate():
    files = ["kernels_plane_wave.hip", "fft.h", "internal.h"]
    h1, h2 = bench.source_hash(files), bench.source_hash(files)
    assert h1 == h2 and len(h1) == 16
    assert int(h1, 16) >= 0
    assert bench.source_hash(files[:1]) != h1          # depends on every listed file
    assert bench.source_hash(["no_such_file.hip"]) is None
    assert np.isfinite(bench.VALU_PEAK_TFLOPS) and abs(bench.VALU_PEAK_TFLOPS - 78.6432) < 1e-9
