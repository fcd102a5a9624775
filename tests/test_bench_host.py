"""The benchmark's host-side parts on the CPU: the refusal of more than one
GPU, the byte models its roofline fractions divide by (checked against
closed forms and a direct count on a small stencil), and the rule that the
counter-measured traffic is reported only for the kernel sources that were
measured."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import spd_problems as P  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_matrix_bytes_both_storages():
    pr = P.make_config("poisson3d_256", size=6)
    A = pr.A
    n = A.shape[0]
    assert bench.matrix_bytes(A, "csr") == 12 * A.nnz + 4 * (n + 1)
    assert bench.matrix_bytes(A, "dia") == 8 * 7 * n
    D = P.make_config("diffusion27_160", size=5).A
    assert bench.matrix_bytes(D, "dia") == 8 * 27 * D.shape[0]


def test_mpk_bytes_closed_forms():
    """Per outer loop at s = 10 with the Chebyshev basis: level 1 reads A and
    one pair level and writes one (|A| + 32 n), levels 2..9 also read the
    level before last (|A| + 48 n), the last sweep reads A and the ten pair
    levels and writes P_s (|A| + 168 n)."""
    n, A = 16777216, 8 * 7 * 16777216
    total, ge2, l1, last = bench.mpk_bytes(n, A, 10, True)
    assert (l1, ge2, last) == (A + 32 * n, A + 48 * n, A + 168 * n)
    assert total == 10 * A + 584 * n == 1144 * n        # the 256^3 figure: 19,193,135,104
    total_n, ge2_n, _, _ = bench.mpk_bytes(n, A, 10, False)
    assert ge2_n == A + 32 * n and total_n == total - 8 * 16 * n
    # s = 1: the last sweep alone
    assert bench.mpk_bytes(n, A, 1, True)[0] == A + 24 * n


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    t = bench.measured_traffic("k_sweep_dia")
    assert t is None or t > 0
    fake = tmp_path / "counters.txt"
    fake.write_text("kernel sources measured (sha256 of kernels.hip, device.hpp, launch.hpp, "
                    "ctl.hpp): 0000000000000000\ntraffic k_sweep_dia per launch (bytes): 123\n")
    monkeypatch.setattr(bench, "COUNTER_FILE", str(fake))
    assert bench.measured_traffic("k_sweep_dia") is None
