"""Host logic of bench.py (CPU): the algorithmic flop counts behind the
roofline figures, checked by brute force against the sums they count, and
the one-GPU contract of the command line."""
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def brute_force_theta_macs(nk, band):
    """Multiply-adds of one direct Theta application on an nk x nk plane:
    single-body shifts m = 1..band of either particle and pair shifts
    m = 1..nk-1 along the anti-diagonal, each counted where its source point
    lies on the plane (zero off the box)."""
    inside = lambda a, b: 0 <= a < nk and 0 <= b < nk  # noqa: E731
    macs = 0
    for n1 in range(nk):
        for n2 in range(nk):
            for m in range(1, band + 1):
                macs += inside(n1 - m, n2) + inside(n1 + m, n2) + inside(n1, n2 - m) + inside(n1, n2 + m)
            for m in range(1, nk):
                macs += inside(n1 - m, n2 + m) + inside(n1 + m, n2 - m)
    return macs


@pytest.mark.parametrize("nk,band", [(5, 1), (8, 1), (8, 3), (12, 11), (16, 4)])
def test_theta_flop_model_counts_the_direct_sums(nk, band):
    assert bench.theta_flops_per_point(nk, band) == pytest.approx(2.0 * brute_force_theta_macs(nk, band) / nk**2,
                                                                 rel=1e-12)


def test_fft_flop_model():
    """5 N log2 N per complex transform of length N = 2 nk: nk row transforms
    (nk/2 forward, nk/2 inverse, two real rows each) and a forward and an
    inverse column transform for each of the N/2 + 1 column frequencies, plus
    2 flops per complex value for the symbol multiply, per plane point."""
    for nk in (32, 64, 128):
        n = 2 * nk
        transforms = nk + 2 * (n // 2 + 1)
        per_plane = transforms * 5 * n * math.log2(n) + (n // 2 + 1) * n * 2
        assert bench.fft_flops_per_point(nk) == pytest.approx(per_plane / nk**2, rel=1e-12)
    assert bench.fft_flops_per_point(128) == pytest.approx(245.28125)


def test_kernel_model_fft_replaces_the_direct_count():
    npts, nk = 1 << 20, 128
    _, direct = bench.kernel_model("theta_stage1", npts, 8, nk, 1, "fp64")
    _, fft = bench.kernel_model("theta_stage1", npts, 8, nk, 1, "fp64", fft=True)
    assert direct == pytest.approx(bench.theta_flops_per_point(nk, 1) * npts)
    assert fft == pytest.approx(bench.fft_flops_per_point(nk) * npts)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
