"""Multi-step Strang calls: the entering half-step sweeps go x1 then x2, the
leaving ones x2 then x1 (the two sweeps act on different axes and commute),
and the x1 half-sweep ending one step runs in the same launch as the one
beginning the next.

Checked here: n steps in one call are bitwise equal to n calls of one step
and to n steps with the joint launch switched off (same arithmetic, fewer
HBM round trips), for every Theta path and both element types; and the
multi-step result still meets the oracle's bar.
"""
import numpy as np
import pytest

from paper_2511_11354_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def eps_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


CASES = {
    # name: (nx, nk, periodic, cells, vext, v12, theta path)
    "stream-32": (32, 32, True, 1, I.cosine(0.5, 20.0), I.smoothed_coulomb(1.0, 1.0), "stream"),
    "stream-12x128": (12, 128, True, 1, I.cosine(0.5, 20.0), I.smoothed_coulomb(2.0, 1.0), "stream"),
    # six Fourier modes: wider than the streaming kernel's band, general kernel
    "general-48": (16, 48, True, 1,
                   I.fourier_modes([(0.3, 0.1), (-0.2, 0.1), (0.1, -0.05), (0.05, 0.05), (0.04, 0.0),
                                    (0.0, 0.03)], 20.0),
                   I.smoothed_coulomb(1.0, 1.0), "auto"),
    "box-33": (33, 32, False, 4, I.harmonic(0.5), None, "auto"),
    # nx = 24 has no register-resident sweep: the general sweep kernel, and
    # the two x1 half-sweeps as two launches through a work buffer
    "general-sweep-24": (24, 32, True, 1, I.cosine(0.5, 20.0), I.smoothed_coulomb(1.0, 1.0), "stream"),
    # 1024 planes of nk = 128: several planes per persistent workgroup, so the
    # cross-plane prefetch of the one-pass Heun kernel runs as at 128^4
    "stream-32x128": (32, 128, True, 1, I.cosine(0.5, 20.0), I.smoothed_coulomb(2.0, 1.0), "stream"),
    # nx = 128: the register-resident sweep of 128-point lines, and the joint
    # two-pass x1 launch of the 128^4 workload
    "stream-128x32": (128, 32, True, 1, I.cosine(0.5, 20.0), I.smoothed_coulomb(1.0, 1.0), "stream"),
    # nx = 256: segmented periodic lines (8 waves x 32 points per line), the
    # sweep of the Wigner-Poisson workloads, with its joint x1 launch
    "seg-256x16": (256, 16, True, 1, I.cosine(0.5, 20.0), I.smoothed_coulomb(1.0, 1.0), "auto"),
    # nx = 129 box: the natural-boundary register sweep of the box workload
    "box-129": (129, 32, False, 4, I.harmonic(0.5), None, "auto"),
}


def make(case, precision, fused=True):
    from paper_2511_11354_amd import wig2

    nx, nk, per, cells, vext, v12, path = CASES[case]
    kw = dict(periodic=per, sem_cells=cells, dt=0.005, precision=precision)
    if not per:
        kw.update(x_min=-15.0, x_max=15.0, k_max=10.0 * np.pi / 3.0)
    s = wig2.Solver(nx, nk, **kw)
    s.set_potentials(vext, v12)
    s.set_theta_path(path)
    s.set_sweep_fusion(fused)
    x, p, _ = s.nodes()
    if per:
        f0 = I.mixture(x, p, seed=nx + nk, period=20.0)
    else:
        f0 = I.symmetrised_pair(x, p, a=(-2.0, 2.0), q=(0.0, 0.0))
    s.set_state(f0)
    return s, f0


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("n", [3, 4])
def test_multi_step_bitwise(case, precision, n):
    s1, _ = make(case, precision)
    s1.step(n)
    many = s1.get_state()
    if CASES[case][6] == "auto" and CASES[case][2]:
        assert s1.theta_path() == "general"
    s2, _ = make(case, precision)
    for _ in range(n):
        s2.step(1)
    one_by_one = s2.get_state()
    s3, _ = make(case, precision, fused=False)
    s3.step(n)
    unfused = s3.get_state()
    ob = s1.observables()
    print(f"{case} {precision} n={n}: theta path {s1.theta_path()}, step {ob['step']}, "
          f"max|diff| one-by-one {np.abs(many - one_by_one).max():.3e}, "
          f"unfused {np.abs(many - unfused).max():.3e}", flush=True)
    assert ob["step"] == n
    assert np.array_equal(many, one_by_one)
    assert np.array_equal(many, unfused)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("case", sorted(CASES))
def test_multi_step_matches_oracle(orc, case):
    nx, nk, per, cells, vext, v12, _ = CASES[case]
    s, f0 = make(case, "fp64")
    s.step(6)
    if per:
        g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
    else:
        g = orc.grid(nx, nk, False, cells, -15.0, 15.0, 10.0 * np.pi / 3.0)
    ref = orc.step(g, f0, orc.tables(g, vext, v12), 6, 0.005)
    e = eps_inf(s.get_state(), ref)
    print(f"{case}: 6 steps in one call vs oracle eps_inf {e:.3e}", flush=True)
    assert e <= 1e-12


@pytest.mark.timeout(600)
@pytest.mark.parametrize("case", ["stream-32x128", "stream-128x32", "box-129", "seg-256x16"])
def test_multi_step_fp32_matches_oracle(orc, case):
    """The FP32 form of the same launch configurations, 3 steps in one call,
    against the FP64 oracle at the FP32 bound (state rounding ~6e-8 per step
    plus FP32 operator sums)."""
    nx, nk, per, cells, vext, v12, _ = CASES[case]
    s, f0 = make(case, "fp32")
    s.step(3)
    if per:
        g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
    else:
        g = orc.grid(nx, nk, False, cells, -15.0, 15.0, 10.0 * np.pi / 3.0)
    ref = orc.step(g, f0, orc.tables(g, vext, v12), 3, 0.005)
    e = eps_inf(s.get_state(), ref)
    print(f"{case} fp32: 3 steps in one call vs oracle eps_inf {e:.3e}", flush=True)
    assert e <= 2e-6
