"""The one-pass Heun step of the general Theta kernel (torus, nk = 32..128):
out = f + (tau/2)(Theta f + Theta g), g = f + tau Theta f, with the plane kept
in LDS between the two applications (pair tiles scattered through it, f
re-read at each lane's points), against the FP64 oracle's Strang steps and
against the streaming kernel's Heun step.  It serves every Strang step
whose single-body band is too wide for the streaming kernel (the mean field,
dense potentials) and the forced "general" path.

FP64 bar: eps_inf = max|f - f_ref| / max|f_ref| <= 1e-12; FP32: 2e-5 after
3 steps (the streaming FP32 path's bound).
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


VEXT = {
    "cos": I.cosine(0.5, 20.0),                                                   # band 1
    "3modes": I.fourier_modes([(0.4, 0.1), (-0.25, 0.2), (0.15, -0.05)], 20.0),  # band 3
}
V12 = I.smoothed_coulomb(1.0, 1.0)


def solver(nx, precision="fp64", pot="cos", two=True, lam=0.0, path="general", dt=0.005):
    from paper_2511_11354_amd import wig2

    s = wig2.Solver(nx, 128, dt=dt, precision=precision, meanfield_lambda=lam)
    s.set_potentials(VEXT[pot], V12 if two else None)
    s.set_theta_path(path)
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=7 + nx, period=20.0)
    s.set_state(f0)
    return s, f0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("nx,pot,two,lam", [(6, "cos", True, 0.0), (5, "3modes", False, 0.0),
                                            (8, "cos", True, 1.0), (7, "3modes", True, 0.5)])
def test_general_heun_steps_match_oracle(orc, nx, pot, two, lam):
    s, f0 = solver(nx, pot=pot, two=two, lam=lam)
    assert s.theta_path() == "general"
    g = orc.grid(nx, 128, True, 1, -10.0, 10.0)
    tb = orc.tables(g, VEXT[pot], V12 if two else None)
    print(f"general heun nx={nx} {pot} two={two} lam={lam}: ", end="", flush=True)
    s.step(3)
    ref = orc.step(g, f0, tb, 3, 0.005, lam=lam, two_body=two)
    e = eps_inf(s.get_state(), ref)
    print(f"3 steps eps_inf {e:.3e}", flush=True)
    assert e <= 1e-12


@pytest.mark.timeout(300)
def test_general_heun_fp32(orc):
    s, f0 = solver(6, precision="fp32", lam=1.0)
    g = orc.grid(6, 128, True, 1, -10.0, 10.0)
    s.step(3)
    ref = orc.step(g, f0, orc.tables(g, VEXT["cos"], V12), 3, 0.005, lam=1.0)
    e = eps_inf(s.get_state(), ref)
    print(f"general heun fp32 lam=1: 3 steps eps_inf {e:.3e}", flush=True)
    assert e <= 2e-5


@pytest.mark.timeout(300)
@pytest.mark.parametrize("scheme", ["strang", "lawson"])
@pytest.mark.parametrize("nx,nk", [(12, 32), (9, 48), (8, 64), (6, 96)])
def test_general_heun_smaller_planes(orc, nx, nk, scheme):
    """The one-pass form at every other plane size it serves (Strang; Lawson
    keeps the two stages), with the Hartree mean field (dense symbols)."""
    from paper_2511_11354_amd import wig2

    s = wig2.Solver(nx, nk, dt=0.005, scheme=scheme, meanfield_lambda=1.0)
    s.set_potentials(VEXT["cos"], V12)
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=3 + nk, period=20.0)
    s.set_state(f0)
    assert s.theta_path() == "general"
    g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
    s.step(3)
    ref = orc.step(g, f0, orc.tables(g, VEXT["cos"], V12), 3, 0.005, scheme=scheme, lam=1.0)
    e = eps_inf(s.get_state(), ref)
    print(f"general heun {scheme} {nx}^2 x {nk}^2 lam=1: 3 steps eps_inf {e:.3e}", flush=True)
    assert e <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
def test_general_heun_matches_stream_heun(precision, tol):
    """Band-1 potential: the one-pass general Heun and the streaming kernel's
    one-pass Heun are the same step up to rounding."""
    s1, _ = solver(8, precision=precision, path="general")
    s2, _ = solver(8, precision=precision, path="stream")
    assert s1.theta_path() == "general" and s2.theta_path() == "stream"
    s1.step(2)
    s2.step(2)
    e = eps_inf(s1.get_state(), s2.get_state())
    print(f"general vs stream heun {precision}: 2 steps eps_inf {e:.3e}", flush=True)
    assert e <= tol
