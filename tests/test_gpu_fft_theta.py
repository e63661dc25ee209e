"""The FFT route to Theta on the torus (the FFT-accelerated two-body cost of
Sec. 3.1.2): each momentum plane's row, column and anti-diagonal
pseudo-differences as one 2-D convolution, zero-padded to N = 2 nk
(nk = 16, 32, 48, 64, 96, 128; N = 2 nk rounded up to 64 R with an in-lane
radix R = 1, 1, 2, 2, 3, 4),
IFFT2(W . FFT2(f)).  Checked against the FP64 oracle's direct sums for single
applications, whole Strang and Lawson steps and the Hartree mean field, where
the single-body symbols are dense.  Also checked against the direct MFMA
kernels at the full 128^4 size.

FP64 bar: eps_inf = max|f - f_ref| / max|f_ref| <= 1e-12.  FP32: 2e-6 per
application, the direct FP32 kernels' bound (the transforms' log2 N
roundings stay near 2e-7 relative at these sizes).
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


POT = {"cos": I.cosine(0.5, 20.0), "dw": I.double_well()}
V12 = I.smoothed_coulomb(1.3, 1.0)


def solver(orc, nx, nk, *, pot="cos", two=True, precision="fp64", scheme="strang", lam=0.0, dt=0.01,
           path="fft"):
    from paper_2511_11354_amd import wig2

    s = wig2.Solver(nx, nk, dt=dt, scheme=scheme, precision=precision, meanfield_lambda=lam)
    s.set_potentials(POT[pot], V12 if two else None)
    s.set_theta_path(path)
    return s, orc.grid(nx, nk, True, 1, -10.0, 10.0)


@pytest.mark.parametrize("nx,nk,pot,two", [(8, 32, "cos", True), (6, 64, "dw", True), (4, 128, "cos", True),
                                           (5, 128, "dw", True), (6, 64, "dw", False), (5, 96, "dw", True),
                                           (7, 48, "cos", True), (9, 16, "dw", True)])
def test_fft_theta_matches_oracle(orc, nx, nk, pot, two):
    s, g = solver(orc, nx, nk, pot=pot, two=two)
    assert s.theta_path() == "fft"
    f = I.random_field((nx, nx, nk, nk), seed=nx * 100 + nk)
    tb = orc.tables(g, POT[pot], V12 if two else None)
    ref = orc.theta_periodic(g, tb["sig_ext"], tb["sig_ext"], tb["vhat12"], f, two)
    out = torch.full(f.shape, float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()  # the fill runs on torch's stream, Theta on the context's
    print(f"fft theta nx={nx} nk={nk} {pot} two={two}: ", end="", flush=True)
    s.theta(torch.from_numpy(f).cuda(), out)
    torch.cuda.synchronize()
    e = eps_inf(out.cpu().numpy(), ref)
    print(f"eps_inf {e:.3e}", flush=True)
    assert e <= 1e-12


@pytest.mark.parametrize("nx,nk", [(8, 32), (7, 48), (6, 64), (4, 96), (4, 128)])
def test_fft_theta_fp32(orc, nx, nk):
    s, g = solver(orc, nx, nk, pot="dw", precision="fp32")
    f = I.random_field((nx, nx, nk, nk), seed=11 + nk)
    tb = orc.tables(g, POT["dw"], V12)
    ref = orc.theta_periodic(g, tb["sig_ext"], tb["sig_ext"], tb["vhat12"], f, True)
    out = torch.full(f.shape, float("nan"), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()  # the fill runs on torch's stream, Theta on the context's
    s.theta(torch.from_numpy(f).float().cuda(), out)
    torch.cuda.synchronize()
    e = eps_inf(out.double().cpu().numpy(), ref)
    print(f"fft theta fp32 nx={nx} nk={nk}: eps_inf {e:.3e}", flush=True)
    assert e <= 2e-6


@pytest.mark.timeout(300)
@pytest.mark.parametrize("scheme", ["strang", "lawson"])
@pytest.mark.parametrize("nx,nk,lam", [(10, 16, 1.0), (8, 32, 0.0), (7, 48, 1.0), (6, 64, 1.0), (5, 96, 1.0), (5, 128, 1.0),
                                       (4, 128, 0.0)])
def test_fft_steps_match_oracle(orc, scheme, nx, nk, lam):
    s, g = solver(orc, nx, nk, scheme=scheme, lam=lam, dt=0.005)
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=5 + nk, period=20.0)
    s.set_state(f0)
    print(f"fft {scheme} nx={nx} nk={nk} lam={lam}: ", end="", flush=True)
    s.step(3)
    ref = orc.step(g, f0, orc.tables(g, POT["cos"], V12), 3, 0.005, scheme=scheme, lam=lam)
    e = eps_inf(s.get_state(), ref)
    print(f"3 steps eps_inf {e:.3e}", flush=True)
    assert s.theta_path() == "fft"
    assert e <= 1e-12


@pytest.mark.timeout(300)
def test_fft_matches_stream_at_full_size():
    """128^4 FP64, the headline workload: one Strang step on the FFT path
    (16384 planes per launch) against the streaming kernel's."""
    from paper_2511_11354_amd import wig2

    nx, nk = 128, 128
    res = []
    for path in ("fft", "stream"):
        s = wig2.Solver(nx, nk, dt=0.01)
        s.set_potentials(POT["cos"], V12)
        s.set_theta_path(path)
        x, p, _ = s.nodes()
        s.set_state(I.mixture(x, p, seed=3, period=20.0))
        print(f"128^4 {path}: ", end="", flush=True)
        s.step(1)
        res.append(s.get_state())
        print("stepped", flush=True)
        del s
        torch.cuda.empty_cache()
    e = eps_inf(res[0], res[1])
    print(f"fft vs stream at 128^4, 1 step: eps_inf {e:.3e}", flush=True)
    assert e <= 1e-12


def test_fft_path_rejected_where_it_does_not_apply():
    from paper_2511_11354_amd import wig2

    # (every torus plane size a context accepts, 16 ... 128, has the FFT route)
    for kw in [dict(nx=5, nk=32, precision="bf16x2"),
               dict(nx=7, nk=32, periodic=False, sem_cells=4, x_min=-6.0, x_max=6.0, k_max=10 * np.pi / 3)]:
        nx, nk = kw.pop("nx"), kw.pop("nk")
        s = wig2.Solver(nx, nk, **kw)
        s.set_potentials(I.harmonic(0.5) if "periodic" in kw else POT["cos"], None)
        with pytest.raises(Exception):
            s.set_theta_path("fft")
        assert s.theta_path() != "fft"


@pytest.mark.timeout(300)
def test_fft_steps_with_xc_match_oracle(orc):
    """Hartree plus the H-L exchange-correlation term (dense symbols from the
    density) on the FFT route, 3 Strang steps against the oracle."""
    from paper_2511_11354_amd import wig2

    nx, nk, dt = 6, 64, 0.005
    s = wig2.Solver(nx, nk, dt=dt, meanfield_lambda=1.0, xc=1, xc_n0=0.05, n_scale=1.0)
    s.set_potentials(POT["cos"], V12)
    s.set_theta_path("fft")
    g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=9, period=20.0)
    s.set_state(f0)
    s.step(3)
    tb = orc.tables(g, POT["cos"], V12)
    ref = orc.step(g, f0, tb, 3, dt, lam=1.0, xc=True, xc_n0=0.05, n_scale=1.0)
    nomf = orc.step(g, f0, tb, 3, dt)
    e = eps_inf(s.get_state(), ref)
    print(f"fft with Hartree + XC: 3 steps eps_inf {e:.3e} (mean field moves the state by {eps_inf(ref, nomf):.3e})",
          flush=True)
    assert eps_inf(ref, nomf) > 1e-6
    assert e <= 1e-12
