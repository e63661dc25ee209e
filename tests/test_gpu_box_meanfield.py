"""The mean field on a box (Sec. 3.2.1 with Sec. 2.3): particle j's SEM matrices
become those of V_ext + V_eff,j, rebuilt on the device before every Theta
evaluation, the Hartree term being the direct convolution with V12 (equal to
the zero-padded transform on 3 nx points, no wrap-around).  Single Theta
applications and whole Strang and Lawson steps against the FP64 oracle,
through the C ABI, with and without the pair term and the H-L XC term, at
plane sizes of the general (nk <= 128) and the panel (nk = 256) kernels.

FP64 bar: eps_inf = max|f - f_ref| / max|f_ref| <= 1e-12.  FP32: 2e-5 for one
application, 1e-4 after 3 steps; BF16X2 (split bf16 operands on the panel
kernel): 2e-4 for one application.
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


VEXT = I.harmonic(0.5)
V12 = I.smoothed_coulomb(1.5, 1.0)
LAM, XC_N0, N_SCALE = 1.0, 0.05, 1.0


def make(orc, nx, nk, cells, *, pair=True, xc=False, lam=LAM, precision="fp64", scheme="strang", dt=0.01,
         half=6.0, k_max=10 * np.pi / 3):
    from paper_2511_11354_amd import wig2

    s = wig2.Solver(nx, nk, periodic=False, sem_cells=cells, x_min=-half, x_max=half, k_max=k_max, dt=dt,
                    scheme=scheme, precision=precision, meanfield_lambda=lam, xc=int(xc), xc_n0=XC_N0,
                    n_scale=N_SCALE)
    s.set_potentials(VEXT, V12 if pair else None)
    g = orc.grid(nx, nk, False, cells, -half, half, k_max)
    return s, g


def oracle_theta(orc, g, f, pair, xc, lam=LAM):
    """Theta with the mean field of f: K_j = K[V_ext + V_eff,j] (+ Theta_12);
    without a pair potential the Hartree term vanishes."""
    tb = orc.tables(g, VEXT, V12 if pair else None)
    n1, n2 = orc.densities(g, f)
    v1 = orc.veff_hxc(g, lam, xc, XC_N0, N_SCALE, tb["v12_pair"], n1)
    v2 = orc.veff_hxc(g, lam, xc, XC_N0, N_SCALE, tb["v12_pair"], n2)
    vx = tb["vext_x"]
    out = orc.theta_dense(g, orc.sem_kernel(g, vx + v1), orc.sem_kernel(g, vx + v2), f)
    if pair:
        out = out + orc.theta12_sem(g, tb["v12_sem"], f)
    return out


@pytest.mark.parametrize("nx,nk,cells", [(7, 32, 4), (6, 64, 8), (5, 128, 8), (5, 256, 16)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("pair,xc", [(True, False), (False, True)])
def test_box_meanfield_theta_matches_oracle(orc, nx, nk, cells, precision, pair, xc):
    s, g = make(orc, nx, nk, cells, pair=pair, xc=xc, precision=precision)
    x, p, _ = s.nodes()
    f = I.symmetrised_pair(x, p, a=(-2.0, 1.5), q=(0.3, -0.4))
    ref = oracle_theta(orc, g, f, pair, xc)
    tb = orc.tables(g, VEXT, V12)
    nomf = orc.theta_dense(g, tb["K"], tb["K"], f) + (orc.theta12_sem(g, tb["v12_sem"], f) if pair else 0.0)
    dt = torch.float64 if precision == "fp64" else torch.float32
    fin = torch.from_numpy(f).to(device="cuda", dtype=dt)
    out = torch.full_like(fin, float("nan"))
    torch.cuda.synchronize()  # the fill runs on torch's stream, Theta on the context's
    print(f"box mean field theta {precision} nx={nx} nk={nk} pair={pair} xc={xc}: ", end="", flush=True)
    s.theta(fin, out)
    torch.cuda.synchronize()
    e = eps_inf(out.double().cpu().numpy(), ref)
    print(f"eps_inf {e:.3e} (the mean field moves Theta by {eps_inf(nomf, ref):.3e})", flush=True)
    assert eps_inf(nomf, ref) > 1e-3
    assert e <= (1e-12 if precision == "fp64" else 2e-5)


def test_box_meanfield_theta_bf16x2_panel(orc):
    s, g = make(orc, 5, 256, 16, pair=True, xc=True, precision="bf16x2")
    x, p, _ = s.nodes()
    f = I.symmetrised_pair(x, p, a=(-2.0, 1.5), q=(0.3, -0.4))
    ref = oracle_theta(orc, g, f, True, True)
    fin = torch.from_numpy(f).to(device="cuda", dtype=torch.float32)
    out = torch.full_like(fin, float("nan"))
    torch.cuda.synchronize()  # the fill runs on torch's stream, Theta on the context's
    s.theta(fin, out)
    torch.cuda.synchronize()
    e = eps_inf(out.double().cpu().numpy(), ref)
    print(f"box mean field theta bf16x2 nk=256: eps_inf {e:.3e}", flush=True)
    assert e <= 2e-4


@pytest.mark.timeout(300)
@pytest.mark.parametrize("scheme", ["strang", "lawson"])
@pytest.mark.parametrize("nx,nk,cells,half,pair,xc", [(17, 32, 4, 8.0, True, True), (9, 64, 8, 8.0, False, True),
                                                       (9, 64, 8, 8.0, True, False)])
def test_box_meanfield_steps_match_oracle(orc, scheme, nx, nk, cells, half, pair, xc):
    s, g = make(orc, nx, nk, cells, pair=pair, xc=xc, scheme=scheme, half=half)
    x, p, _ = s.nodes()
    f0 = I.symmetrised_pair(x, p, a=(-2.0, 2.0), q=(0.0, 0.0))
    s.set_state(f0)
    tb = orc.tables(g, VEXT, V12 if pair else None)
    print(f"box mean field {scheme} nx={nx} nk={nk} pair={pair} xc={xc}: ", end="", flush=True)
    s.step(3)
    ref = orc.step(g, f0, tb, 3, 0.01, scheme=scheme, lam=LAM, xc=xc, xc_n0=XC_N0, n_scale=N_SCALE)
    nomf = orc.step(g, f0, tb, 3, 0.01, scheme=scheme)
    e = eps_inf(s.get_state(), ref)
    print(f"3 steps eps_inf {e:.3e} (the mean field moves the state by {eps_inf(ref, nomf):.3e})", flush=True)
    assert eps_inf(ref, nomf) > 1e-5
    assert e <= 1e-12


def test_box_meanfield_fp32_steps(orc):
    s, g = make(orc, 17, 64, 8, pair=True, xc=True, precision="fp32", half=8.0)
    x, p, _ = s.nodes()
    f0 = I.symmetrised_pair(x, p, a=(-2.0, 2.0), q=(0.0, 0.0))
    s.set_state(f0)
    s.step(3)
    ref = orc.step(g, f0, orc.tables(g, VEXT, V12), 3, 0.01, lam=LAM, xc=True, xc_n0=XC_N0, n_scale=N_SCALE)
    e = eps_inf(s.get_state(), ref)
    print(f"box mean field fp32 3 steps eps_inf {e:.3e}", flush=True)
    assert e <= 1e-4


@pytest.mark.parametrize("scheme", ["strang", "lawson"])
def test_box_meanfield_nk256_panel_step(orc, scheme):
    """nk = 256 boxes take the panel kernel; particle 2 reads its own matrices."""
    s, g = make(orc, 5, 256, 16, pair=True, xc=True, scheme=scheme)
    x, p, _ = s.nodes()
    f0 = I.symmetrised_pair(x, p, a=(-2.0, 2.0), q=(0.0, 0.0))
    s.set_state(f0)
    s.step(1)
    ref = orc.step(g, f0, orc.tables(g, VEXT, V12), 1, 0.01, scheme=scheme, lam=LAM, xc=True, xc_n0=XC_N0,
                   n_scale=N_SCALE)
    e = eps_inf(s.get_state(), ref)
    print(f"box mean field nk=256 panel {scheme} 1 step eps_inf {e:.3e}", flush=True)
    assert e <= 1e-12


def test_box_poisson_hartree_rejected():
    """The neutralised Poisson form needs a torus."""
    from paper_2511_11354_amd import wig2

    s = wig2.Solver(7, 32, periodic=False, sem_cells=4, x_min=-6.0, x_max=6.0, k_max=10 * np.pi / 3,
                    meanfield_lambda=1.0)
    with pytest.raises(Exception):
        s.set_hartree("poisson")
