"""The box two-body operator (Sec. 3.2.2: y-lattice, D_V, the two-body
tensor) on the matrix cores against the FP64 oracle, through the C ABI:
single applications of Theta (single-body SEM matrices plus the pair term)
at every plane size the box supports, in FP64 and FP32, in place and out of
place, and whole Strang and Lawson steps of a box with a pair potential.

FP64 bar: eps_inf = max|f - f_ref| / max|f_ref| <= 1e-12.  FP32: 2e-5 for one
application (24 nk flops per point accumulated in FP32 through four chained
products), 1e-4 after 3 steps.
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


def make(orc, nx, nk, cells, precision="fp64", scheme="strang", dt=0.01, k_max=10 * np.pi / 3, half=6.0):
    """A box [-half, half] with nx nodes and nk = cells x nodes momenta."""
    from paper_2511_11354_amd import wig2

    s = wig2.Solver(nx, nk, periodic=False, sem_cells=cells, x_min=-half, x_max=half, k_max=k_max, dt=dt,
                    scheme=scheme, precision=precision)
    s.set_potentials(VEXT, V12)
    g = orc.grid(nx, nk, False, cells, -half, half, k_max)
    return s, g


def oracle_theta(orc, g, f):
    tb = orc.tables(g, VEXT, V12)
    return orc.theta_dense(g, tb["K"], tb["K"], f) + orc.theta12_sem(g, tb["v12_sem"], f)


@pytest.mark.parametrize("nx,nk,cells", [(7, 32, 4), (6, 64, 8), (5, 96, 6), (4, 128, 8), (5, 256, 16)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_box_pair_theta_matches_oracle(orc, nx, nk, cells, precision):
    s, g = make(orc, nx, nk, cells, precision)
    x, p, _ = s.nodes()
    f = I.symmetrised_pair(x, p, a=(-2.0, 1.5), q=(0.3, -0.4))
    ref = oracle_theta(orc, g, f)
    tb = orc.tables(g, VEXT, V12)
    pair = orc.theta12_sem(g, tb["v12_sem"], f)
    dt = torch.float64 if precision == "fp64" else torch.float32
    fin = torch.from_numpy(f).to(device="cuda", dtype=dt)
    out = torch.full_like(fin, float("nan"))  # every point must be written
    torch.cuda.synchronize()  # the fill runs on torch's stream, Theta on the context's
    print(f"box pair theta {precision} nx={nx} nk={nk}: ", end="", flush=True)
    s.theta(fin, out)
    torch.cuda.synchronize()
    e = eps_inf(out.double().cpu().numpy(), ref)
    print(f"eps_inf {e:.3e} (pair term max {np.abs(pair).max():.3e} of {np.abs(ref).max():.3e})", flush=True)
    assert np.abs(pair).max() > 0.05 * np.abs(ref).max()
    assert e <= (1e-12 if precision == "fp64" else 2e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_box_pair_theta_in_place(orc, precision):
    """Output aliasing the input takes the accumulator route: the result is
    bitwise the out-of-place one."""
    s, _ = make(orc, 6, 64, 8, precision)
    x, p, _ = s.nodes()
    f = I.symmetrised_pair(x, p, a=(-2.0, 1.5), q=(0.3, -0.4))
    dt = torch.float64 if precision == "fp64" else torch.float32
    fin = torch.from_numpy(f).to(device="cuda", dtype=dt)
    out = torch.full_like(fin, float("nan"))  # every point must be written
    torch.cuda.synchronize()  # the fill runs on torch's stream, Theta on the context's
    s.theta(fin, out)
    s.theta(fin, fin)
    torch.cuda.synchronize()
    assert torch.equal(out, fin)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("scheme", ["strang", "lawson"])
@pytest.mark.parametrize("nx,nk,cells,half", [(33, 32, 4, 15.0), (9, 64, 8, 8.0)])
def test_box_pair_steps_match_oracle(orc, scheme, nx, nk, cells, half):
    s, g = make(orc, nx, nk, cells, scheme=scheme, dt=0.01, half=half)
    x, p, _ = s.nodes()
    f0 = I.symmetrised_pair(x, p, a=(-2.0, 2.0), q=(0.0, 0.0))
    tb = orc.tables(g, VEXT, V12)
    s.set_state(f0)
    print(f"box pair {scheme} nx={nx} nk={nk}: ", end="", flush=True)
    s.step(3)
    ref = orc.step(g, f0, tb, 3, 0.01, scheme=scheme)
    nov = orc.step(g, f0, orc.tables(g, VEXT, None), 3, 0.01, scheme=scheme)
    e = eps_inf(s.get_state(), ref)
    print(f"3 steps eps_inf {e:.3e} (pair term moves the state by {eps_inf(ref, nov):.3e})", flush=True)
    assert eps_inf(ref, nov) > 1e-4
    assert e <= 1e-12


def test_box_pair_fp32_steps(orc):
    s, g = make(orc, 17, 64, 8, precision="fp32", dt=0.01, half=8.0)
    x, p, _ = s.nodes()
    f0 = I.symmetrised_pair(x, p, a=(-2.0, 2.0), q=(0.0, 0.0))
    s.set_state(f0)
    s.step(3)
    ref = orc.step(g, f0, orc.tables(g, VEXT, V12), 3, 0.01)
    e = eps_inf(s.get_state(), ref)
    print(f"box pair fp32 3 steps eps_inf {e:.3e}", flush=True)
    assert e <= 1e-4


def test_box_pair_nk256_panel_step(orc):
    """nk = 256 boxes take the panel single-body kernel (one-operand forms);
    the pair term rides on its forms."""
    s, g = make(orc, 5, 256, 16, dt=0.01)
    x, p, _ = s.nodes()
    f0 = I.symmetrised_pair(x, p, a=(-2.0, 2.0), q=(0.0, 0.0))
    s.set_state(f0)
    s.step(1)
    ref = orc.step(g, f0, orc.tables(g, VEXT, V12), 1, 0.01)
    e = eps_inf(s.get_state(), ref)
    print(f"box pair nk=256 panel 1 step eps_inf {e:.3e}", flush=True)
    assert e <= 1e-12
