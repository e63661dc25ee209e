"""The streaming Theta kernel (persistent workgroups, next-plane prefetch,
pair term from skewed tiles, single-body differences on the vector ALUs)
against the FP64 oracle and against the general kernel.

It is selected automatically for a torus with a single-body band of at most
4 modes at the plane sizes where it is the faster kernel; these tests force
it at every size it supports, and check the automatic choice.  The Heun step is
evaluated as g = f + tau Theta f, f' = (f + g)/2 + (tau/2) Theta g, which
differs from the oracle's f + (tau/2)(Theta f + Theta g) only by rounding.
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


POTS = {
    "cos": I.cosine(0.5, 20.0),                                           # band 1
    "3modes": I.fourier_modes([(0.4, 0.1), (-0.25, 0.2), (0.15, -0.05)], 20.0),  # band 3
    "zero": I.zero(),                                                     # band 0
}


def solver(nx, nk, pot, two, precision="fp64", scheme="strang", dt=0.01, path="stream"):
    from paper_2511_11354_amd import wig2

    s = wig2.Solver(nx, nk, dt=dt, scheme=scheme, precision=precision)
    s.set_potentials(POTS[pot], I.smoothed_coulomb(1.3, 1.0) if two else None)
    s.set_theta_path(path)
    return s


@pytest.mark.parametrize("nx,nk", [(9, 32), (7, 48), (6, 64), (5, 96), (5, 128), (17, 128)])
@pytest.mark.parametrize("pot", ["cos", "3modes", "zero"])
@pytest.mark.parametrize("two", [True, False])
def test_stream_theta_matches_oracle(orc, nx, nk, pot, two):
    s = solver(nx, nk, pot, two)
    assert s.theta_path() == "stream"
    g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
    tb = orc.tables(g, POTS[pot], I.smoothed_coulomb(1.3, 1.0) if two else None)
    f = I.random_field((nx, nx, nk, nk), seed=31 * nx + nk)
    ref = orc.theta_periodic(g, tb["sig_ext"], tb["sig_ext"], tb["vhat12"], f, two)
    fin = torch.from_numpy(f).cuda()
    # NaN-filled outputs: every point must be written
    out = torch.full_like(fin, float("nan"))
    torch.cuda.synchronize()  # the fill runs on torch's stream, Theta on the context's
    s.theta(fin, out)
    s.set_theta_path("general")
    out_g = torch.full_like(fin, float("nan"))
    torch.cuda.synchronize()  # the fill runs on torch's stream, Theta on the context's
    s.theta(fin, out_g)
    torch.cuda.synchronize()
    got, gen = out.cpu().numpy(), out_g.cpu().numpy()
    if pot == "zero" and not two:
        # no potential at all: Theta f = 0 exactly, on both kernels
        print(f"stream theta nx={nx} nk={nk} without potentials: max |out| {np.abs(got).max():.1e}", flush=True)
        assert np.max(np.abs(ref)) == 0.0
        assert np.all(got == 0.0) and np.all(gen == 0.0)
        return
    e, eg = eps_inf(got, ref), eps_inf(got, gen)
    print(f"stream theta nx={nx} nk={nk} {pot} two={two}: vs oracle {e:.3e}, vs general {eg:.3e}",
          flush=True)
    assert e <= 1e-12 and eg <= 1e-13


@pytest.mark.parametrize("scheme", ["strang", "lawson"])
@pytest.mark.parametrize("nx,nk,pot", [(32, 32, "cos"), (12, 64, "3modes"), (8, 128, "cos")])
def test_stream_steps_match_oracle(orc, scheme, nx, nk, pot):
    s = solver(nx, nk, pot, True, scheme=scheme, dt=0.005)
    assert s.theta_path() == "stream"
    g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
    tb = orc.tables(g, POTS[pot], I.smoothed_coulomb(1.3, 1.0))
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=nx + nk, period=20.0)
    s.set_state(f0)
    s.step(1)
    e1 = eps_inf(s.get_state(), orc.step(g, f0, tb, 1, 0.005, scheme=scheme))
    s.step(4)
    ref = orc.step(g, f0, tb, 5, 0.005, scheme=scheme)
    e5 = eps_inf(s.get_state(), ref)
    print(f"stream {scheme} nx={nx} nk={nk} {pot}: eps_inf 1 step {e1:.3e}, 5 steps {e5:.3e}",
          flush=True)
    assert e1 <= 1e-12 and e5 <= 1e-12


def test_stream_tiny_workload_20_steps(orc):
    """Periodic 32^4 workload, 20 steps of both schemes through the streaming
    kernel (its default path)."""
    w = I.tiny_periodic()
    g = orc.grid(w.nx, w.nk, True, 1, w.x_min, w.x_max)
    tb = orc.tables(g, w.vext, w.v12)
    for scheme in ("strang", "lawson"):
        from paper_2511_11354_amd import wig2

        s = wig2.Solver(w.nx, w.nk, dt=w.dt, scheme=scheme)
        s.set_potentials(w.vext, w.v12)
        assert s.theta_path() == "stream"
        x, p, _ = s.nodes()
        f0 = I.symmetrised_pair(x, p)
        s.set_state(f0)
        s.step(20)
        e = eps_inf(s.get_state(), orc.step(g, f0, tb, 20, w.dt, scheme=scheme))
        print(f"32^4 {scheme} 20 steps (stream): eps_inf {e:.3e}", flush=True)
        assert e <= 1e-12


@pytest.mark.parametrize("nk", [32, 48, 64, 96, 128])
def test_stream_fp32(orc, nk):
    nx = 8
    s = solver(nx, nk, "cos", True, precision="fp32", dt=0.005)
    assert s.theta_path() == "stream"
    g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
    tb = orc.tables(g, POTS["cos"], I.smoothed_coulomb(1.3, 1.0))
    f = I.random_field((nx, nx, nk, nk), seed=3)
    ref = orc.theta_periodic(g, tb["sig_ext"], tb["sig_ext"], tb["vhat12"], f, True)
    fin = torch.from_numpy(f).float().cuda()
    out = torch.full_like(fin, float("nan"))  # every point must be written
    s.theta(fin, out)
    torch.cuda.synchronize()
    e = eps_inf(out.double().cpu().numpy(), ref)
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=4, period=20.0)
    s.set_state(f0)
    s.step(5)
    es = eps_inf(s.get_state(), orc.step(g, f0, tb, 5, 0.005))
    print(f"stream fp32 nk={nk}: theta eps_inf {e:.3e}, 5 steps {es:.3e}", flush=True)
    assert e <= 2e-6 and es <= 1e-5


def test_stream_path_selection():
    from paper_2511_11354_amd import wig2

    s = wig2.Solver(8, 64, dt=0.01)
    s.set_potentials(I.double_well(), I.smoothed_coulomb(1.0, 1.0))  # dense band
    assert s.theta_path() == "general"
    with pytest.raises(wig2.Wig2Error):
        s.set_theta_path("stream")
    s2 = wig2.Solver(8, 16, dt=0.01)  # nk = 16: general only
    s2.set_potentials(I.cosine(0.5, 20.0), None)
    assert s2.theta_path() == "general"
    s3 = wig2.Solver(8, 64, dt=0.01, precision="bf16x2")  # split-BF16 streaming kernel
    s3.set_potentials(I.cosine(0.5, 20.0), None)
    assert s3.theta_path() == "stream"
    # automatic choice: the streaming kernel at every plane size it supports
    for prec, nk, want in (("fp64", 64, "stream"), ("fp32", 128, "stream"), ("fp32", 64, "stream"),
                           ("fp32", 96, "stream"), ("fp32", 32, "stream"), ("fp64", 48, "stream")):
        s4 = wig2.Solver(4, nk, dt=0.01, precision=prec)
        s4.set_potentials(I.cosine(0.5, 20.0), I.smoothed_coulomb(1.0, 1.0))
        assert s4.theta_path() == want, (prec, nk)
        s4.set_theta_path("stream")
        assert s4.theta_path() == "stream"
