"""Parity at the full 128^4 periodic workload, in the launch configuration
the benchmark times: the oracle recomputes sampled planes (Theta) and sampled
lines (advection) one by one; whole steps are checked through properties that
hold at any size, and a whole step is compared in full at 64^4."""
import numpy as np
import pytest

from paper_2511_11354_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def big(orc):
    from paper_2511_11354_amd import wig2

    w = I.large_periodic(u=1.0)
    s = wig2.Solver(w.nx, w.nk, x_min=w.x_min, x_max=w.x_max, dt=w.dt)
    s.set_potentials(w.vext, w.v12)
    g = orc.grid(w.nx, w.nk, True, 1, w.x_min, w.x_max)
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=0, period=w.x_max - w.x_min)
    tb = orc.tables(g, w.vext, w.v12)
    print("128^4 input ready", flush=True)
    return w, s, g, f0, tb


def test_theta_sampled_planes(orc, big):
    w, s, g, f0, tb = big
    fin = torch.from_numpy(f0).cuda()
    out = torch.full_like(fin, float("nan"))  # every point must be written
    s.theta(fin, out)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(out).any())
    got = out.cpu().numpy()
    del out, fin
    rng = np.random.default_rng(1)
    # random planes plus corners, the diagonal (no pair term) and the bulk
    planes = sorted(set(rng.integers(0, w.nx * w.nx, 24).tolist())
                    | {0, w.nx * w.nx - 1, w.nx + 1, 64 * w.nx + 64, 70 * w.nx + 50})
    err, scale = 0.0, 0.0
    for pl in planes:
        ref = orc.theta_periodic(g, tb["sig_ext"], tb["sig_ext"], tb["vhat12"], f0, True, pl, 1)
        i1, i2 = divmod(pl, w.nx)
        r, o = ref[i1, i2], got[i1, i2]
        err = max(err, np.abs(o - r).max())
        scale = max(scale, np.abs(r).max())
    # eps_inf over the sampled planes (global maximum as in Sec. 5.1); the
    # whole-grid maximum of |Theta f| bounds the sampled one from above
    e = err / scale
    print(f"128^4 theta over {len(planes)} planes: eps_inf {e:.3e} (scale {scale:.3e}, "
          f"grid max {np.abs(got).max():.3e})")
    assert scale > 0.1 * np.abs(got).max()
    assert e <= 1e-12


@pytest.mark.parametrize("dim", [1, 2])
def test_advect_sampled_lines(orc, big, dim):
    w, s, g, f0, tb = big
    fin = torch.from_numpy(f0).cuda()
    out = torch.full_like(fin, float("nan"))  # every point must be written
    s.advect(dim, 0.5 * w.dt, fin, out)
    torch.cuda.synchronize()
    assert not bool(torch.isnan(out).any())
    got = out.cpu().numpy()
    del out, fin
    nk2 = w.nk * w.nk
    worst = 0.0
    # runs of nk lines (fixed other-x index and n1, all n2) through the bulk
    # of the packets and one at the p-box edge
    for line0 in (64 * nk2 + 64 * w.nk, 40 * nk2 + 70 * w.nk, 100 * nk2 + 60 * w.nk,
                  127 * nk2 + 120 * w.nk):
        ref = orc.advect(g, dim, 0.5 * w.dt, f0, line0, w.nk)
        flat_r, flat_o = ref.reshape(-1), got.reshape(-1)
        # gather the touched lines
        for line in range(line0, line0 + w.nk):
            o_, rem = divmod(line, nk2)
            if dim == 1:
                idx = o_ * nk2 + rem + np.arange(w.nx) * w.nx * nk2
            else:
                idx = o_ * w.nx * nk2 + rem + np.arange(w.nx) * nk2
            r, o = flat_r[idx], flat_o[idx]
            worst = max(worst, np.abs(o - r).max() / np.abs(f0).max())
    print(f"128^4 advect dim {dim}: eps_inf {worst:.3e} (line max {np.abs(flat_r).max():.3e})")
    assert worst <= 1e-12


def test_step_properties_full_size(big):
    """One step of the 128^4 workload: mass changes only by p-edge leakage,
    exchange symmetry holds to rounding, and the step is deterministic."""
    w, s, g, f0, tb = big
    s.set_state(f0)
    ob0 = s.observables()
    s.step(1)
    ob1 = s.observables()
    f1 = s.get_state()
    sym = np.abs(f1 - f1.transpose(1, 0, 3, 2)).max() / np.abs(f1).max()
    print(f"128^4 one step: mass {ob0['mass']:.15f} -> {ob1['mass']:.15f}, symmetry {sym:.2e}")
    assert abs(ob1["mass"] - ob0["mass"]) < 1e-9
    assert sym < 1e-13
    s.set_state(f0)
    s.step(1)
    assert np.array_equal(s.get_state(), f1)


def test_step_mid_size_full_parity(orc):
    from paper_2511_11354_amd import wig2

    nx = nk = 64
    vext, v12 = I.cosine(0.5, 20.0), I.smoothed_coulomb(2.0, 1.0)
    s = wig2.Solver(nx, nk, dt=0.005)
    s.set_potentials(vext, v12)
    g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=2, period=20.0)
    s.set_state(f0)
    s.step(1)
    ref = orc.step(g, f0, orc.tables(g, vext, v12), 1, 0.005)
    e = np.abs(s.get_state() - ref).max() / np.abs(ref).max()
    print(f"64^4 one step eps_inf {e:.3e}")
    assert e <= 1e-12


@pytest.mark.timeout(900)
def test_two_steps_full_grid_vs_oracle(orc, big):
    """The benchmark's 128^4 FP64 workload, two Strang steps in one call (the
    one-pass Heun kernel with its cross-plane prefetch over all 16384 planes,
    and the joint two-pass x1 launch between the steps), compared point by
    point over the whole grid with two oracle steps."""
    w, s, g, f0, tb = big
    s.set_state(f0)
    s.step(2)
    got = s.get_state()
    print("128^4: two GPU steps done, running two oracle steps", flush=True)
    ref = orc.step(g, f0, tb, 2, w.dt)
    e = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"128^4 two steps, full grid: eps_inf {e:.3e}", flush=True)
    assert e <= 1e-12
