"""wig2_advect_noalloc: the sweep of wig2_advect without device allocation
(static per-device scratch for the general sweep's coefficients), for
callers that cannot allocate.  Checked through the C ABI against
wig2_advect on two calls in a row, the second on a smaller state, in the
general sweep (which uses the scratch) and in a register-resident sweep."""
import numpy as np
import pytest

from paper_2511_11354_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# (nx, nk, periodic, s): nx = 24 has no register sweep; s = 3.0 moves more
# than one cell (general sweep); the last pair is register-resident
CALLS = [
    [(24, 48, True, 0.01), (16, 32, True, 3.0)],
    [(33, 32, False, 2.5), (20, 16, False, 0.05)],
    [(32, 32, True, 0.02), (16, 16, True, 0.01)],
]


def _solver(nx, nk, periodic, precision):
    from paper_2511_11354_amd import wig2

    kw = dict(periodic=periodic, precision=precision)
    if not periodic:
        kw.update(sem_cells=2, x_min=-15.0, x_max=15.0, k_max=3.0)
    s = wig2.Solver(nx, nk, **kw)
    s.set_potentials(None, None)
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("calls", CALLS)
def test_advect_noalloc_equals_advect(calls, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    for k, (nx, nk, per, s) in enumerate(calls):
        sol = _solver(nx, nk, per, precision)
        f = torch.from_numpy(I.random_field((nx, nx, nk, nk), seed=70 + 3 * k + nx)).to("cuda", dt)
        for dim in (1, 2):
            a = torch.full_like(f, float("nan"))
            b = torch.full_like(f, float("nan"))
            sol.advect_noalloc(dim, s, f, a)
            sol.advect(dim, s, f, b)
            torch.cuda.synchronize()
            print(f"{precision} nx={nx} nk={nk} per={per} s={s} dim={dim}: "
                  f"max|noalloc - advect| {float((a - b).abs().max()):.3e}", flush=True)
            assert torch.equal(a, b)
        sol.close()


def test_advect_noalloc_rejects_large_general_sweep():
    from paper_2511_11354_amd import wig2

    # 48^2 x 64^2 FP64 is 75 MB: more than the 64 MiB scratch for the general
    # sweep (s = 3 moves lines by more than one cell); the register sweep is fine
    sol = _solver(48, 64, True, "fp64")
    f = torch.zeros((48, 48, 64, 64), dtype=torch.float64, device="cuda")
    out = torch.empty_like(f)
    with pytest.raises(wig2.Wig2Error) as ei:
        sol.advect_noalloc(1, 3.0, f, out)
    assert ei.value.code == wig2.EINVAL and "64 MiB" in str(ei.value)
    sol.advect_noalloc(1, 0.001, f, out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out) == 0
