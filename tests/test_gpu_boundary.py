"""Boundary calls that hand the library caller-owned data: a torch-owned
device state stepped in place (wig2_bind_state)."""
import numpy as np
import pytest

from paper_2511_11354_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision,scheme", [("fp64", "strang"), ("fp64", "lawson"),
                                              ("fp32", "strang")])
def test_bind_state_steps_caller_tensor_in_place(orc, precision, scheme):
    from paper_2511_11354_amd import wig2

    nx, nk = 32, 32
    vext, v12 = I.cosine(0.5, 20.0), I.smoothed_coulomb(1.0, 1.0)
    ref = wig2.Solver(nx, nk, dt=0.01, precision=precision, scheme=scheme)
    ref.set_potentials(vext, v12)
    x, p, _ = ref.nodes()
    f0 = I.symmetrised_pair(x, p)
    ref.set_state(f0)
    ref.step(3)
    ob_ref = ref.observables()
    want = ref.get_state()

    s = wig2.Solver(nx, nk, dt=0.01, precision=precision, scheme=scheme)
    s.set_potentials(vext, v12)
    dt = torch.float64 if precision == "fp64" else torch.float32
    f = torch.from_numpy(f0).to("cuda", dt)
    addr = f.data_ptr()
    s.bind_state(f)
    s.step(3)
    torch.cuda.synchronize()
    assert f.data_ptr() == addr
    got = f.double().cpu().numpy()
    assert np.array_equal(got, want)                 # stepped in place, bitwise as set_state
    assert np.array_equal(s.get_state(), want)
    ob = s.observables()
    assert ob["step"] == 3 and ob["mass"] == ob_ref["mass"] and ob["energy"] == ob_ref["energy"]
    if precision == "fp64":
        g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
        o = orc.step(g, f0, orc.tables(g, vext, v12), 3, 0.01, scheme=scheme)
        assert np.max(np.abs(got - o)) / np.max(np.abs(o)) <= 1e-12
    # the caller writes a new state into its tensor: the next step starts there
    f.copy_(torch.from_numpy(f0).to("cuda", dt))
    s.bind_state(f)
    s.step(3)
    torch.cuda.synchronize()
    assert np.array_equal(f.double().cpu().numpy(), want)
    # unbinding returns to the context's own buffer, which needs a state again
    s.bind_state(None)
    with pytest.raises(wig2.Wig2Error):
        s.step(1)
    s.set_state(f0)
    s.step(3)
    assert np.array_equal(s.get_state(), want)


def test_bind_state_rejects_mismatch():
    from paper_2511_11354_amd import wig2

    s = wig2.Solver(16, 32, dt=0.01, precision="fp64")
    s.set_potentials(I.cosine(0.5, 20.0), None)
    L = wig2.lib()
    import ctypes
    f32 = torch.zeros((16, 16, 32, 32), dtype=torch.float32, device="cuda")
    assert L.wig2_bind_state(s._h, ctypes.c_void_p(f32.data_ptr()), wig2.FP32) == wig2.EINVAL
    host = np.zeros((16, 16, 32, 32))
    assert L.wig2_bind_state(s._h, ctypes.c_void_p(host.ctypes.data), wig2.FP64) == wig2.EINVAL
    f64 = torch.zeros((16 * 16 * 32 * 32 + 1,), dtype=torch.float64, device="cuda")
    assert L.wig2_bind_state(s._h, ctypes.c_void_p(f64.data_ptr() + 8), wig2.FP64) == wig2.EINVAL
