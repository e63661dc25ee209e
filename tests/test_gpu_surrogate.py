"""Learned pair-increment surrogate on the GPU: gradients and inference
against the numpy reference (tests/surrogate_ref.py), the fallback and
exact-check semantics against the exact path, training on collected blocks,
and the error paths."""
import numpy as np
import pytest

import surrogate_ref as S
from paper_2511_11354_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def W():
    from paper_2511_11354_amd import wig2

    return wig2


def solver(nx, nk, precision="fp64", v12=True, dt=0.005, seed=3):
    s = W().Solver(nx, nk, dt=dt, precision=precision)
    s.set_potentials(I.cosine(0.5, 20.0), I.smoothed_coulomb(1.5, 1.0) if v12 else None)
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=seed, period=20.0)
    s.set_state(f0)
    return s, f0


def random_model(seed=0, scales=(2.0, 1e-3, 1.5)):
    m = W().Surrogate(block=4, epochs=1, batch=4096, lr=1e-3, seed=seed)
    rng = np.random.default_rng(seed)
    p = (0.3 * rng.standard_normal(S.P)).astype(np.float32)
    m.set_params(p, np.array(scales, dtype=np.float32))
    return m, p


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gradient_matches_reference(precision):
    nx, nk = 4, 32
    s, _ = solver(nx, nk, precision)
    m, p = random_model(1)
    rng = np.random.default_rng(2)
    ft = rng.standard_normal((nx, nx, nk, nk))
    delta = 1e-3 * rng.standard_normal((nx, nx, nk, nk))
    dt = torch.float64 if precision == "fp64" else torch.float32
    g, loss = m.grad(s, torch.from_numpy(ft).to(dtype=dt, device="cuda"),
                     torch.from_numpy(delta).to(dtype=dt, device="cuda"))
    ftr = ft if precision == "fp64" else ft.astype(np.float32).astype(np.float64)
    dr = delta if precision == "fp64" else delta.astype(np.float32).astype(np.float64)
    X = S.features(ftr, 2.0, 1.5)
    t = dr.ravel() / 1e-3
    gr = S.grad(p.astype(np.float64), X, t)
    lr = S.loss(p.astype(np.float64), X, t)
    e = np.abs(g - gr).max() / np.abs(gr).max()
    print(f"surrogate grad {precision}: rel err {e:.2e}, loss {loss:.6f} vs {lr:.6f}", flush=True)
    assert e <= 1e-4 and abs(loss - lr) <= 1e-4 * lr


def test_inference_block_matches_reference():
    """With the drift check switched off, a block is B steps without the pair
    term plus out_scale * NN(f_t) (BF16 weights): compare with a context
    that has no pair potential (same kernels) plus the numpy model."""
    nx, nk, B = 8, 32, 4
    s, f0 = solver(nx, nk)
    ref, _ = solver(nx, nk, v12=False)
    m, p = random_model(5, scales=(3.0, 2e-4, 1.5))
    s.attach_surrogate(m, drift_tol=1e30, exact_check_every=0)
    s.step(B)
    got = s.get_state()
    rep = s.surrogate_report()
    ref.step(B)
    fnov = ref.get_state()
    X = S.features(f0, 3.0, 1.5)
    y, _ = S.forward(S.bf16_round(p), X)
    want = fnov + 2e-4 * y.reshape(f0.shape)
    e = np.abs(got - want).max() / np.abs(2e-4 * y).max()
    print(f"surrogate block vs reference: rel err of the increment {e:.2e}, report {rep}", flush=True)
    assert rep["blocks"] == 1 and rep["fallbacks"] == 0
    assert e <= 5e-5


def test_zero_tolerance_falls_back_to_exact_bitwise():
    nx, nk, B = 8, 32, 4
    s, _ = solver(nx, nk)
    ex, _ = solver(nx, nk)
    m, _ = random_model(7)
    s.attach_surrogate(m, drift_tol=0.0, exact_check_every=0)
    s.step(3 * B + 1)
    ex.step(3 * B + 1)
    rep = s.surrogate_report()
    assert rep["blocks"] == 3 and rep["fallbacks"] == 3
    assert np.array_equal(s.get_state(), ex.get_state())
    assert s.observables()["fallbacks"] == 3


def test_exact_checks_keep_the_exact_result():
    nx, nk, B = 8, 32, 4
    s, _ = solver(nx, nk)
    m, _ = random_model(9, scales=(3.0, 1e-12, 1.5))  # negligible increment
    s.attach_surrogate(m, drift_tol=1e30, exact_check_every=2)
    s.step(2 * B)
    rep = s.surrogate_report()
    assert rep["blocks"] == 2 and rep["checks"] == 1 and rep["fallbacks"] == 0
    assert rep["last_check_eps"] > 0.0  # the no-pair block differs from the exact one
    # block 1 took the surrogate, block 2 was recomputed exactly from its start
    s2, _ = solver(nx, nk)
    s2.attach_surrogate(m, drift_tol=1e30, exact_check_every=0)
    s2.step(B)
    s2.detach_surrogate()
    s2.step(B)
    assert np.array_equal(s.get_state(), s2.get_state())


def test_training_lowers_the_loss():
    """Collect blocks of a 32^4 FP32 trajectory: training on them lowers the
    loss on a held-out trajectory (other initial state, same grid)."""
    m = W().Surrogate(block=8, epochs=4, batch=16384, lr=3e-3, seed=11)
    held, _ = solver(32, 32, "fp32", seed=21)
    m.collect(held, blocks=1, train=False)
    before = m.stats()["eval_loss"]
    tr, _ = solver(32, 32, "fp32", seed=20)
    m.collect(tr, blocks=3, train=True)
    held2, _ = solver(32, 32, "fp32", seed=21)
    m.collect(held2, blocks=1, train=False)
    st = m.stats()
    print(f"surrogate held-out loss: untrained {before:.4e} -> trained {st['eval_loss']:.4e}; "
          f"last train loss {st['train_loss']:.4e}, {st['updates']} Adam steps", flush=True)
    assert st["updates"] == 3 * 4 * ((32 ** 4 + 16383) // 16384)
    assert st["eval_loss"] < 0.5 * before


def test_trained_surrogate_beats_the_method_without_it():
    """What the trained network gains over the method without it: on a
    held-out 32^4 FP32 state, one block of B steps with the surrogate's pair
    increment (no fallback, no exact check) is closer to the exact block
    than the same block without the pair term, which is what the surrogate
    replaces."""
    B = 8
    m = W().Surrogate(block=B, epochs=4, batch=16384, lr=3e-3, seed=11)
    for seed in (20, 22):
        tr, _ = solver(32, 32, "fp32", seed=seed)
        m.collect(tr, blocks=2, train=True)
    exact, f0 = solver(32, 32, "fp32", seed=21)
    exact.step(B)
    fe = exact.get_state()
    sur, _ = solver(32, 32, "fp32", seed=21)
    sur.attach_surrogate(m, drift_tol=1e30, exact_check_every=0)
    sur.step(B)
    fs = sur.get_state()
    assert sur.surrogate_report()["fallbacks"] == 0
    nov, _ = solver(32, 32, "fp32", v12=False, seed=21)
    nov.step(B)
    fn = nov.get_state()
    scale = np.abs(fe).max()
    e_sur, e_nov = np.abs(fs - fe).max() / scale, np.abs(fn - fe).max() / scale
    r_sur = np.sqrt(np.mean((fs - fe) ** 2)) / scale
    r_nov = np.sqrt(np.mean((fn - fe) ** 2)) / scale
    print(f"one block of {B} steps vs exact: without the pair term eps_inf {e_nov:.3e} (rms {r_nov:.3e}), "
          f"with the trained surrogate {e_sur:.3e} (rms {r_sur:.3e}): gain {e_nov / e_sur:.1f}x "
          f"(rms {r_nov / r_sur:.1f}x)", flush=True)
    assert e_sur < 0.5 * e_nov and r_sur < 0.5 * r_nov


def test_surrogate_rejections():
    wig2 = W()
    m = wig2.Surrogate(block=4, epochs=1, batch=4096, lr=1e-3, seed=0)
    s, _ = solver(8, 32)
    with pytest.raises(wig2.Wig2Error):
        s.attach_surrogate(m)  # no scales yet
    nopair, _ = solver(8, 32, v12=False)
    with pytest.raises(wig2.Wig2Error):
        m.collect(nopair, blocks=1)
    m.collect(s, blocks=1, train=False)  # fixes dt = 0.005 and the scales
    other, _ = solver(8, 32, dt=0.01)
    with pytest.raises(wig2.Wig2Error):
        m.collect(other, blocks=1)
    bx = wig2.Solver(9, 32, periodic=False, sem_cells=4, x_min=-15.0, x_max=15.0, k_max=3.0, dt=0.005)
    bx.set_potentials(I.harmonic(0.5), None)
    with pytest.raises(wig2.Wig2Error):
        bx.attach_surrogate(m)
