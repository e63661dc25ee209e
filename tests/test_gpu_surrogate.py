"""Learned pair-increment surrogate on the GPU (4-D separable convolutional
network, BF16 on the matrix cores): gradients and inference against the
numpy reference (tests/surrogate_ref.py), the fallback and exact-check
semantics against the exact path, training on collected blocks and on a
batched ensemble, what the trained network gains over the method without
it, and the error paths."""
import numpy as np
import pytest

import surrogate_ref as S
from paper_2511_11354_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SMALL = S.Config(blocks=1, k_p=5, k_x=3)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def W():
    from paper_2511_11354_amd import wig2

    return wig2


def solver(nx, nk, precision="fp64", v12=True, dt=0.005, seed=3, u=1.5):
    s = W().Solver(nx, nk, dt=dt, precision=precision)
    s.set_potentials(I.cosine(0.5, 20.0), I.smoothed_coulomb(u, 1.0) if v12 else None)
    x, p, _ = s.nodes()
    f0 = I.mixture(x, p, seed=seed, period=20.0)
    s.set_state(f0)
    return s, f0


def random_model(cfg, seed=0, scales=(2.0, 1e-3, 1.5), wscale=0.3, block=4):
    m = W().Surrogate(blocks=cfg.blocks, k_p=cfg.k_p, k_x=cfg.k_x, block=block, epochs=1, lr=1e-3, seed=seed)
    assert m.nparams == cfg.nparams
    rng = np.random.default_rng(seed)
    p = (wscale * rng.standard_normal(cfg.nparams) / np.sqrt(S.C * 3)).astype(np.float32)
    p[-33:] = (0.3 * rng.standard_normal(33)).astype(np.float32)  # head: w_o, b_o, a
    m.set_params(p, np.array(scales, dtype=np.float32))
    return m, p


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gradient_matches_reference(precision):
    """Full-grid gradient (forward, output head, weight and input gradients
    of every layer on the bf16 matrix cores) against the numpy reference
    with the same bf16 rounding points, 8^2 x 32^2."""
    nx, nk = 8, 32
    s, _ = solver(nx, nk, precision)
    m, p = random_model(SMALL, 1, wscale=3.0)
    rng = np.random.default_rng(2)
    ft = rng.standard_normal((nx, nx, nk, nk))
    delta = 1e-3 * rng.standard_normal((nx, nx, nk, nk))
    dt = torch.float64 if precision == "fp64" else torch.float32
    g, loss = m.grad(s, torch.from_numpy(ft).to(dtype=dt, device="cuda"),
                     torch.from_numpy(delta).to(dtype=dt, device="cuda"))
    ftr = ft if precision == "fp64" else ft.astype(np.float32).astype(np.float64)
    dr = delta if precision == "fp64" else delta.astype(np.float32).astype(np.float64)
    feat = S.features(ftr, 2.0, 1.5)
    t = dr / 1e-3
    gr = S.grad(p.astype(np.float64), SMALL, feat, t)
    lr = S.loss(p.astype(np.float64), SMALL, feat, t)
    e = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    o, worst = 0, 0.0
    for _, k in SMALL.layers():
        n = S.C * S.C * k + S.C
        worst = max(worst, np.linalg.norm(g[o:o + n] - gr[o:o + n]) / np.linalg.norm(gr[o:o + n]))
        o += n
    eh = np.linalg.norm(g[o:] - gr[o:]) / np.linalg.norm(gr[o:])
    print(f"surrogate grad {precision}: rel err {e:.2e} (worst layer {worst:.2e}, head {eh:.2e}), "
          f"loss {loss:.6f} vs {lr:.6f}", flush=True)
    assert e <= 1e-2 and worst <= 2e-2 and eh <= 1e-2
    assert abs(loss - lr) <= 1e-3 * lr


def test_inference_block_matches_reference():
    """The full 194,145-parameter network: with the drift check off, a block
    is B steps without the pair term plus out_scale * y(f_t); compare with a
    context without the pair potential (same kernels) plus the numpy model."""
    cfg = S.Config()
    nx, nk, B = 8, 32, 4
    s, f0 = solver(nx, nk)
    ref, _ = solver(nx, nk, v12=False)
    m, p = random_model(cfg, 5, scales=(3.0, 2e-4, 1.5))
    s.attach_surrogate(m, drift_tol=1e30, exact_check_every=0)
    s.step(B)
    got = s.get_state()
    rep = s.surrogate_report()
    ref.step(B)
    fnov = ref.get_state()
    y, _ = S.forward(p.astype(np.float64), cfg, S.features(f0, 3.0, 1.5))
    y64, _ = S.forward(p.astype(np.float64), cfg, S.features(f0, 3.0, 1.5, rnd=False), rnd=False)
    inc = 2e-4 * y
    scale = np.abs(inc).max()
    e = np.abs((got - fnov) - inc).max() / scale
    d = np.abs(2e-4 * y64 - inc).max() / scale  # what bf16 storage itself moves the increment
    print(f"surrogate block vs reference: rel err of the increment {e:.2e} (bf16 storage vs FP64: {d:.2e}), "
          f"report {rep}", flush=True)
    assert rep["blocks"] == 1 and rep["fallbacks"] == 0
    # 36 layers of bf16 activations: rounding-boundary differences between the
    # FP32 (GPU) and FP64 (reference) pre-rounding values accumulate; a wrong
    # axis, tap or channel would be an O(1) error
    assert e <= 5e-2 and e <= 2.0 * d


def test_zero_tolerance_falls_back_to_exact_bitwise():
    nx, nk, B = 8, 32, 4
    s, _ = solver(nx, nk)
    ex, _ = solver(nx, nk)
    m, _ = random_model(SMALL, 7)
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
    m, _ = random_model(SMALL, 9, scales=(3.0, 1e-12, 1.5))  # negligible increment
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


def _train(m, seeds, blocks=2):
    for seed in seeds:
        tr, _ = solver(32, 32, "fp32", seed=seed)
        m.collect(tr, blocks=blocks, train=True)


def test_training_lowers_the_loss():
    """Collect blocks of a 32^4 FP32 trajectory: full-grid Adam steps on them
    lower the loss on a held-out trajectory (other initial state)."""
    m = W().Surrogate(block=8, epochs=24, lr=2e-3, seed=11)
    held, _ = solver(32, 32, "fp32", seed=21)
    m.collect(held, blocks=1, train=False)
    before = m.stats()["eval_loss"]
    _train(m, (20,), blocks=3)
    held2, _ = solver(32, 32, "fp32", seed=21)
    m.collect(held2, blocks=1, train=False)
    st = m.stats()
    print(f"surrogate held-out loss: untrained {before:.4e} -> trained {st['eval_loss']:.4e}; "
          f"last train loss {st['train_loss']:.4e}, {st['updates']} Adam steps", flush=True)
    assert st["updates"] == 3 * 24
    assert st["eval_loss"] < 0.3 * before


def _gain(m, B=8, seed=21):
    exact, f0 = solver(32, 32, "fp32", seed=seed)
    exact.step(B)
    fe = exact.get_state()
    sur, _ = solver(32, 32, "fp32", seed=seed)
    sur.attach_surrogate(m, drift_tol=1e30, exact_check_every=0)
    sur.step(B)
    fs = sur.get_state()
    assert sur.surrogate_report()["fallbacks"] == 0
    nov, _ = solver(32, 32, "fp32", v12=False, seed=seed)
    nov.step(B)
    fn = nov.get_state()
    scale = np.abs(fe).max()
    return (np.abs(fs - fe).max() / scale, np.abs(fn - fe).max() / scale,
            np.sqrt(np.mean((fs - fe) ** 2)) / scale, np.sqrt(np.mean((fn - fe) ** 2)) / scale)


def test_trained_surrogate_beats_the_method_without_it():
    """What the trained network gains over the method without it: on a
    held-out 32^4 FP32 state, one block of B steps with the surrogate's pair
    increment (no fallback, no exact check) is closer to the exact block
    than the same block without the pair term, which is what it replaces."""
    m = W().Surrogate(block=8, epochs=24, lr=2e-3, seed=11)
    _train(m, (20, 22))
    e_sur, e_nov, r_sur, r_nov = _gain(m)
    print(f"one block of 8 steps vs exact: without the pair term eps_inf {e_nov:.3e} (rms {r_nov:.3e}), "
          f"with the trained surrogate {e_sur:.3e} (rms {r_sur:.3e}): gain {e_nov / e_sur:.1f}x "
          f"(rms {r_nov / r_sur:.1f}x)", flush=True)
    assert e_sur < 0.5 * e_nov and r_sur < 0.5 * r_nov


def test_train_on_batched_ensemble():
    """wig2_surrogate_train: a model trained on the instances of a batch
    (uneven grids, their own pair strengths) through the C ABI; the batch's
    states are left as they were, and the model beats the method without
    the pair term on a held-out state."""
    wig2 = W()
    specs, pots, states = [], [], []
    for i, (nx, nk, u) in enumerate([(32, 32, 1.2), (32, 48, 2.0), (48, 32, 0.8)]):
        specs.append(dict(nx=nx, nk=nk, dt=0.005))
        pots.append((I.cosine(0.5, 20.0), I.smoothed_coulomb(u, 1.0)))
    b = wig2.Batch(specs, precision="fp32")
    for i, sp in enumerate(specs):
        b.set_potentials(i, *pots[i])
        s = wig2.Solver(sp["nx"], sp["nk"], dt=0.005, precision="fp32")
        x, p, _ = s.nodes()
        f0 = I.mixture(x, p, seed=40 + i, period=20.0)
        states.append(f0.astype(np.float32).astype(np.float64))
        b.set_state(i, f0)
        s.close()
    m = wig2.Surrogate.train_on_batch(b, block=8, epochs=16, lr=2e-3, seed=3, train_blocks=3,
                                      max_points=48 * 48 * 32 * 32)
    st = m.stats()
    for i in range(len(specs)):
        assert np.array_equal(b.get_state(i), states[i])
    e_sur, e_nov, r_sur, r_nov = _gain(m)
    print(f"batch-trained surrogate: {st['updates']} Adam steps, last train loss {st['train_loss']:.3e}; "
          f"held-out block eps_inf {e_sur:.3e} vs {e_nov:.3e} without the pair term "
          f"(rms {r_sur:.3e} vs {r_nov:.3e})", flush=True)
    assert st["updates"] == 3 * 3 * 16
    assert e_sur < 0.85 * e_nov and r_sur < 0.85 * r_nov


def test_surrogate_rejections():
    wig2 = W()
    with pytest.raises(wig2.Wig2Error):
        wig2.Surrogate(k_p=4)  # even tap count
    m = wig2.Surrogate(blocks=1, k_p=5, k_x=3, block=4, epochs=1, lr=1e-3, seed=0)
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
