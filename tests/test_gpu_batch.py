"""Batched ensembles (one launch per phase, HIP-graph replay, autotuned
tiling) against the single-context path and the FP64 oracle."""
import numpy as np
import pytest

from paper_2511_11354_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SPECS = [(32, 48), (16, 32), (48, 16), (32, 32), (16, 64), (48, 48)]


def _inst(i, nx, nk):
    u = 0.5 + 0.4 * i
    return dict(nx=nx, nk=nk, dt=0.005), I.cosine(0.5, 20.0), I.smoothed_coulomb(u, 1.0), 100 + i


def _build(precision):
    from paper_2511_11354_amd import wig2

    specs, pots, states = [], [], []
    for i, (nx, nk) in enumerate(SPECS):
        sp, ve, v12, seed = _inst(i, nx, nk)
        specs.append(sp)
        pots.append((ve, v12))
    b = wig2.Batch(specs, precision=precision)
    for i, (nx, nk) in enumerate(SPECS):
        b.set_potentials(i, *pots[i])
        s = wig2.Solver(nx, nk, dt=0.005, precision=precision)
        x, p, _ = s.nodes()
        f0 = I.mixture(x, p, seed=100 + i, period=20.0)
        states.append(f0)
        b.set_state(i, f0)
        s.close()
    return b, pots, states


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_single_instances(precision):
    """Every instance of the batch is bitwise the same instance stepped alone
    (same per-plane and per-line arithmetic, different work distribution):
    the streaming one-pass Heun kernel takes every size here but nk = 16,
    which takes the general kernel, in both."""
    from paper_2511_11354_amd import wig2

    b, pots, states = _build(precision)
    b.step(1)   # direct pass + graph capture
    b.step(3)   # graph replays
    for i, (nx, nk) in enumerate(SPECS):
        s = wig2.Solver(nx, nk, dt=0.005, precision=precision)
        s.set_potentials(*pots[i])
        s.set_state(states[i])
        s.step(4)
        a, c = b.get_state(i), s.get_state()
        assert np.array_equal(a, c), (i, np.abs(a - c).max())
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_reset_after_steps(precision):
    """Setting one instance's state (and potentials) right after steps were
    queued is ordered after them: the instance then evolves bitwise as in a
    fresh batch, and its neighbours are untouched by the reset."""
    b, pots, states = _build(precision)
    b.step(1)
    b.step(3)            # graph replays still in flight when the setters run
    b.set_state(2, states[2])
    b.set_potentials(2, *pots[2])
    b.step(2)
    fresh, _, _ = _build(precision)
    fresh.step(2)
    a2, f2 = b.get_state(2), fresh.get_state(2)
    assert np.array_equal(a2, f2), np.abs(a2 - f2).max()
    ref0 = _build(precision)[0]
    ref0.step(6)
    assert np.array_equal(b.get_state(0), ref0.get_state(0))


def test_batch_fp64_matches_oracle(orc):
    b, pots, states = _build("fp64")
    b.step(3)
    worst = 0.0
    for i, (nx, nk) in enumerate(SPECS):
        g = orc.grid(nx, nk, True, 1, -10.0, 10.0)
        ref = orc.step(g, states[i], orc.tables(g, *pots[i]), 3, 0.005)
        e = np.abs(b.get_state(i) - ref).max() / np.abs(ref).max()
        worst = max(worst, e)
        ob = b.observables(i)
        ro = orc.observables(g, ref, orc.tables(g, *pots[i])["vext_x"], orc.tables(g, *pots[i])["v12_pair"])
        assert abs(ob["mass"] - ro["mass"]) <= 1e-12 and abs(ob["energy"] - ro["energy"]) <= 1e-12
    print(f"batch fp64 vs oracle, 3 steps: worst eps_inf {worst:.3e}")
    assert worst <= 1e-12


def test_batch_tune_keeps_results(tmp_path):
    """Tuning changes only the work distribution: results stay bitwise equal,
    the cache is written and re-read."""
    b1, _, _ = _build("fp32")
    b1.step(2)
    ref = [b1.get_state(i) for i in range(len(SPECS))]
    b2, _, _ = _build("fp32")
    cache = tmp_path / "tune.json"
    b2.tune(str(cache))
    info = b2.info()
    print("tuned:", info)
    assert cache.exists() and "planes" in cache.read_text()
    b2.step(2)
    for i in range(len(SPECS)):
        assert np.array_equal(b2.get_state(i), ref[i])
    b3, _, _ = _build("fp32")
    b3.tune(str(cache))  # from the cache
    assert b3.info() == info


def test_batch_rejects_unsupported():
    from paper_2511_11354_amd import wig2

    with pytest.raises(wig2.Wig2Error):
        wig2.Batch([dict(nx=24, nk=32)], precision="fp32")  # nx outside the register set
    with pytest.raises(wig2.Wig2Error):
        wig2.Batch([dict(nx=32, nk=40)], precision="fp32")
    b = wig2.Batch([dict(nx=32, nk=32)], precision="fp32")
    with pytest.raises(wig2.Wig2Error):
        b.step(1)  # no potentials / state yet
