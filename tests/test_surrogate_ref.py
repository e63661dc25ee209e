"""Pins of the numpy surrogate reference (plain FP64, no bfloat16 rounding):
its back-propagated gradient against central finite differences of its
loss, the adjoint identity of its convolution and transpose along every
axis, the direction of its shifts, and the feature layout against a direct
per-point loop."""
import numpy as np
import pytest

import surrogate_ref as S

CFG = S.Config(blocks=1, k_p=3, k_x=3)


def _setup(seed=0, nx=4, nk=16):
    rng = np.random.default_rng(seed)
    ft = rng.standard_normal((nx, nx, nk, nk))
    p = 0.4 * rng.standard_normal(CFG.nparams)
    feat = S.features(ft, 0.7, 1.3, rnd=False)
    target = rng.standard_normal((nx, nx, nk, nk))
    return ft, p, feat, target


def test_gradient_matches_finite_differences():
    _, p, feat, target = _setup()
    g = S.grad(p, CFG, feat, target, rnd=False)
    assert g.shape == (CFG.nparams,)
    rng = np.random.default_rng(1)
    idx = sorted(set(rng.integers(0, CFG.nparams, 40).tolist()) | set(range(CFG.nparams - 33, CFG.nparams)))
    h = 1e-6
    for j in idx:
        e = np.zeros_like(p)
        e[j] = h
        fd = (S.loss(p + e, CFG, feat, target, rnd=False) - S.loss(p - e, CFG, feat, target, rnd=False)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), (j, fd, g[j])


@pytest.mark.parametrize("axis", [0, 1, 2, 3])
def test_conv_transpose_is_adjoint(axis):
    rng = np.random.default_rng(2 + axis)
    h = rng.standard_normal((4, 4, 16, 16, S.C))
    z = rng.standard_normal((4, 4, 16, 16, S.C))
    W = rng.standard_normal((S.C, 5, S.C))
    lhs = np.sum(S.conv(h, W, axis) * z)
    rhs = np.sum(h * S.conv_t(z, W, axis))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


@pytest.mark.parametrize("axis", [0, 1, 2, 3])
def test_conv_tap_direction(axis):
    """Tap t reads the point (t - K // 2) steps ahead along the axis: an
    impulse at position 5 appears at 5 - (t - K // 2) in the output."""
    h = np.zeros((8, 8, 16, 16, S.C))
    h[5, 5, 5, 5, 3] = 1.0
    W = np.zeros((S.C, 3, S.C))
    W[7, 2, 3] = 1.0  # tap 2: offset +1, channel 3 -> 7
    out = S.conv(h, W, axis)
    pos = [5, 5, 5, 5]
    pos[S.ARRAY_AXIS[axis]] = 4
    assert out[tuple(pos) + (7,)] == 1.0 and np.count_nonzero(out) == 1


def test_features_against_point_loop():
    rng = np.random.default_rng(4)
    nx, nk = 3, 16
    ft = rng.standard_normal((nx, nx, nk, nk))
    feat = S.features(ft, 0.5, 2.0, rnd=False)

    def at(i1, i2, a, b):
        return ft[i1, i2, a, b] if 0 <= a < nk and 0 <= b < nk else 0.0

    for (i1, i2, n1, n2) in [(0, 0, 0, 0), (1, 2, 3, 15), (2, 0, 8, 8), (0, 1, 15, 0)]:
        ang = 2 * np.pi * ((i1 - i2) % nx) / nx
        assert feat[i1, i2, n1, n2, 0] == 0.5 * ft[i1, i2, n1, n2]
        for m in range(1, 16):
            want = 0.5 * 2.0 * np.sin(m * ang) * (at(i1, i2, n1 - m, n2 + m) - at(i1, i2, n1 + m, n2 - m))
            assert abs(feat[i1, i2, n1, n2, m] - want) <= 1e-14


def test_full_config_size():
    assert S.Config().nparams == 194145
