"""Pins of the numpy surrogate reference: its back-propagated gradient
against central finite differences of its loss (FP64), and the feature
layout against a direct per-point loop."""
import numpy as np

import surrogate_ref as S


def _setup(seed=0):
    rng = np.random.default_rng(seed)
    ft = rng.standard_normal((3, 3, 16, 16))
    p = 0.4 * rng.standard_normal(S.P)
    X = S.features(ft, 0.7, 1.3)
    t = rng.standard_normal(X.shape[0])
    return ft, p, X, t


def test_gradient_matches_finite_differences():
    _, p, X, t = _setup()
    g = S.grad(p, X, t)
    rng = np.random.default_rng(1)
    idx = rng.choice(S.P, 60, replace=False).tolist() + [S.P - 1, 0, S.H * S.D]
    for j in idx:
        e = np.zeros(S.P)
        e[j] = 1e-6
        fd = (S.loss(p + e, X, t) - S.loss(p - e, X, t)) / 2e-6
        assert abs(fd - g[j]) <= 1e-7 * max(1.0, abs(g[j])), (j, fd, g[j])


def test_features_direct_loop():
    ft, _, X, _ = _setup(3)
    nx, nk = 3, 16
    Xr = X.reshape(nx, nx, nk, nk, S.D)
    rng = np.random.default_rng(4)
    for _ in range(50):
        i1, i2, n1, n2 = (int(v) for v in rng.integers(0, [nx, nx, nk, nk]))
        ang = 2 * np.pi * ((i1 - i2) % nx) / nx

        def v(m):
            a, b = n1 - m, n2 + m
            return 0.7 * ft[i1, i2, a, b] if (0 <= a < nk and 0 <= b < nk) else 0.0

        assert Xr[i1, i2, n1, n2, 0] == v(0)
        for m in range(1, S.R + 1):
            assert np.isclose(Xr[i1, i2, n1, n2, m], np.sin(m * ang) * (v(m) - v(-m)), rtol=1e-15, atol=1e-15)
            assert np.isclose(Xr[i1, i2, n1, n2, S.R + m], np.cos(m * ang) * (v(m) + v(-m)),
                              rtol=1e-15, atol=1e-15)
        assert np.isclose(Xr[i1, i2, n1, n2, 2 * S.R + 1], np.sin(ang))
        assert np.isclose(Xr[i1, i2, n1, n2, 2 * S.R + 2], np.cos(ang))
        assert Xr[i1, i2, n1, n2, 2 * S.R + 3] == 1.3


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159], dtype=np.float32)
    r = S.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0 + 2 ** -7 or r[1] == 1.0  # tie to even: 1 + 2^-8 -> 1.0
    assert r[1] == 1.0
    assert r[2] == 1.0 + 2 ** -7
    assert abs(r[3] + 3.140625) < 1e-12
