"""Plain FP64 numpy reference of the learned pair-increment surrogate
(test infrastructure): features, forward pass, mean-squared-error loss and
its gradient by explicit back-propagation.  Independent of the HIP kernels;
pinned to central finite differences in tests/test_surrogate_ref.py.

Model per grid point (i1, i2, n1, n2) of a state f_t[nx, nx, nk, nk], with
v_m = s_in f_t(i1, i2, n1 - m, n2 + m) (0 off the p-box), l = (i1 - i2) mod nx,
a = 2 pi l / nx:
  x = [v_0;  sin(m a) (v_m - v_-m), m = 1..R;  cos(m a) (v_m + v_-m), m = 1..R;
       sin(a), cos(a), U]
  y = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3 + a . x,   Delta ~ s_out y.
Parameters are packed as W1[H][D], b1[H], W2[H][H], b2[H], w3[H], b3, a[D].
"""
import numpy as np

R, H = 8, 16
D = 2 * R + 1 + 3
P = H * D + H + H * H + H + H + 1 + D


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * D].reshape(H, D); o += H * D
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]; o += 1
    a = p[o:o + D]
    return W1, b1, W2, b2, w3, b3, a


def shifted(ft, m):
    """v(n1, n2) = f_t(n1 - m, n2 + m), zero where that leaves the p-box."""
    nk = ft.shape[2]
    sh = np.zeros_like(ft)
    a0, a1 = max(0, m), min(nk, nk + m)          # n1 range with n1 - m in [0, nk)
    b0, b1 = max(0, -m), min(nk, nk - m)         # n2 range with n2 + m in [0, nk)
    if a0 < a1 and b0 < b1:
        sh[:, :, a0:a1, b0:b1] = ft[:, :, a0 - m:a1 - m, b0 + m:b1 + m]
    return sh


def features(ft, in_scale, u):
    """X[npts, D] in the state's point order (i1, i2, n1, n2)."""
    nx, _, nk, _ = ft.shape
    X = np.zeros((nx, nx, nk, nk, D))
    i1 = np.arange(nx)[:, None]
    i2 = np.arange(nx)[None, :]
    ang = 2.0 * np.pi * ((i1 - i2) % nx) / nx
    X[..., 0] = in_scale * ft
    for m in range(1, R + 1):
        vp, vm = in_scale * shifted(ft, m), in_scale * shifted(ft, -m)
        X[..., m] = np.sin(m * ang)[:, :, None, None] * (vp - vm)
        X[..., R + m] = np.cos(m * ang)[:, :, None, None] * (vp + vm)
    X[..., 2 * R + 1] = np.sin(ang)[:, :, None, None]
    X[..., 2 * R + 2] = np.cos(ang)[:, :, None, None]
    X[..., 2 * R + 3] = u
    return X.reshape(-1, D)


def forward(p, X):
    W1, b1, W2, b2, w3, b3, a = unpack(p)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ w3 + b3 + X @ a, (h1, h2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - t) ** 2))


def grad(p, X, t):
    """d loss / d p for loss = mean (y - t)^2."""
    W1, b1, W2, b2, w3, b3, a = unpack(p)
    y, (h1, h2) = forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - t) / n
    dz2 = (dy[:, None] * w3[None, :]) * (1.0 - h2 ** 2)
    dz1 = (dz2 @ W2) * (1.0 - h1 ** 2)
    g = np.concatenate([(dz1.T @ X).ravel(), dz1.sum(0), (dz2.T @ h1).ravel(), dz2.sum(0),
                        h2.T @ dy, [dy.sum()], X.T @ dy])
    return g


def bf16_round(p):
    """Round FP32 values to bfloat16 (nearest, ties to even), back as float64."""
    a = np.asarray(p, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((a + 0x7FFF + ((a >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
