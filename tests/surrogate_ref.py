"""Plain numpy reference of the learned pair-increment surrogate (test
infrastructure): features, the 4-D separable convolutional network, the
mean-squared-error loss and its gradient by explicit back-propagation, in
FP64.  With `rnd=True` the activations, weights and the back-propagated
pre-activation gradients are rounded to bfloat16 where the GPU stores them;
with `rnd=False` it is plain FP64 (pinned to central finite differences in
tests/test_surrogate_ref.py).  Independent of the HIP kernels.

Model on a state f_t[nx, nx, nk, nk] (grid point P = (i1, i2, n1, n2)),
a = 2 pi ((i1 - i2) mod nx) / nx, f_t = 0 off the p-box:
  c_0 = s_in f_t(n1, n2),
  c_m = s_in U sin(m a) [f_t(n1 - m, n2 + m) - f_t(n1 + m, n2 - m)], m = 1..15;
  h_0 = c;  per layer l (axis p1, p2, x1, x2 in turn, K taps, centre K // 2)
  z_l(P)[c] = b_l[c] + sum_{t, c'} W_l[c][t][c'] h_l(P + (t - K // 2) e_axis)[c']
  (zero off the p-box along p1 / p2, periodic along x1 / x2),
  t_l = tanh(z_l), h_{l+1} = h_l + t_l;
  y = b_o + w_o . h_L + a . c.
Parameter vector: per layer W_l[16][K][16] then b_l[16]; then w_o[16], b_o, a[16].
"""
from dataclasses import dataclass

import numpy as np

C = 16
# array axis of each convolution axis: p1 -> n1 (2), p2 -> n2 (3), x1 -> i1 (0), x2 -> i2 (1)
ARRAY_AXIS = {0: 2, 1: 3, 2: 0, 3: 1}
PERIODIC = {0: False, 1: False, 2: True, 3: True}


@dataclass
class Config:
    blocks: int = 9
    k_p: int = 35
    k_x: int = 7

    def layers(self):
        out = []
        for _ in range(self.blocks):
            for axis in range(4):
                out.append((axis, self.k_p if axis < 2 else self.k_x))
        return out

    @property
    def nparams(self):
        return sum(C * C * k + C for _, k in self.layers()) + 2 * C + 1


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p, cfg):
    p = np.asarray(p, dtype=np.float64)
    o, Ws = 0, []
    for axis, k in cfg.layers():
        W = p[o:o + C * C * k].reshape(C, k, C)
        o += C * C * k
        b = p[o:o + C]
        o += C
        Ws.append((axis, k, W, b))
    wo = p[o:o + C]
    bo = p[o + C]
    a = p[o + C + 1:o + 2 * C + 1]
    return Ws, wo, bo, a


def features(ft, s_in, u, rnd=True):
    nx, _, nk, _ = ft.shape
    F = np.pad(np.asarray(ft, dtype=np.float64), ((0, 0), (0, 0), (15, 15), (15, 15)))
    i = np.arange(nx)
    ang = 2 * np.pi * ((i[:, None] - i[None, :]) % nx) / nx
    out = np.zeros((nx, nx, nk, nk, C))
    out[..., 0] = s_in * ft
    for m in range(1, C):
        d = F[:, :, 15 - m:15 - m + nk, 15 + m:15 + m + nk] - F[:, :, 15 + m:15 + m + nk, 15 - m:15 - m + nk]
        out[..., m] = s_in * u * np.sin(m * ang)[:, :, None, None] * d
    return bf16(out) if rnd else out


def shift(h, o, axis):
    """g(P) = h(P + o e_axis): periodic in x, zero off the box in p."""
    ax = ARRAY_AXIS[axis]
    if o == 0:
        return h
    if PERIODIC[axis]:
        return np.roll(h, -o, axis=ax)
    g = np.zeros_like(h)
    n = h.shape[ax]
    src = [slice(None)] * h.ndim
    dst = [slice(None)] * h.ndim
    if o > 0:
        src[ax], dst[ax] = slice(o, n), slice(0, n - o)
    else:
        src[ax], dst[ax] = slice(0, n + o), slice(-o, n)
    g[tuple(dst)] = h[tuple(src)]
    return g


def conv(h, W, axis):
    """sum_{t, c'} W[c][t][c'] h(P + (t - K // 2) e_axis)[c']."""
    k = W.shape[1]
    out = np.zeros(h.shape[:-1] + (C,))
    for t in range(k):
        out += shift(h, t - k // 2, axis) @ W[:, t, :].T
    return out


def conv_t(z, W, axis):
    """The adjoint of conv: sum_{t, c} W[c][t][c'] z(P - (t - K // 2) e_axis)[c]."""
    k = W.shape[1]
    out = np.zeros(z.shape[:-1] + (C,))
    for t in range(k):
        out += shift(z, -(t - k // 2), axis) @ W[:, t, :]
    return out


def forward(p, cfg, feat, rnd=True):
    Ws, wo, bo, a = unpack(p, cfg)
    h = feat
    hs, ts = [h], []
    for axis, k, W, b in Ws:
        Wq = bf16(W) if rnd else W
        t = np.tanh(conv(h, Wq, axis) + b)
        h = bf16(h + t) if rnd else h + t
        ts.append(bf16(t) if rnd else t)
        hs.append(h)
    y = bo + h @ wo + feat @ a
    return y, (hs, ts)


def loss(p, cfg, feat, target, rnd=True):
    y, _ = forward(p, cfg, feat, rnd)
    return float(np.mean((y - target) ** 2))


def grad(p, cfg, feat, target, rnd=True):
    """Gradient of mean((y - target)^2) by explicit back-propagation."""
    Ws, wo, bo, a = unpack(p, cfg)
    y, (hs, ts) = forward(p, cfg, feat, rnd)
    n = y.size
    dy = 2.0 * (y - target) / n
    g_layers = []
    dh = dy[..., None] * wo
    for li in range(len(Ws) - 1, -1, -1):
        axis, k, W, _ = Ws[li]
        dz = dh * (1.0 - ts[li] ** 2)
        if rnd:
            dz = bf16(dz)
        hl = hs[li]
        gW = np.zeros((C, k, C))
        for t in range(k):
            gW[:, t, :] = dz.reshape(-1, C).T @ shift(hl, t - k // 2, axis).reshape(-1, C)
        gb = dz.reshape(-1, C).sum(axis=0)
        g_layers.append(np.concatenate([gW.ravel(), gb]))
        if li > 0:
            dh = dh + conv_t(dz, bf16(W) if rnd else W, axis)
    g_layers.reverse()
    g_head = np.concatenate([(dy[..., None] * hs[-1]).reshape(-1, C).sum(axis=0), [dy.sum()],
                             (dy[..., None] * feat).reshape(-1, C).sum(axis=0)])
    return np.concatenate(g_layers + [g_head])
