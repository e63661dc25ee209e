"""Independent reference for the whole step: two particles on a ring, evolved
exactly (dense eigendecomposition of H in a truncated Fourier basis), then
Wigner-transformed onto the (x_i, p_n) lattice.

For a band-limited psi(x1,x2) = sum_k c_k e^{2 pi i k.x/L} the periodic Weyl-
Wigner transform (Sec. 2.2, with the y-integral over one period 2L and
p_n = n hbar pi / L) is exact and finite:
    f(x, p_n) = (2L/(2 pi hbar))^2 sum_{k + k' = n} c_k conj(c_k') e^{2 pi i (k-k').x/L}
(per particle dimension).  With V_ext and V12 single cosine modes the pseudo-
difference operator is exact, so the only differences to the grid scheme are
the cubic-spline interpolation (O(h^4)) and the time splitting (O(tau^2)).

Uses numpy only; shares nothing with the oracle or the HIP path.
"""
from __future__ import annotations

import math

import numpy as np


class RingPair:
    def __init__(self, L=20.0, M=16, v0=0.6, u=0.9, hbar=1.0, mass=1.0, sigma=1.5,
                 a=(-2.0, 2.0), kq=(1, -1)):
        self.L, self.M, self.hbar = L, M, hbar
        self.ks = np.arange(-M // 2, M // 2)
        ks = self.ks
        # initial symmetrised pair of periodic Gaussian packets with momenta
        # 2 pi kq / L, projected on |k| < M/2 and normalised.
        nf = 256
        xs = -0.5 * L + np.arange(nf) * L / nf

        def phi(a0, kq0):
            q = 2 * math.pi * kq0 / L * hbar
            return sum((2 * math.pi * sigma**2) ** -0.25
                       * np.exp(-((xs - a0 - j * L) ** 2) / (4 * sigma**2) + 1j * q * xs / hbar)
                       for j in (-1, 0, 1))

        pa, pb = phi(a[0], kq[0]), phi(a[1], kq[1])
        psi = np.outer(pa, pb) + np.outer(pb, pa)
        C = np.fft.fft2(psi) / nf**2
        kk = np.fft.fftfreq(nf, 1.0 / nf).astype(int)
        ph = np.exp(-2j * math.pi * kk * (-0.5 * L) / L)
        C = C * ph[:, None] * ph[None, :]
        c = np.array([[C[k1 % nf, k2 % nf] for k2 in ks] for k1 in ks])
        self.c0 = c / math.sqrt((abs(c) ** 2).sum() * L * L)
        # H in the truncated basis: kinetic + V0 cos(2 pi x_j/L) + U cos(2 pi (x1-x2)/L)
        nb = M * M
        H = np.zeros((nb, nb))
        kin = hbar**2 / (2 * mass) * (2 * math.pi / L) ** 2
        for i in range(M):
            for j in range(M):
                r = i * M + j
                H[r, r] = kin * (ks[i] ** 2 + ks[j] ** 2)
                for d in (-1, 1):
                    if 0 <= i + d < M:
                        H[(i + d) * M + j, r] += v0 / 2
                    if 0 <= j + d < M:
                        H[i * M + j + d, r] += v0 / 2
                    if 0 <= i + d < M and 0 <= j - d < M:
                        H[(i + d) * M + j - d, r] += u / 2
        self.ev, self.Q = np.linalg.eigh(H)

    def coeffs(self, t):
        v = self.c0.reshape(-1)
        w = self.Q @ (np.exp(-1j * self.ev * t / self.hbar) * (self.Q.conj().T @ v))
        return w.reshape(self.M, self.M)

    def wigner(self, c, nx, nk):
        L, M, ks = self.L, self.M, self.ks
        x = -0.5 * L + np.arange(nx) * L / nx
        E = np.exp(2j * math.pi * np.outer(x, np.arange(-2 * M, 2 * M + 1)) / L)
        f = np.zeros((nx, nx, nk, nk))
        for a1, k1 in enumerate(ks):
            for b1, k1p in enumerate(ks):
                n1 = k1 + k1p + nk // 2
                if not 0 <= n1 < nk:
                    continue
                e1 = E[:, k1 - k1p + 2 * M]
                # all (k2, k2') at once
                cc = c[a1, :][:, None] * np.conj(c[b1, :])[None, :]  # [a2, b2]
                for a2, k2 in enumerate(ks):
                    for b2, k2p in enumerate(ks):
                        n2 = k2 + k2p + nk // 2
                        if not 0 <= n2 < nk:
                            continue
                        f[:, :, n1, n2] += (cc[a2, b2] * np.outer(e1, E[:, k2 - k2p + 2 * M])).real
        return f * (2 * L / (2 * math.pi * self.hbar)) ** 2
