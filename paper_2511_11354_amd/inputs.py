"""Seeded synthetic inputs: potentials, initial Wigner functions, workloads.

This module holds none of the method's arithmetic.  It evaluates closed-form
potentials and initial states at node arrays handed to it by the caller, so the
oracle and the HIP path can both be fed from it without sharing any code.

Initial states follow the analytic initial conditions of the paper's
experiments (Sec. 5.2-5.3): Gaussian wave packets, either as the Wigner
function of a symmetrised two-particle pure state or as an incoherent,
exchange-symmetric mixture of packet pairs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# potentials (plain Python callables of one float)
# --------------------------------------------------------------------------


def cosine(v0: float, L: float):
    """V(x) = v0 cos(2 pi x / L)."""
    return lambda x: v0 * math.cos(2.0 * math.pi * x / L)


def fourier_modes(coeffs, L: float):
    """V(x) = sum_m a_m cos(2 pi m x / L) + b_m sin(2 pi m x / L) for
    coeffs = [(a_1, b_1), (a_2, b_2), ...]: a lattice potential whose
    single-body symbol has exactly len(coeffs) modes."""
    cs = [(m + 1, float(a), float(b)) for m, (a, b) in enumerate(coeffs)]
    return lambda x: sum(a * math.cos(2.0 * math.pi * m * x / L) + b * math.sin(2.0 * math.pi * m * x / L)
                         for m, a, b in cs)


def smoothed_coulomb(u: float = 1.0, eps: float = 1.0):
    """V12(r) = u / sqrt(r^2 + eps)  (Sec. 2.3, 1-D smoothed Coulomb)."""
    return lambda r: u / math.sqrt(r * r + eps)


def gaussian_pair(hb: float):
    """V12(r) = hb exp(-r^2/2)  (the two-body convergence test, Sec. 5.1.2)."""
    return lambda r: hb * math.exp(-0.5 * r * r)


def gaussian_well(r0: float):
    """V(x) = (2 pi)^{-1/2} exp(-(x + r0)^2/2)  (the XC convergence test, Sec. 5.1.1)."""
    return lambda x: math.exp(-0.5 * (x + r0) ** 2) / math.sqrt(2.0 * math.pi)


def harmonic(omega: float = 0.5):
    """V(x) = omega^2 x^2 / 2."""
    return lambda x: 0.5 * omega * omega * x * x


def double_well():
    """V(x) = (x^2 - 4)^2 / 32."""
    return lambda x: (x * x - 4.0) ** 2 / 32.0


def zero():
    return lambda x: 0.0


# --------------------------------------------------------------------------
# Gaussian packets in phase space
# --------------------------------------------------------------------------


def cross_wigner(x, p, a_j, q_j, a_k, q_k, sigma=1.0, hbar=1.0):
    """Cross-Wigner function of two Gaussian packets
    phi(x) = (2 pi sigma^2)^{-1/4} exp(-(x - a)^2/(4 sigma^2) + i q x / hbar):
      W_jk = (1/(pi hbar)) exp(-(x - abar)^2/(2 sigma^2) - 2 sigma^2 (p - qbar)^2/hbar^2)
             * exp(i [dq x - (p - qbar) da] / hbar).
    x, p broadcast against each other."""
    ab, qb = 0.5 * (a_j + a_k), 0.5 * (q_j + q_k)
    da, dq = a_j - a_k, q_j - q_k
    g = np.exp(-((x - ab) ** 2) / (2 * sigma**2) - 2 * sigma**2 * (p - qb) ** 2 / hbar**2)
    return g * np.exp(1j * (dq * x - (p - qb) * da) / hbar) / (math.pi * hbar)


def symmetrised_pair(x, p, a=(-2.0, 2.0), q=(0.5, -0.5), sigma=1.0, hbar=1.0):
    """Wigner function f(x1,x2,p1,p2) of the bosonic pure state
    psi = N (phi_a phi_b + phi_b phi_a), laid out [i1][i2][n1][n2]:
      f = N^2 [W_aa W_bb + W_bb W_aa + 2 Re(W_ab W_ba)],  N^2 = 1/(2(1+|s|^2)),
    s = <phi_a|phi_b>, |s| = exp(-da^2/(8 sigma^2) - sigma^2 dq^2/(2 hbar^2))."""
    X, P = np.meshgrid(np.asarray(x, float), np.asarray(p, float), indexing="ij")
    (aa, ab_), (qa, qb) = a, q
    Waa = cross_wigner(X, P, aa, qa, aa, qa, sigma, hbar).real
    Wbb = cross_wigner(X, P, ab_, qb, ab_, qb, sigma, hbar).real
    Wab = cross_wigner(X, P, aa, qa, ab_, qb, sigma, hbar)
    Wba = np.conj(Wab)
    s2 = math.exp(-((aa - ab_) ** 2) / (4 * sigma**2) - sigma**2 * (qa - qb) ** 2 / hbar**2)
    n2 = 1.0 / (2.0 * (1.0 + s2))
    # f[i1, i2, n1, n2] = W(x_i1, p_n1) W'(x_i2, p_n2)
    t = (np.einsum("ac,bd->abcd", Waa, Wbb) + np.einsum("ac,bd->abcd", Wbb, Waa)
         + 2.0 * np.einsum("ac,bd->abcd", Wab, Wba).real)
    return np.ascontiguousarray(n2 * t)


def packet(x, p, a, q, sigma=1.0, hbar=1.0, period=None):
    """G(x,p) = (1/(pi hbar)) exp(-(x-a)^2/(2 sigma^2) - 2 sigma^2 (p-q)^2/hbar^2),
    summed over the images x +- period when a period is given."""
    X, P = np.meshgrid(np.asarray(x, float), np.asarray(p, float), indexing="ij")
    shifts = [0.0] if period is None else [-period, 0.0, period]
    g = sum(np.exp(-((X - a - s) ** 2) / (2 * sigma**2)) for s in shifts)
    return g * np.exp(-2 * sigma**2 * (P - q) ** 2 / hbar**2) / (math.pi * hbar)


def mixture_params(seed: int):
    """Seeded packet set for the Gaussian-mixture workloads: K ~ U{2,3,4},
    a_j ~ U[-5,5], q_j ~ U[-1.5,1.5], w_j ~ U[0.5,1.5] (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    K = int(rng.integers(2, 5))
    a = rng.uniform(-5.0, 5.0, K)
    q = rng.uniform(-1.5, 1.5, K)
    w = rng.uniform(0.5, 1.5, K)
    return a, q, w


def mixture(x, p, seed: int, sigma=1.0, hbar=1.0, period=None, dtype=np.float64):
    """Exchange-symmetric incoherent mixture
      f = sum_{i != j} w_i w_j G_i(x1,p1) G_j(x2,p2) / sum_{i != j} w_i w_j,
    assembled as (A x A - sum_i w_i^2 G_i x G_i) / norm with A = sum_i w_i G_i,
    one x1 slab at a time."""
    a, q, w = mixture_params(seed)
    G = [packet(x, p, a[j], q[j], sigma, hbar, period) for j in range(len(a))]
    A = sum(w[j] * G[j] for j in range(len(a)))
    norm = float(w.sum() ** 2 - (w**2).sum())
    nx, nk = A.shape
    f = np.empty((nx, nx, nk, nk), dtype=dtype)
    for i1 in range(nx):
        slab = A[i1][None, :, None] * A[:, None, :]
        for j in range(len(a)):
            slab -= (w[j] ** 2) * G[j][i1][None, :, None] * G[j][:, None, :]
        f[i1] = slab / norm
    return f


def random_field(shape, seed: int, dtype=np.float64):
    """Plain seeded normal noise (for operator-level parity on unstructured data)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    nx: int
    nk: int
    periodic: bool = True
    cells: int = 1
    x_min: float = -10.0
    x_max: float = 10.0
    k_max: float = 0.0
    hbar: float = 1.0
    mass: float = 1.0
    dt: float = 0.01
    steps: int = 20
    vext: object = None
    v12: object = None
    extra: dict = field(default_factory=dict)

    @property
    def points(self) -> int:
        return self.nx * self.nx * self.nk * self.nk


def tiny_periodic() -> Workload:
    """Periodic box L=20, 32^4, V_ext = 0.5 cos(2 pi x/L), V12 = 1/sqrt(r^2+1),
    symmetrised packets at +-2 with momenta +-0.5, dt = 0.01, 20 Strang steps."""
    return Workload("periodic-32x32x32x32-fp64", 32, 32, dt=0.01, steps=20,
                    vext=cosine(0.5, 20.0), v12=smoothed_coulomb(1.0, 1.0))


def large_periodic(u: float = 1.0) -> Workload:
    """Periodic box L=20, 128^4, same V_ext, V12 = U/sqrt(r^2+1), dt = 0.005,
    seeded Gaussian-mixture initial states."""
    return Workload("periodic-128x128x128x128", 128, 128, dt=0.005, steps=1000,
                    vext=cosine(0.5, 20.0), v12=smoothed_coulomb(u, 1.0), extra={"U": u})


def box_sem(nx=129, cells=16, nodes=16, potential="harmonic", pair_u=None) -> Workload:
    """Non-periodic box [-15,15], natural spline, SEM momentum grid on
    [-10 pi/3, 10 pi/3] with `cells` x `nodes` Chebyshev-Gauss points; with
    pair_u the smoothed Coulomb pair potential pair_u / sqrt(r^2 + 1)."""
    v = harmonic(0.5) if potential == "harmonic" else double_well()
    tag = "" if pair_u is None else f"-pair{pair_u:g}"
    return Workload(f"box-sem-{nx}x{cells * nodes}-{potential}{tag}", nx, cells * nodes,
                    periodic=False, cells=cells, x_min=-15.0, x_max=15.0,
                    k_max=10.0 * math.pi / 3.0, dt=0.01, steps=1000, vext=v,
                    v12=None if pair_u is None else smoothed_coulomb(pair_u, 1.0),
                    extra={} if pair_u is None else {"U": pair_u})


def ensemble(seed0: int = 1000, count: int = 64):
    """Batched ensemble: per instance (seed 1000+s) Nx, Nk ~ U{32,48,64,96},
    U ~ U[0.5, 3], L = 20, V_ext = 0.5 cos, dt = 0.005."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(seed0 + s)
        nx = int(rng.choice([32, 48, 64, 96]))
        nk = int(rng.choice([32, 48, 64, 96]))
        u = float(rng.uniform(0.5, 3.0))
        out.append(Workload(f"ens-{s}", nx, nk, dt=0.005, steps=1000, vext=cosine(0.5, 20.0),
                            v12=smoothed_coulomb(u, 1.0), extra={"U": u, "seed": seed0 + s}))
    return out


# --------------------------------------------------------------------------
# Plasma workloads of Sec. 5 (Wigner-Poisson with the two-body term)
# --------------------------------------------------------------------------


def plasma_state(x, p, kind="landau", eps=0.1, k=0.4, dtype=np.float64):
    """Uncorrelated initial states of Sec. 5, f(x1,x2,p1,p2) = g(x1,p1) g(x2,p2):
      landau:     g = (1/sqrt(2 pi)) (1 + eps cos k x) e^{-p^2/2}
      two-stream: g = (1 + eps cos k x) (1 + 5 p^2) e^{-p^2/2} / (6 sqrt(2 pi))
    (the printed 1/(2 pi) and 1/(6 sqrt(2 pi))^2 split between the particles)."""
    X, P = np.meshgrid(np.asarray(x, float), np.asarray(p, float), indexing="ij")
    if kind == "landau":
        g = (1 + eps * np.cos(k * X)) * np.exp(-P**2 / 2) / math.sqrt(2 * math.pi)
    elif kind == "two-stream":
        g = (1 + eps * np.cos(k * X)) * (1 + 5 * P**2) * np.exp(-P**2 / 2) / (6 * math.sqrt(2 * math.pi))
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(np.einsum("ac,bd->abcd", g, g).astype(dtype))


def plasma(kind="landau", nx=256, nk=128, eps=None, pair_eps=1.0, gamma=1.0, two_body=True) -> Workload:
    """Quantum Landau damping / two-stream instability of Sec. 5: torus
    [-5 pi, 5 pi] (dx = 5 pi / 128 at nx = 256; the printed 257 nodes count
    the periodic end twice), dp = hbar pi / L = 0.1 (nk = 128: p in
    [-6.4, 6.3]), dt = 0.01, no V_ext; the neutralised-Poisson Hartree term
    with weight 1/L (reading: the density in the Poisson equation per unit
    length of the other particle's coordinate, so the plasma frequency is 1),
    and the pair potential gamma / sqrt(r^2 + pair_eps) when two_body."""
    L = 10 * math.pi
    if eps is None:
        eps = 0.1 if kind == "landau" else 0.02
    v12 = smoothed_coulomb(gamma, pair_eps) if two_body else None
    tag = f"-pair{pair_eps:g}" if two_body else "-hartree"
    return Workload(f"{kind}-{nx}x{nk}{tag}", nx, nk, x_min=-L / 2, x_max=L / 2, dt=0.01, steps=20000,
                    vext=None, v12=v12,
                    extra={"kind": kind, "eps": eps, "k": 0.4, "lam": 1.0 / L, "hartree": "poisson"})
