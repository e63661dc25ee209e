"""Plain FP64 CPU oracle for the two-body Wigner step (arXiv:2511.11354).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_2511_11354_amd``) never imports it, and it imports nothing from the
product.  The arithmetic lives in ``wig2_oracle.c`` (plain loops, no BLAS, no
FFT); this module only marshals numpy arrays through ctypes.

Functions follow the paper's sections:
  * grid and momentum nodes ............ Sec. 3.1 (torus), Sec. 3.2 (box, SEM)
  * neutralised Poisson Hartree ........ Sec. 3.1.1 (1-D Coulomb example)
  * symbols sig_m, Vhat_m .............. Sec. 3.1.1 / 3.1.2 (eqs. Hartree_FSM,
                                         two_body_FSM; sign: eq. sWigner)
  * SEM single-body matrix ............. Sec. 3.2.1 (eq. Chebyshev_PDO)
  * SEM two-body operator .............. Sec. 3.2.2 (Poisson summation, D_V, O tensor)
  * cubic-spline advection ............. Sec. 4.1 (B-splines, A_per, A_nat)
  * Strang / Lawson step ............... Sec. 4.1 (Lawson predictor-corrector)
  * observables, 1-RDM entropy ......... Sec. 2.2, Sec. 5.3, Appendix B
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "wig2_oracle.c")

_dp = ctypes.POINTER(ctypes.c_double)


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("nk", ctypes.c_int), ("periodic", ctypes.c_int),
                ("cells", ctypes.c_int), ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
                ("k_max", ctypes.c_double), ("hbar", ctypes.c_double), ("mass", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("scheme", ctypes.c_int), ("lam", ctypes.c_double),
                ("xc", ctypes.c_int), ("xc_n0", ctypes.c_double), ("n_scale", ctypes.c_double),
                ("two_body", ctypes.c_int), ("hartree", ctypes.c_int)]


class Tables(ctypes.Structure):
    _fields_ = [("sig_ext", _dp), ("vhat12", _dp), ("K", _dp), ("v12_pair", _dp), ("v12_sem", _dp)]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C99, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", _SO, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        G = ctypes.POINTER(Grid)
        P = ctypes.POINTER(Params)
        T = ctypes.POINTER(Tables)
        sig = {
            "or_num_threads": ([], ctypes.c_int),
            "or_set_threads": ([ctypes.c_int], None),
            "or_dx": ([G], ctypes.c_double),
            "or_xnodes": ([G, _dp], None),
            "or_pnodes": ([G, _dp, _dp], None),
            "or_sigma_ext": ([G, _dp, _dp], None),
            "or_vhat12": ([G, _dp, _dp], None),
            "or_sigma_hxc": ([G, _dp, _dp], None),
            "or_veff_hxc": ([G, P, _dp, _dp, _dp], None),
            "or_densities": ([G, _dp, _dp, _dp], None),
            "or_hartree_poisson": ([G, _dp, _dp], None),
            "or_hartree_padded": ([G, _dp, _dp, _dp], None),
            "or_theta_periodic": ([G, _dp, _dp, _dp, ctypes.c_int, ctypes.c_long, ctypes.c_long,
                                   _dp, _dp], None),
            "or_theta_dense": ([G, _dp, _dp, ctypes.c_long, ctypes.c_long, _dp, _dp], None),
            "or_sem_kernel": ([G, _dp, _dp], None),
            "or_sem12_dy": ([G], ctypes.c_double),
            "or_theta12_sem": ([G, _dp, ctypes.c_long, ctypes.c_long, _dp, _dp], None),
            "or_advect": ([G, ctypes.c_int, ctypes.c_double, ctypes.c_long, ctypes.c_long,
                           _dp, _dp], ctypes.c_int),
            "or_step": ([G, P, T, _dp, ctypes.c_long], ctypes.c_int),
            "or_observables": ([G, _dp, _dp, _dp, _dp, _dp, _dp, _dp], None),
            "or_rho1_entropy": ([G, _dp, _dp, _dp], ctypes.c_int),
            "or_jacobi_eigvals": ([ctypes.c_int, _dp, _dp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def grid(nx, nk, periodic=True, cells=1, x_min=-10.0, x_max=10.0, k_max=0.0, hbar=1.0, mass=1.0):
    return Grid(nx, nk, int(periodic), cells, x_min, x_max, k_max, hbar, mass)


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def dx(g: Grid) -> float:
    return lib().or_dx(ctypes.byref(g))


def xnodes(g: Grid) -> np.ndarray:
    x = np.zeros(g.nx)
    lib().or_xnodes(ctypes.byref(g), _p(x))
    return x


def pnodes(g: Grid):
    p = np.zeros(g.nk)
    w = np.zeros(g.nk)
    lib().or_pnodes(ctypes.byref(g), _p(p), _p(w))
    return p, w


def symbol_sample_points(g: Grid) -> np.ndarray:
    """y_j = x_min + j L/(2nk): where V_ext is sampled for its symbol."""
    L = g.x_max - g.x_min
    return g.x_min + np.arange(2 * g.nk) * L / (2 * g.nk)


def pair_sample_points(g: Grid) -> np.ndarray:
    """r_j = -L/2 + j L/(2nk): where V12 is sampled for its Fourier modes."""
    L = g.x_max - g.x_min
    return -0.5 * L + np.arange(2 * g.nk) * L / (2 * g.nk)


def pair_separations(g: Grid) -> np.ndarray:
    """x_i1 - x_i2 for every pair, wrapped to the minimum image on the torus."""
    x = xnodes(g)
    r = x[:, None] - x[None, :]
    if g.periodic:
        L = g.x_max - g.x_min
        r = r - L * np.floor((r + 0.5 * L) / L)
    return np.ascontiguousarray(r)


def sigma_ext(g: Grid, v_y: np.ndarray) -> np.ndarray:
    s = np.zeros((g.nx, g.nk))
    lib().or_sigma_ext(ctypes.byref(g), _p(np.ascontiguousarray(v_y, dtype=np.float64)), _p(s))
    return s


def vhat12(g: Grid, v12_r: np.ndarray) -> np.ndarray:
    v = np.zeros(g.nk)
    lib().or_vhat12(ctypes.byref(g), _p(np.ascontiguousarray(v12_r, dtype=np.float64)), _p(v))
    return v


def sigma_hxc(g: Grid, v_x: np.ndarray) -> np.ndarray:
    s = np.zeros((g.nx, g.nk))
    lib().or_sigma_hxc(ctypes.byref(g), _p(np.ascontiguousarray(v_x, dtype=np.float64)), _p(s))
    return s


def densities(g: Grid, f: np.ndarray):
    n1 = np.zeros(g.nx)
    n2 = np.zeros(g.nx)
    lib().or_densities(ctypes.byref(g), _p(f), _p(n1), _p(n2))
    return n1, n2


def veff_hxc(g: Grid, lam, xc, xc_n0, n_scale, v12_pair, n, hartree="pair"):
    prm = Params(0.0, 0, lam, int(xc), xc_n0, n_scale, 1, HARTREE[hartree])
    v = np.zeros(g.nx)
    lib().or_veff_hxc(ctypes.byref(g), ctypes.byref(prm), _p(v12_pair), _p(np.ascontiguousarray(n, dtype=np.float64)),
                      _p(v))
    return v


HARTREE = {"pair": 0, "poisson": 1}


def hartree_padded_points(g: Grid) -> np.ndarray:
    """Separations nu dx, nu in [-3nx/2, 3nx/2), at which the zero-padded box
    Hartree term samples V12."""
    nt = 3 * g.nx
    return np.arange(-(nt // 2), nt - nt // 2) * dx(g)


def hartree_padded(g: Grid, v12_pad, n):
    """Box Hartree potential by the zero-padded transform (Sec. 3.2.1 remark)."""
    v = np.zeros(g.nx)
    lib().or_hartree_padded(ctypes.byref(g), _p(np.ascontiguousarray(v12_pad, dtype=np.float64)),
                            _p(np.ascontiguousarray(n, dtype=np.float64)), _p(v))
    return v


def hartree_poisson(g: Grid, n):
    """Neutralised-background Poisson Hartree potential (Sec. 3.1.1 example)."""
    v = np.zeros(g.nx)
    lib().or_hartree_poisson(ctypes.byref(g), _p(np.ascontiguousarray(n, dtype=np.float64)), _p(v))
    return v


def _out(f, out):
    """A caller-supplied output array (written only where the call computes)
    or a fresh zeroed one."""
    if out is None:
        return np.zeros_like(f)
    if out.shape != f.shape or out.dtype != np.float64 or not out.flags.c_contiguous:
        raise ValueError("out must be a C-contiguous float64 array of f's shape")
    return out


def theta_periodic(g: Grid, sig1, sig2, vh12, f, two_body=True, plane0=0, nplanes=None, out=None):
    if nplanes is None:
        nplanes = g.nx * g.nx - plane0
    out = _out(f, out)
    lib().or_theta_periodic(ctypes.byref(g), _p(sig1), _p(sig2), _p(vh12), int(two_body),
                            plane0, nplanes, _p(f), _p(out))
    return out


def theta_dense(g: Grid, K1, K2, f, plane0=0, nplanes=None, out=None):
    if nplanes is None:
        nplanes = g.nx * g.nx - plane0
    out = _out(f, out)
    lib().or_theta_dense(ctypes.byref(g), _p(K1), _p(K2), plane0, nplanes, _p(f), _p(out))
    return out


def sem_kernel(g: Grid, v_x: np.ndarray) -> np.ndarray:
    K = np.zeros((g.nx, g.nk, g.nk))
    lib().or_sem_kernel(ctypes.byref(g), _p(np.ascontiguousarray(v_x, dtype=np.float64)), _p(K))
    return K


def sem12_dy(g: Grid) -> float:
    return lib().or_sem12_dy(ctypes.byref(g))


def sem12_sample_points(g: Grid) -> np.ndarray:
    """Arguments l dx + d dy (l in [-(nx-1), nx-1], d in [-(nk-1), nk-1]) at
    which the two-body SEM operator of the box samples V12."""
    l = np.arange(-(g.nx - 1), g.nx)[:, None]
    d = np.arange(-(g.nk - 1), g.nk)[None, :]
    return l * dx(g) + d * sem12_dy(g)


def theta12_sem(g: Grid, v12_tab, f, plane0=0, nplanes=None, out=None):
    """Box two-body operator (Sec. 3.2.2) on the planes [plane0, plane0 + nplanes)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    np_ = g.nx * g.nx if nplanes is None else nplanes
    out = _out(f, out)
    lib().or_theta12_sem(ctypes.byref(g), _p(np.ascontiguousarray(v12_tab, dtype=np.float64)), plane0, np_,
                         _p(f), _p(out))
    return out


def advect(g: Grid, dim: int, s: float, f: np.ndarray, line0=0, nlines=None, out=None) -> np.ndarray:
    if nlines is None:
        nlines = g.nx * g.nk * g.nk - line0
    out = _out(f, out)
    rc = lib().or_advect(ctypes.byref(g), dim, s, line0, nlines, _p(f), _p(out))
    if rc:
        raise RuntimeError("or_advect failed")
    return out


def tables(g: Grid, vext=None, v12=None):
    """Sample the potentials (Python callables) where the method needs them and
    build the oracle's tables."""
    d = {}
    if g.periodic:
        vy = np.array([vext(y) for y in symbol_sample_points(g)]) if vext else np.zeros(2 * g.nk)
        d["sig_ext"] = sigma_ext(g, vy)
        vr = np.array([v12(r) for r in pair_sample_points(g)]) if v12 else np.zeros(2 * g.nk)
        d["vhat12"] = vhat12(g, vr)
        d["K"] = None
    else:
        vx = np.array([vext(x) for x in xnodes(g)]) if vext else np.zeros(g.nx)
        d["K"] = sem_kernel(g, vx)
        d["sig_ext"] = None
        d["vhat12"] = None
        d["v12_sem"] = (np.ascontiguousarray(np.vectorize(v12)(sem12_sample_points(g)), dtype=np.float64)
                        if v12 else None)
    r = pair_separations(g)
    d["v12_pair"] = np.ascontiguousarray(np.vectorize(v12)(r) if v12 else np.zeros_like(r))
    d["vext_x"] = np.array([vext(x) for x in xnodes(g)]) if vext else np.zeros(g.nx)
    return d


def step(g: Grid, f: np.ndarray, tb: dict, nsteps: int, dt: float, scheme: str = "strang",
         lam: float = 0.0, xc: bool = False, xc_n0: float = 1.0, n_scale: float = 1.0,
         two_body: bool = True, hartree: str = "pair") -> np.ndarray:
    out = np.ascontiguousarray(f, dtype=np.float64).copy()
    prm = Params(dt, 0 if scheme == "strang" else 1, lam, int(xc), xc_n0, n_scale, int(two_body),
                 HARTREE[hartree])
    t = Tables(_p(tb["sig_ext"]), _p(tb["vhat12"]), _p(tb["K"]), _p(tb["v12_pair"]), _p(tb.get("v12_sem")))
    rc = lib().or_step(ctypes.byref(g), ctypes.byref(prm), ctypes.byref(t), _p(out), nsteps)
    if rc:
        raise RuntimeError(f"or_step failed ({rc})")
    return out


def observables(g: Grid, f: np.ndarray, vext_x=None, v12_pair=None):
    scal = np.zeros(3)
    n1 = np.zeros(g.nx)
    n12 = np.zeros((g.nx, g.nx))
    f1 = np.zeros((g.nx, g.nk))
    lib().or_observables(ctypes.byref(g), _p(f), _p(vext_x), _p(v12_pair), _p(scal), _p(n1),
                         _p(n12), _p(f1))
    return {"mass": scal[0], "energy": scal[1], "l2": scal[2], "n1": n1, "n12": n12, "f1": f1}


def rho1_entropy(g: Grid, f1: np.ndarray):
    ev = np.zeros((g.nx + 1) // 2)
    s = ctypes.c_double(0.0)
    lib().or_rho1_entropy(ctypes.byref(g), _p(np.ascontiguousarray(f1)), _p(ev), ctypes.byref(s))
    return ev, s.value


def jacobi_eigvals(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64).copy()
    ev = np.zeros(a.shape[0])
    lib().or_jacobi_eigvals(a.shape[0], _p(a), _p(ev))
    return np.sort(ev)


def errors(f: np.ndarray, ref: np.ndarray):
    """Relative L-inf and L2 errors of Sec. 5.1 (integral = grid average)."""
    m = np.max(np.abs(ref))
    return float(np.max(np.abs(f - ref)) / m), float(np.sqrt(np.mean((f - ref) ** 2)) / m)
