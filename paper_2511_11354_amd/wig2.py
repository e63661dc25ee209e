"""ctypes binding of libwig2 (C ABI in include/wig2.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device buffers may be torch tensors (``.data_ptr()`` is passed through); torch
is used for device memory and streams, nothing else.  Loading fails loudly if
the built library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwig2.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENOTSUP, ENUMERIC = 0, -1, -2, -3, -4, -5, -6
STRANG, LAWSON_PC = 0, 1
FP64, FP32, BF16X2 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x2": BF16X2}
SCHEMES = {"strang": STRANG, "lawson": LAWSON_PC}


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nk", ctypes.c_int32), ("periodic", ctypes.c_int32),
                ("sem_cells", ctypes.c_int32), ("x_min", ctypes.c_double),
                ("x_max", ctypes.c_double), ("k_max", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("hbar", ctypes.c_double), ("mass", ctypes.c_double), ("dt", ctypes.c_double),
                ("scheme", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("meanfield_lambda", ctypes.c_double), ("xc", ctypes.c_int32),
                ("xc_n0", ctypes.c_double), ("n_scale", ctypes.c_double)]


class Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double), ("mass", ctypes.c_double),
                ("energy", ctypes.c_double), ("l2", ctypes.c_double),
                ("entropy_vn", ctypes.c_double), ("fallbacks", ctypes.c_int32)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("blocks", ctypes.c_int32), ("k_p", ctypes.c_int32),
                ("k_x", ctypes.c_int32), ("block", ctypes.c_int32), ("epochs", ctypes.c_int32),
                ("lr", ctypes.c_double), ("seed", ctypes.c_uint64), ("train_blocks", ctypes.c_int32),
                ("max_points", ctypes.c_int32)]

PROF_NAMES = ("advect_x1", "advect_x2", "theta_stage1", "theta_stage2", "meanfield", "theta_heun",
              "advect_x1x1", "pair_sem")

FN1 = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_double, ctypes.c_void_p)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p

# name -> (argtypes, restype)
SIGNATURES = {
    "wig2_create": ([ctypes.POINTER(Grid), ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)],
                    ctypes.c_int),
    "wig2_set_potentials": ([_vp, FN1, FN1, _vp], ctypes.c_int),
    "wig2_set_state": ([_vp, _dp], ctypes.c_int),
    "wig2_get_state": ([_vp, _dp], ctypes.c_int),
    "wig2_state_buffer": ([_vp, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "wig2_state_written": ([_vp], ctypes.c_int),
    "wig2_bind_state": ([_vp, _vp, ctypes.c_int32], ctypes.c_int),
    "wig2_step": ([_vp, ctypes.c_int64], ctypes.c_int),
    "wig2_observables": ([_vp, ctypes.POINTER(Obs), _dp, _dp, _dp], ctypes.c_int),
    "wig2_theta": ([_vp, _vp, _vp], ctypes.c_int),
    "wig2_advect": ([_vp, ctypes.c_int32, ctypes.c_double, _vp, _vp], ctypes.c_int),
    "wig2_advect_noalloc": ([_vp, ctypes.c_int32, ctypes.c_double, _vp, _vp], ctypes.c_int),
    "wig2_nodes": ([_vp, _dp, _dp, _dp], ctypes.c_int),
    "wig2_profile": ([_vp, ctypes.c_int32], ctypes.c_int),
    "wig2_profile_read": ([_vp, _dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32], ctypes.c_int),
    "wig2_band": ([_vp], ctypes.c_int),
    "wig2_set_theta_path": ([_vp, ctypes.c_int32], ctypes.c_int),
    "wig2_set_hartree": ([_vp, ctypes.c_int32], ctypes.c_int),
    "wig2_set_sweep_fusion": ([_vp, ctypes.c_int32], ctypes.c_int),
    "wig2_theta_path": ([_vp], ctypes.c_int),
    "wig2_batch_create": ([ctypes.c_int32, ctypes.POINTER(Grid), ctypes.POINTER(Params), _vp,
                           ctypes.POINTER(_vp)], ctypes.c_int),
    "wig2_batch_set_potentials": ([_vp, ctypes.c_int32, FN1, FN1, _vp], ctypes.c_int),
    "wig2_batch_set_state": ([_vp, ctypes.c_int32, _dp], ctypes.c_int),
    "wig2_batch_get_state": ([_vp, ctypes.c_int32, _dp], ctypes.c_int),
    "wig2_batch_step": ([_vp, ctypes.c_int64], ctypes.c_int),
    "wig2_batch_observables": ([_vp, ctypes.c_int32, ctypes.POINTER(Obs), _dp, _dp, _dp],
                               ctypes.c_int),
    "wig2_batch_tune": ([_vp, ctypes.c_char_p, ctypes.c_int32], ctypes.c_int),
    "wig2_batch_info": ([_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
                        ctypes.c_int),
    "wig2_batch_destroy": ([_vp], None),
    "wig2_batch_last_error": ([_vp], ctypes.c_char_p),
    "wig2_surrogate_create": ([ctypes.POINTER(TrainCfg), ctypes.POINTER(_vp)], ctypes.c_int),
    "wig2_surrogate_size": ([_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "wig2_surrogate_train": ([_vp, ctypes.POINTER(TrainCfg), ctypes.POINTER(_vp)], ctypes.c_int),
    "wig2_surrogate_destroy": ([_vp], None),
    "wig2_surrogate_last_error": ([_vp], ctypes.c_char_p),
    "wig2_surrogate_collect": ([_vp, _vp, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "wig2_surrogate_stats": ([_vp, _dp, _dp, ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "wig2_surrogate_get_params": ([_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
                                  ctypes.c_int),
    "wig2_surrogate_set_params": ([_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
                                  ctypes.c_int),
    "wig2_surrogate_grad": ([_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_float), _dp], ctypes.c_int),
    "wig2_surrogate_attach": ([_vp, _vp, ctypes.c_double, ctypes.c_int32], ctypes.c_int),
    "wig2_surrogate_detach": ([_vp], ctypes.c_int),
    "wig2_surrogate_report": ([_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_int64), _dp], ctypes.c_int),
    "wig2_destroy": ([_vp], None),
    "wig2_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "wig2_last_error": ([_vp], ctypes.c_char_p),
}

_lib = None


def lib():
    """Load libwig2.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2511_11354_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class Wig2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
        return a.ctypes.data_as(_dp)
    return a


def _dev(t):
    """Device pointer of a torch tensor (or an int address).  The library
    works on its context's stream; work that torch has queued on the
    tensor's current stream (the fill or cast that produced it) is waited
    for first, so the call sees the finished tensor."""
    if hasattr(t, "data_ptr"):
        assert t.is_cuda and t.is_contiguous()
        import torch

        torch.cuda.current_stream(t.device).synchronize()
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


class Solver:
    """One context: grid, parameters, potentials and the device-resident state."""

    def __init__(self, nx, nk, *, periodic=True, sem_cells=1, x_min=-10.0, x_max=10.0,
                 k_max=0.0, hbar=1.0, mass=1.0, dt=0.01, scheme="strang", precision="fp64",
                 meanfield_lambda=0.0, xc=False, xc_n0=1.0, n_scale=1.0, stream=None):
        self._L = lib()
        self.grid = Grid(nx, nk, int(periodic), sem_cells, x_min, x_max, k_max)
        self.params = Params(hbar, mass, dt, SCHEMES[scheme], PRECISIONS[precision],
                             meanfield_lambda, int(xc), xc_n0, n_scale)
        self.nx, self.nk = nx, nk
        self.shape = (nx, nx, nk, nk)
        self.precision = precision
        self._cbs = []
        h = ctypes.c_void_p()
        s = None if stream is None else ctypes.c_void_p(int(stream))
        rc = self._L.wig2_create(ctypes.byref(self.grid), ctypes.byref(self.params), s,
                                 ctypes.byref(h))
        if rc != OK:
            raise Wig2Error(rc, f"wig2_create: {self._L.wig2_strerror(rc).decode()}")
        self._h = h

    # -- helpers ----------------------------------------------------------------
    def _check(self, rc, what):
        if rc != OK:
            msg = self._L.wig2_last_error(self._h).decode() or self._L.wig2_strerror(rc).decode()
            raise Wig2Error(rc, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._L.wig2_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API --------------------------------------------------------------------
    def set_potentials(self, v_ext=None, v12=None):
        cb = lambda fn: FN1(0) if fn is None else FN1(lambda x, u: float(fn(x)))
        a, b = cb(v_ext), cb(v12)
        self._cbs = [a, b]
        self._check(self._L.wig2_set_potentials(self._h, a, b, None), "wig2_set_potentials")

    def set_state(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == self.shape
        self._check(self._L.wig2_set_state(self._h, _ptr(f)), "wig2_set_state")

    def get_state(self):
        f = np.empty(self.shape, dtype=np.float64)
        self._check(self._L.wig2_get_state(self._h, _ptr(f)), "wig2_get_state")
        return f

    def state_buffer(self):
        p = ctypes.c_void_p()
        eb = ctypes.c_int32()
        self._check(self._L.wig2_state_buffer(self._h, ctypes.byref(p), ctypes.byref(eb)),
                    "wig2_state_buffer")
        return p.value, eb.value

    def state_written(self):
        self._check(self._L.wig2_state_written(self._h), "wig2_state_written")

    def bind_state(self, f_dev):
        """Step a caller-owned device tensor in place (None unbinds).  The
        tensor must outlive the binding."""
        if f_dev is None:
            self._check(self._L.wig2_bind_state(self._h, None, 0), "wig2_bind_state")
            self._bound = None
            return
        assert tuple(f_dev.shape) == self.shape
        dtype = FP64 if self.precision == "fp64" else FP32
        self._check(self._L.wig2_bind_state(self._h, _dev(f_dev), dtype), "wig2_bind_state")
        self._bound = f_dev

    def step(self, n=1):
        self._check(self._L.wig2_step(self._h, int(n)), "wig2_step")

    def observables(self):
        o = Obs()
        n1 = np.zeros(self.nx)
        n12 = np.zeros((self.nx, self.nx))
        f1 = np.zeros((self.nx, self.nk))
        self._check(self._L.wig2_observables(self._h, ctypes.byref(o), _ptr(n1), _ptr(n12),
                                             _ptr(f1)), "wig2_observables")
        return {"step": o.step, "t": o.t, "mass": o.mass, "energy": o.energy, "l2": o.l2,
                "entropy": o.entropy_vn, "fallbacks": o.fallbacks, "n1": n1, "n12": n12, "f1": f1}

    def theta(self, f_in, f_out):
        self._check(self._L.wig2_theta(self._h, _dev(f_in), _dev(f_out)), "wig2_theta")

    def advect(self, dim, s, f_in, f_out):
        self._check(self._L.wig2_advect(self._h, int(dim), float(s), _dev(f_in), _dev(f_out)),
                    "wig2_advect")

    def advect_noalloc(self, dim, s, f_in, f_out):
        """wig2_advect without device allocation (static per-device scratch)."""
        self._check(self._L.wig2_advect_noalloc(self._h, int(dim), float(s), _dev(f_in), _dev(f_out)),
                    "wig2_advect_noalloc")

    def profile(self, enable=True):
        self._check(self._L.wig2_profile(self._h, int(enable)), "wig2_profile")

    def profile_read(self, reset=True):
        ms = np.zeros(len(PROF_NAMES))
        cnt = (ctypes.c_int64 * len(PROF_NAMES))()
        self._check(self._L.wig2_profile_read(self._h, _ptr(ms), cnt, int(reset)),
                    "wig2_profile_read")
        return {n: (float(ms[i]), int(cnt[i])) for i, n in enumerate(PROF_NAMES)}

    HARTREE = {"pair": 0, "poisson": 1}

    def set_hartree(self, form: str):
        """Hartree term of the mean field: "pair" (convolution with V12) or
        "poisson" (neutralised 1-D Coulomb, the Wigner-Poisson system)."""
        self._check(self._L.wig2_set_hartree(self._h, self.HARTREE[form]), "wig2_set_hartree")

    def set_sweep_fusion(self, enable=True):
        """Strang: run consecutive x1 half-sweeps of a multi-step call as one
        launch (default) or as two."""
        self._check(self._L.wig2_set_sweep_fusion(self._h, int(bool(enable))), "wig2_set_sweep_fusion")

    THETA_PATHS = {"auto": 0, "general": 1, "stream": 2, "fft": 4}

    def set_theta_path(self, path: str):
        """Theta kernel choice: "auto", "general", "stream" or "fft"."""
        self._check(self._L.wig2_set_theta_path(self._h, self.THETA_PATHS[path]), "wig2_set_theta_path")

    def theta_path(self) -> str:
        """Kernel the next step uses ("general", "stream", "panel" or "fft")."""
        r = self._L.wig2_theta_path(self._h)
        if r < 0:
            self._check(r, "wig2_theta_path")
        return {1: "general", 2: "stream", 3: "panel", 4: "fft"}[r]

    def attach_surrogate(self, model, drift_tol=1e-6, exact_check_every=8):
        """Advance whole blocks with the learned pair increment (exact
        fallback when mass or energy drift by more than drift_tol)."""
        self._sur = model
        self._check(self._L.wig2_surrogate_attach(self._h, model._h, float(drift_tol),
                                                  int(exact_check_every)), "wig2_surrogate_attach")

    def detach_surrogate(self):
        self._check(self._L.wig2_surrogate_detach(self._h), "wig2_surrogate_detach")
        self._sur = None

    def surrogate_report(self):
        b, f, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        e = ctypes.c_double()
        self._check(self._L.wig2_surrogate_report(self._h, ctypes.byref(b), ctypes.byref(f),
                                                  ctypes.byref(c), ctypes.byref(e)),
                    "wig2_surrogate_report")
        return {"blocks": b.value, "fallbacks": f.value, "checks": c.value, "last_check_eps": e.value}

    def band(self):
        b = self._L.wig2_band(self._h)
        if b < 0:
            self._check(b, "wig2_band")
        return b

    def nodes(self):
        x = np.zeros(self.nx)
        p = np.zeros(self.nk)
        w = np.zeros(self.nk)
        self._check(self._L.wig2_nodes(self._h, _ptr(x), _ptr(p), _ptr(w)), "wig2_nodes")
        return x, p, w


class Batch:
    """An ensemble of uneven periodic instances advanced together."""

    def __init__(self, specs, *, precision="fp32", stream=None):
        """specs: list of dicts with nx, nk and optional x_min, x_max, hbar,
        mass, dt (Strang, torus)."""
        self._L = lib()
        n = len(specs)
        G = (Grid * n)()
        P = (Params * n)()
        self.shapes = []
        for i, sp in enumerate(specs):
            G[i] = Grid(sp["nx"], sp["nk"], 1, 1, sp.get("x_min", -10.0), sp.get("x_max", 10.0), 0.0)
            P[i] = Params(sp.get("hbar", 1.0), sp.get("mass", 1.0), sp.get("dt", 0.005), STRANG,
                          PRECISIONS[precision], 0.0, 0, 1.0, 1.0)
            self.shapes.append((sp["nx"], sp["nx"], sp["nk"], sp["nk"]))
        self.n = n
        self._cbs = {}
        h = ctypes.c_void_p()
        s = None if stream is None else ctypes.c_void_p(int(stream))
        rc = self._L.wig2_batch_create(n, G, P, s, ctypes.byref(h))
        if rc != OK:
            raise Wig2Error(rc, f"wig2_batch_create: {self._L.wig2_strerror(rc).decode()}")
        self._h = h

    def _check(self, rc, what):
        if rc != OK:
            msg = self._L.wig2_batch_last_error(self._h).decode() or self._L.wig2_strerror(rc).decode()
            raise Wig2Error(rc, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._L.wig2_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_potentials(self, i, v_ext=None, v12=None):
        cb = lambda fn: FN1(0) if fn is None else FN1(lambda x, u: float(fn(x)))
        a, b = cb(v_ext), cb(v12)
        self._cbs[i] = (a, b)
        self._check(self._L.wig2_batch_set_potentials(self._h, i, a, b, None),
                    "wig2_batch_set_potentials")

    def set_state(self, i, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == self.shapes[i]
        self._check(self._L.wig2_batch_set_state(self._h, i, _ptr(f)), "wig2_batch_set_state")

    def get_state(self, i):
        f = np.empty(self.shapes[i], dtype=np.float64)
        self._check(self._L.wig2_batch_get_state(self._h, i, _ptr(f)), "wig2_batch_get_state")
        return f

    def bind_state(self, f_dev):
        """Step a caller-owned device tensor in place (None unbinds).  The
        tensor must outlive the binding."""
        if f_dev is None:
            self._check(self._L.wig2_bind_state(self._h, None, 0), "wig2_bind_state")
            self._bound = None
            return
        assert tuple(f_dev.shape) == self.shape
        dtype = FP64 if self.precision == "fp64" else FP32
        self._check(self._L.wig2_bind_state(self._h, _dev(f_dev), dtype), "wig2_bind_state")
        self._bound = f_dev

    def step(self, n=1):
        self._check(self._L.wig2_batch_step(self._h, int(n)), "wig2_batch_step")

    def observables(self, i):
        o = Obs()
        nx, nk = self.shapes[i][0], self.shapes[i][2]
        n1, n12, f1 = np.zeros(nx), np.zeros((nx, nx)), np.zeros((nx, nk))
        self._check(self._L.wig2_batch_observables(self._h, i, ctypes.byref(o), _ptr(n1),
                                                   _ptr(n12), _ptr(f1)), "wig2_batch_observables")
        return {"mass": o.mass, "energy": o.energy, "l2": o.l2, "entropy": o.entropy_vn,
                "n1": n1, "n12": n12, "f1": f1}

    def tune(self, cache_path=None, force=False):
        p = None if cache_path is None else str(cache_path).encode()
        self._check(self._L.wig2_batch_tune(self._h, p, int(force)), "wig2_batch_tune")

    def info(self):
        tp = ctypes.c_int64()
        tg = (ctypes.c_int32 * 6)()
        ag = (ctypes.c_int32 * 6)()
        pp = (ctypes.c_int32 * 6)()
        self._check(self._L.wig2_batch_info(self._h, ctypes.byref(tp), tg, ag, pp),
                    "wig2_batch_info")
        cls = (16, 32, 48, 64, 96, 128)
        return {"points": tp.value, "theta_grid": dict(zip(cls, list(tg))),
                "advect_grid": dict(zip(cls, list(ag))), "planes_per_group": dict(zip(cls, list(pp)))}


class Surrogate:
    """Learned pair-increment model (wig2_surrogate_*): a 4-D separable
    convolutional network (16 channels; `blocks` blocks of p1, p2, x1, x2
    convolutions with k_p / k_x taps).  Create, collect / train on a
    Solver's exact trajectory or on a Batch, attach to a Solver."""

    def __init__(self, *, blocks=9, k_p=35, k_x=7, block=8, epochs=2, lr=1e-3, seed=0, train_blocks=1,
                 max_points=0, _handle=None):
        self._L = lib()
        self.cfg = TrainCfg(16, blocks, k_p, k_x, block, epochs, lr, seed, train_blocks, max_points)
        if _handle is None:
            h = ctypes.c_void_p()
            rc = self._L.wig2_surrogate_create(ctypes.byref(self.cfg), ctypes.byref(h))
            if rc != OK:
                raise Wig2Error(rc, f"wig2_surrogate_create: {self._L.wig2_strerror(rc).decode()}")
            self._h = h
        else:
            self._h = _handle
        n, nl = ctypes.c_int64(), ctypes.c_int32()
        self._check(self._L.wig2_surrogate_size(self._h, ctypes.byref(n), ctypes.byref(nl)), "wig2_surrogate_size")
        self.nparams, self.nlayers = n.value, nl.value

    @classmethod
    def train_on_batch(cls, batch, **cfg):
        """wig2_surrogate_train: a new model trained on the instances of a Batch."""
        tmp = cls.__new__(cls)
        tmp._L = lib()
        c = dict(blocks=9, k_p=35, k_x=7, block=8, epochs=2, lr=1e-3, seed=0, train_blocks=1, max_points=0)
        c.update(cfg)
        tc = TrainCfg(16, c["blocks"], c["k_p"], c["k_x"], c["block"], c["epochs"], c["lr"], c["seed"],
                      c["train_blocks"], c["max_points"])
        h = ctypes.c_void_p()
        rc = tmp._L.wig2_surrogate_train(batch._h, ctypes.byref(tc), ctypes.byref(h))
        if rc != OK:
            raise Wig2Error(rc, f"wig2_surrogate_train: {tmp._L.wig2_strerror(rc).decode()}")
        return cls(_handle=h, **c)

    def _check(self, rc, what):
        if rc != OK:
            msg = self._L.wig2_surrogate_last_error(self._h).decode() or self._L.wig2_strerror(rc).decode()
            raise Wig2Error(rc, f"{what}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._L.wig2_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def collect(self, solver, blocks=1, train=True):
        self._check(self._L.wig2_surrogate_collect(self._h, solver._h, int(blocks), int(train)),
                    "wig2_surrogate_collect")

    def stats(self):
        tl, el = ctypes.c_double(), ctypes.c_double()
        up, sm = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._L.wig2_surrogate_stats(self._h, ctypes.byref(tl), ctypes.byref(el),
                                                 ctypes.byref(up), ctypes.byref(sm)), "wig2_surrogate_stats")
        return {"train_loss": tl.value, "eval_loss": el.value, "updates": up.value, "samples": sm.value}

    def get_params(self):
        p = np.zeros(self.nparams, dtype=np.float32)
        sc = np.zeros(3, dtype=np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        self._check(self._L.wig2_surrogate_get_params(self._h, p.ctypes.data_as(fp), sc.ctypes.data_as(fp)),
                    "wig2_surrogate_get_params")
        return p, sc

    def set_params(self, params=None, scales=None):
        fp = ctypes.POINTER(ctypes.c_float)
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if p is not None:
            assert p.size == self.nparams
        sc = None if scales is None else np.ascontiguousarray(scales, dtype=np.float32)
        self._check(self._L.wig2_surrogate_set_params(self._h, None if p is None else p.ctypes.data_as(fp),
                                                      None if sc is None else sc.ctypes.data_as(fp)),
                    "wig2_surrogate_set_params")

    def grad(self, solver, ft_dev, delta_dev):
        """Gradient of the mean squared error over all points (device fields)."""
        g = np.zeros(self.nparams, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(self._L.wig2_surrogate_grad(self._h, solver._h, _dev(ft_dev), _dev(delta_dev),
                                                g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                ctypes.byref(loss)), "wig2_surrogate_grad")
        return g, loss.value
