"""CPU-side checks of the C ABI: the built library loads, exports every entry
point that include/wig2.h declares, and rejects invalid arguments before any
device work (these calls never reach a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2511_11354_amd import wig2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "wig2.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wig2_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("wig2_create", "wig2_set_potentials", "wig2_step", "wig2_observables",
              "wig2_destroy", "wig2_theta", "wig2_advect"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(wig2.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding's table covers the same set
    assert set(wig2.SIGNATURES) == set(_declared())


def test_strerror_codes():
    L = wig2.lib()
    for code in (wig2.OK, wig2.EINVAL, wig2.ENOMEM, wig2.EDEVICE, wig2.ESTATE, wig2.ENOTSUP,
                 wig2.ENUMERIC):
        assert L.wig2_strerror(code)
    assert L.wig2_last_error(None) == b"null context"


@pytest.mark.parametrize("grid,params,code", [
    (dict(nx=2, nk=32), {}, wig2.EINVAL),                      # too few x points
    (dict(nx=16, nk=32, x_min=1.0, x_max=1.0), {}, wig2.EINVAL),  # empty box
    (dict(nx=16, nk=32), dict(hbar=0.0), wig2.EINVAL),
    (dict(nx=16, nk=32), dict(mass=-1.0), wig2.EINVAL),
    (dict(nx=16, nk=32), dict(dt=float("nan")), wig2.EINVAL),
    (dict(nx=16, nk=32), dict(scheme=7), wig2.EINVAL),
    (dict(nx=16, nk=32), dict(precision=9), wig2.EINVAL),
    (dict(nx=16, nk=33, periodic=0, sem_cells=4, k_max=3.0), {}, wig2.EINVAL),  # nk % cells
    (dict(nx=16, nk=32, periodic=0, sem_cells=4, k_max=0.0), {}, wig2.EINVAL),
    (dict(nx=16, nk=40), {}, wig2.ENOTSUP),                    # not a Theta tile size
    (dict(nx=16, nk=48), dict(precision=wig2.BF16X2), wig2.ENOTSUP),
    (dict(nx=16, nk=32, periodic=0, sem_cells=4, k_max=3.0), dict(precision=wig2.BF16X2),
     wig2.ENOTSUP),                                            # BF16X2 box needs the panel size
])
def test_create_rejects_before_device_work(grid, params, code):
    L = wig2.lib()
    g = dict(nx=16, nk=32, periodic=1, sem_cells=1, x_min=-10.0, x_max=10.0, k_max=0.0)
    g.update(grid)
    p = dict(hbar=1.0, mass=1.0, dt=0.01, scheme=0, precision=0, meanfield_lambda=0.0, xc=0,
             xc_n0=1.0, n_scale=1.0)
    p.update(params)
    G = wig2.Grid(**g)
    P = wig2.Params(**p)
    h = ctypes.c_void_p()
    assert L.wig2_create(ctypes.byref(G), ctypes.byref(P), None, ctypes.byref(h)) == code
    assert not h.value


def test_null_arguments():
    L = wig2.lib()
    h = ctypes.c_void_p()
    assert L.wig2_create(None, None, None, ctypes.byref(h)) == wig2.EINVAL
    assert L.wig2_step(None, 1) == wig2.EINVAL
    assert L.wig2_set_state(None, None) == wig2.EINVAL
    L.wig2_destroy(None)


def _enum(prefix):
    txt = open(os.path.join(ROOT, "include", "wig2.h")).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(rf"\b({prefix}[A-Z0-9_]+)\s*=\s*(\d+)", txt)}


def test_binding_tables_match_header_enums():
    """The binding's Theta-path names and profile classes carry the values
    include/wig2.h assigns (the binding holds no values of its own)."""
    paths = _enum("WIG2_THETA_")
    assert wig2.Solver.THETA_PATHS == {"auto": paths["WIG2_THETA_AUTO"], "general": paths["WIG2_THETA_GENERAL"],
                                       "stream": paths["WIG2_THETA_STREAM"], "fft": paths["WIG2_THETA_FFT"]}
    assert paths["WIG2_THETA_PANEL"] not in wig2.Solver.THETA_PATHS.values()  # reported, never chosen
    prof = _enum("WIG2_PROF_")
    n = prof.pop("WIG2_PROF_N")
    assert len(wig2.PROF_NAMES) == n
    for name, i in prof.items():
        assert wig2.PROF_NAMES[i] == name[len("WIG2_PROF_"):].lower()
