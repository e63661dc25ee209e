"""Benchmark: 4-D phase-space point-updates/s of the two-body Wigner step.

Default workload: periodic box L = 20, 128^4 points, V_ext = 0.5 cos(2 pi x/L),
V12 = 1/sqrt(r^2 + 1), seeded Gaussian-mixture state (seed 0), dt = 0.005,
Strang step (A/2, Heun on Theta, A/2), FP64.  One JSON line on stdout.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|fp32|bf16x2]
                    [--workload large|tiny|box|ensemble|surrogate|accuracy]
                    [--scheme strang|lawson] [--no-cpu]

A "step" is one full time step over the whole grid (2 Theta applications and
4 advection sweeps).  The state is resident in HBM before timing starts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "4-D phase-space point-updates/s (FP64 vs mixed/surrogate) at stated err"
PEAK = {"hbm_gbs": 8000.0, "fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}  # MI355X, TFLOP/s dense
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x2": "bf16x2(f32 acc)"}


def theta_flops_per_point(nk: int, band: int) -> float:
    """Algorithmic flops of one Theta application per grid point: every
    non-zero multiply-add of the single-body products (band modes each side,
    off the box excluded) and of the pair term along anti-diagonals."""
    m1 = 2.0 * band - band * (band + 1) / nk          # MACs per point, one particle
    lens = [min(s + 1, 2 * nk - 1 - s) for s in range(2 * nk - 1)]
    m12 = sum(l * (l - 1) for l in lens) / (nk * nk)   # MACs per point, pair term
    return 2.0 * (2.0 * m1 + m12)


def fft_flops_per_point(nk):
    """Theta by 2-D FFT convolution of a plane zero-padded to N = 2 nk: nk/2
    forward and nk/2 inverse row transforms (two real rows per complex
    transform), a forward and an inverse transform for each of the N/2 + 1
    column frequencies, 5 N log2 N flops per complex transform of length N,
    and the multiply by the purely imaginary symbol (2 flops per complex
    value), per plane point."""
    n = 2 * nk
    per_plane = (nk + 2 * (n // 2 + 1)) * 5.0 * n * math.log2(n) + (n // 2 + 1) * 2.0 * n
    return per_plane / (nk * nk)


def kernel_model(name, npts, elem, nk, band, precision, dense=False, pair=False, fft=False):
    """Algorithmic (bytes, flops) of one launch of a kernel class.  dense: the
    box's SEM operator, two dense nk x nk products per plane (4 nk flops/pt);
    pair: the box's two-body SEM operator, four products per plane through
    the y-lattice (24 nk flops/pt), part of every Theta application; fft:
    Theta by the FFT convolution (fft_flops_per_point)."""
    if name == "advect_x1x1":
        return 2 * elem * npts, 40.0 * npts  # two sweeps, one read and one write
    if name.startswith("advect"):
        return 2 * elem * npts, 20.0 * npts
    if name == "pair_sem":
        return 3 * elem * npts, 24.0 * nk * npts  # read x, read and write out
    if name == "meanfield" and dense:
        # plane integrals of the state, then both particles' SEM matrices:
        # nx^2 nk^2 = npts terms of 7 flops (Im(E Q), two multiply-adds)
        return elem * npts, 4.0 * npts + 7.0 * npts
    fl = (4.0 * nk if dense else theta_flops_per_point(nk, band)) * npts
    if fft:
        fl = fft_flops_per_point(nk) * npts
    if pair:
        fl += 24.0 * nk * npts
    if name == "theta_stage1":
        return 2 * elem * npts, fl          # read f, write Theta f
    if name == "theta_stage2":
        return 3 * elem * npts, fl + 4 * npts  # read the two states, write the Heun result
    if name == "theta_heun":
        return 2 * elem * npts, 2 * fl + 6 * npts  # both Heun stages: read f, write f+
    return elem * npts, 4.0 * npts


def source_digest(*rel):
    h = hashlib.sha256()
    for r in rel:
        with open(os.path.join(ROOT, r), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_file, kernel_class, workload, precision):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), valid
    only while the kernel source is unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        key = f"{kernel_class}/{workload}/{precision}"
        e = rec.get(key)
        if not e or e.get("source_sha") != source_digest(kernel_file):
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, f0, budget_s=20.0, gpu_theta=None, gpu_advect=None):
    """The CPU oracle timed on a bounded sample of the same workload: Theta on
    a set of x-pair planes and spline sweeps on a set of lines, scaled to one
    whole step (2 Theta + 4 sweeps) per grid point."""
    import numpy as np

    import oracle

    g = oracle.grid(w.nx, w.nk, True, 1, w.x_min, w.x_max)
    tb = oracle.tables(g, w.vext, w.v12)
    nplanes_all = w.nx * w.nx
    nlines_all = w.nx * w.nk * w.nk

    def timed(fn, start, count):
        t0 = time.perf_counter()
        fn(start, count)
        return time.perf_counter() - t0

    # one output array for every call, allocated and paged in before any
    # timing: a full-grid allocation per sampled call would be charged to a
    # few planes and then scaled up to the whole grid
    out = np.ones_like(f0)
    th = lambda p0, n: oracle.theta_periodic(g, tb["sig_ext"], tb["sig_ext"], tb["vhat12"], f0, True,
                                             p0, n, out=out)
    sw = lambda l0, n: (oracle.advect(g, 1, 0.5 * w.dt, f0, l0, n, out=out),
                        oracle.advect(g, 2, 0.5 * w.dt, f0, l0, n, out=out))
    # a pilot run sizes the sample so that it takes about budget_s in all:
    # half on Theta planes, half on sweep lines (both directions)
    # (the pilot takes at least two planes per oracle thread: fewer planes
    # than threads would time a partly idle pool and undersize the sample)
    p0 = min(nplanes_all, max(4, 2 * oracle.num_threads()))
    per_plane = timed(th, 0, p0) / p0
    l0 = min(nlines_all, w.nk * w.nk)
    per_line = timed(sw, 0, l0) / l0
    npl = max(1, min(nplanes_all - p0, int(0.5 * budget_s / per_plane)))
    nli = max(1, min(nlines_all - l0, int(0.5 * budget_s / per_line)))
    s_theta = timed(th, p0, npl)
    err = None
    if gpu_theta is not None:
        # the GPU path's Theta of the same state against the oracle's on the
        # sampled planes (written by the timed call)
        sl = slice(p0 * w.nk * w.nk, (p0 + npl) * w.nk * w.nk)
        r, o = out.reshape(-1)[sl], gpu_theta.reshape(-1)[sl]
        err = {"eps_inf_theta": float(np.abs(o - r).max() / np.abs(r).max()),
               "theta_planes": [p0, p0 + npl - 1]}
    s_sweep = timed(sw, l0, nli)
    t_theta = s_theta / npl * nplanes_all
    t_sweep = s_sweep / (2 * nli) * nlines_all
    t_step = 2 * t_theta + 4 * t_sweep
    if gpu_advect is not None:
        # the GPU path's x1 half-step sweep against the oracle's on a run of
        # lines through the packets (untimed)
        nli_e = min(nlines_all, 8 * w.nk * w.nk)
        le = (w.nx // 2) * w.nk * w.nk - nli_e // 2
        oracle.advect(g, 1, 0.5 * w.dt, f0, le, nli_e, out=out)
        nk2 = w.nk * w.nk
        lines = np.arange(le, le + nli_e)
        o_, rem = lines // nk2, lines % nk2
        idx = (o_ * nk2 + rem)[:, None] + np.arange(w.nx)[None, :] * w.nx * nk2
        r, o = out.reshape(-1)[idx], gpu_advect.reshape(-1)[idx]
        err = dict(err or {}, eps_inf_advect_x1=float(np.abs(o - r).max() / np.abs(r).max()),
                   advect_lines=[int(le), int(le + nli_e - 1)])
    return {"value": w.points / t_step, "unit": "point-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": (f"FP64 oracle on {npl} of {nplanes_all} x-pair planes (Theta) and "
                       f"{nli} of {nlines_all} lines per sweep direction, scaled to one step "
                       f"of 2 Theta + 4 sweeps"),
            "sample_s": s_theta + s_sweep, "s_per_step_extrapolated": t_step, "error_vs_oracle": err}


def bench_surrogate(a):
    """Learned pair-increment surrogate at the periodic 128^4 shape (FP32):
    trained through wig2_surrogate_train on a batch of ensemble instances
    (seeds 1000+, those of at most 48^2 x 64^2 points), then the same number
    of blocks from the mixture state (seed 0) advanced exactly and with the
    surrogate attached (drift tolerance 1e-6, exact check every 8 blocks),
    and with the surrogate alone (no monitor, no checks); both rates, the
    fallbacks and the final eps_inf against the exact run are reported."""
    import numpy as np
    import torch

    from paper_2511_11354_amd import inputs as I
    from paper_2511_11354_amd import wig2

    prec = a.precision or "fp32"
    B = 8
    ens = I.ensemble()
    pick = [i for i, w in enumerate(ens) if w.points <= 48 * 48 * 64 * 64][:6]
    b = wig2.Batch([dict(nx=ens[i].nx, nk=ens[i].nk, dt=ens[i].dt) for i in pick], precision=prec)
    for j, i in enumerate(pick):
        w = ens[i]
        b.set_potentials(j, w.vext, w.v12)
        s = wig2.Solver(w.nx, w.nk, dt=w.dt, precision=prec)
        x, p, _ = s.nodes()
        b.set_state(j, I.mixture(x, p, seed=w.extra["seed"], period=20.0))
        s.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    model = wig2.Surrogate.train_on_batch(b, block=B, epochs=8, lr=2e-3, seed=0, train_blocks=2)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    st = model.stats()
    b.close()

    w = I.large_periodic(u=1.0)
    runs = {}
    nblocks = max(1, a.steps // B)
    f0 = None
    for mode in ("exact", "surrogate", "unchecked"):
        s = wig2.Solver(w.nx, w.nk, dt=w.dt, precision=prec)
        s.set_potentials(w.vext, w.v12)
        if f0 is None:
            x, p, _ = s.nodes()
            f0 = I.mixture(x, p, seed=0, period=20.0)
        s.set_state(f0)
        s.step(B)  # warm-up block (exact)
        if mode == "surrogate":
            s.attach_surrogate(model, drift_tol=1e-6, exact_check_every=8)
        elif mode == "unchecked":
            s.attach_surrogate(model, drift_tol=1e30, exact_check_every=0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.step(nblocks * B)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        runs[mode] = {"state": s.get_state(), "seconds": dt, "value": w.points * nblocks * B / dt,
                      "report": s.surrogate_report() if mode != "exact" else None}
        s.close()
        del s
        torch.cuda.synchronize()
    fe = runs["exact"]["state"]
    eps = float(np.abs(runs["surrogate"]["state"] - fe).max() / np.abs(fe).max())
    eps_u = float(np.abs(runs["unchecked"]["state"] - fe).max() / np.abs(fe).max())
    # the method without what the surrogate supplies: the same steps with no
    # pair term, against the exact run
    s = wig2.Solver(w.nx, w.nk, dt=w.dt, precision=prec)
    s.set_potentials(w.vext, None)
    s.set_state(f0)
    s.step(B + nblocks * B)
    eps_nov = float(np.abs(s.get_state() - fe).max() / np.abs(fe).max())
    s.close()
    out = {
        "metric": METRIC, "value": runs["surrogate"]["value"], "unit": "point-updates/s", "n_gpus": 1,
        "steps": nblocks * B, "warmup": B, "ms_per_step": runs["surrogate"]["seconds"] / (nblocks * B) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": w.name + "-surrogate", "nx": w.nx, "nk": w.nk, "points": w.points,
                   "dt": w.dt, "block": B, "drift_tol": 1e-6, "exact_check_every": 8,
                   "model": {"params": model.nparams, "conv_layers": model.nlayers, "channels": 16,
                             "blocks": 9, "k_p": 35, "k_x": 7},
                   "train_instances": [ens[i].name for i in pick], "seed": 0},
        "exact": {"value": runs["exact"]["value"],
                  "ms_per_step": runs["exact"]["seconds"] / (nblocks * B) * 1e3},
        "speedup_vs_exact": runs["exact"]["seconds"] / runs["surrogate"]["seconds"],
        "unchecked": {"value": runs["unchecked"]["value"],
                      "ms_per_step": runs["unchecked"]["seconds"] / (nblocks * B) * 1e3,
                      "speedup_vs_exact": runs["exact"]["seconds"] / runs["unchecked"]["seconds"],
                      "eps_inf_vs_exact": eps_u, **runs["unchecked"]["report"]},
        "surrogate": dict(runs["surrogate"]["report"], eps_inf_vs_exact=eps, eps_inf_without_pair_term=eps_nov,
                          train_seconds=t_train, **st),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def bench_accuracy(a):
    """The reduced-precision forms against the FP64 GPU path on the periodic
    128^4 workload (mixture seed 0): every form advances the same initial
    state by the same steps; at checkpoints the one-particle density n1 and
    the pair density n12 (FP64 reductions) are compared with FP64's, as
    max|n - n_fp64| / max|n_fp64|, the state itself as eps_inf =
    max|f - f_fp64| / max|f_fp64| and eps_2 = rms(f - f_fp64) / max|f_fp64|,
    and the mass and energy drift are recorded.  Rates are timed between
    checkpoints (observables and state copies excluded)."""
    import numpy as np
    import torch

    from paper_2511_11354_amd import inputs as I
    from paper_2511_11354_amd import wig2

    w = I.large_periodic(u=1.0)
    nsteps = a.steps
    marks = sorted({m for m in (1, 10, 100, nsteps) if m <= nsteps})
    f0 = None
    ref = {}
    fref = {}
    forms = {}

    def state_errors(f, r):
        # chunked over x1 slabs: eps_inf and eps_2 against the FP64 state
        mx = num = 0.0
        dmax = 0.0
        for i in range(f.shape[0]):
            d = f[i] - r[i]
            dmax = max(dmax, float(np.abs(d).max()))
            num += float(np.sum(d * d))
            mx = max(mx, float(np.abs(r[i]).max()))
        return dmax / mx, math.sqrt(num / f.size) / mx
    for prec in ("fp64", "fp32", "bf16x2"):
        s = wig2.Solver(w.nx, w.nk, x_min=w.x_min, x_max=w.x_max, dt=w.dt, precision=prec)
        s.set_potentials(w.vext, w.v12)
        if f0 is None:
            x, p, _ = s.nodes()
            f0 = I.mixture(x, p, seed=0, period=w.x_max - w.x_min)
        s.set_state(f0)
        ob0 = s.observables()
        done, secs, rows = 0, 0.0, []
        for m in marks:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(m - done)
            torch.cuda.synchronize()
            secs += time.perf_counter() - t0
            done = m
            ob = s.observables()
            row = {"step": m, "mass_drift": abs(ob["mass"] - ob0["mass"]) / abs(ob0["mass"]),
                   "energy_drift": abs(ob["energy"] - ob0["energy"]) / abs(ob0["energy"])}
            if prec == "fp64":
                ref[m] = (ob["n1"].copy(), ob["n12"].copy(), ob["mass"], ob["energy"])
                fref[m] = s.get_state()
            else:
                row["eps_inf"], row["eps_2"] = state_errors(s.get_state(), fref[m])
                n1r, n12r, mr, er = ref[m]
                row["err_n1"] = float(np.abs(ob["n1"] - n1r).max() / np.abs(n1r).max())
                row["err_n12"] = float(np.abs(ob["n12"] - n12r).max() / np.abs(n12r).max())
                row["err_mass"] = abs(ob["mass"] - mr) / abs(mr)
                row["err_energy"] = abs(ob["energy"] - er) / abs(er)
            rows.append(row)
            print(f"accuracy: {prec} step {m} {row}", file=sys.stderr, flush=True)
        forms[prec] = {"value": w.points * nsteps / secs, "ms_per_step": secs / nsteps * 1e3,
                       "theta_kernel": s.theta_path(), "checkpoints": rows}
        s.close()
        del s
        torch.cuda.synchronize()
    out = {
        "metric": METRIC, "value": forms["fp64"]["value"], "unit": "point-updates/s", "n_gpus": 1,
        "steps": nsteps, "warmup": 0, "ms_per_step": forms["fp64"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE["fp64"],
        "data": "synthetic",
        "config": {"workload": w.name + "-accuracy", "nx": w.nx, "nk": w.nk, "points": w.points,
                   "dt": w.dt, "scheme": "strang", "V12_U": 1.0, "seed": 0,
                   "error": "max-abs difference / max-abs FP64 value, per checkpoint"},
        "forms": forms, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def bench_ensemble(a):
    """64 uneven periodic instances (seeds 1000..1063): one batched step of
    the whole ensemble per 'step', FP32, against a loop over 64 single
    contexts doing the same steps."""
    import torch

    from paper_2511_11354_amd import inputs as I
    from paper_2511_11354_amd import wig2

    prec = a.precision if a.precision != "bf16x2" else "fp32"
    ens = I.ensemble()
    specs = [dict(nx=w.nx, nk=w.nk, dt=w.dt) for w in ens]
    b = wig2.Batch(specs, precision=prec)
    singles, shared = [], []
    one = torch.cuda.Stream()
    for i, w in enumerate(ens):
        b.set_potentials(i, w.vext, w.v12)
        s = wig2.Solver(w.nx, w.nk, dt=w.dt, precision=prec)
        s.set_potentials(w.vext, w.v12)
        x, p, _ = s.nodes()
        f0 = I.mixture(x, p, seed=w.extra["seed"], period=w.x_max - w.x_min)
        b.set_state(i, f0)
        s.set_state(f0)
        singles.append(s)
        s1 = wig2.Solver(w.nx, w.nk, dt=w.dt, precision=prec, stream=one.cuda_stream)
        s1.set_potentials(w.vext, w.v12)
        s1.set_state(f0)
        shared.append(s1)
    t0 = time.perf_counter()
    b.tune(a.tune_cache)
    t_tune = time.perf_counter() - t0
    total = sum(w.points for w in ens)
    b.step(max(1, a.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(a.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for s in singles:
        s.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        for s in singles:
            s.step(1)
    torch.cuda.synchronize()
    dt_loop = time.perf_counter() - t0
    for s in shared:
        s.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        for s in shared:
            s.step(1)
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    sizes = {}
    for w in ens:
        sizes[f"{w.nx}x{w.nk}"] = sizes.get(f"{w.nx}x{w.nk}", 0) + 1
    out = {
        "metric": METRIC, "value": total * a.steps / dt, "unit": "point-updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": "ensemble-64-uneven", "instances": len(ens), "points": total,
                   "sizes_nx_x_nk": sizes, "precision": prec, "dt": 0.005, "scheme": "strang"},
        "loop_of_single_contexts": {"value": total * a.steps / dt_loop,
                                    "ms_per_step": dt_loop / a.steps * 1e3,
                                    "note": "one stream per context (runs concurrently)"},
        "loop_on_one_stream": {"value": total * a.steps / dt_seq,
                               "ms_per_step": dt_seq / a.steps * 1e3},
        "speedup_vs_loop": dt_loop / dt,
        "speedup_vs_one_stream_loop": dt_seq / dt,
        "tuning": dict(b.info(), seconds=t_tune),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "bf16x2"],
                    help="default: fp64 for the single-grid workloads, fp32 for the ensemble")
    ap.add_argument("--scheme", default="strang", choices=["strang", "lawson"])
    ap.add_argument("--workload", default="large",
                    choices=["large", "tiny", "ensemble", "box", "box-pair", "box-meanfield", "landau",
                             "two-stream", "surrogate", "accuracy"],
                    help="large: periodic 128^4 (default); tiny: periodic 32^4; ensemble: 64 "
                         "uneven periodic instances; box: 129^2 x 256^2 SEM box; box-pair: the "
                         "same box with the smoothed Coulomb pair potential (two-body SEM "
                         "operator), FP64 by default; box-meanfield: box-pair with the "
                         "Hartree mean field lambda = 1 (SEM matrices of V_ext + V_eff "
                         "rebuilt per Theta sub-step); landau, two-stream: the Wigner-Poisson "
                         "workloads of Sec. 5 at 256^2 x 128^2 (neutralised Poisson Hartree, "
                         "pair potential 1/sqrt(r^2 + 1)), FP64; surrogate: "
                         "128^4 FP32 with the learned pair increment; accuracy: FP32 and "
                         "split-BF16 against FP64 at 128^4 over --steps steps")
    ap.add_argument("--potential", default="harmonic", choices=["harmonic", "double_well"],
                    help="V_ext of the box workload")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "gpurun_out", "tune_cache.json"),
                    help="autotuner cache for the ensemble workload (runtime output, untracked)")
    ap.add_argument("--forms", default="fp32,bf16x2,hartree,fft",
                    help="extra legs of the default 128^4 line, comma separated: fp32, bf16x2 "
                         "(same workload and steps, errors against the FP64 run's final state), "
                         "hartree (FP64 with the mean field lambda = 1) and fft (FP64, Theta by "
                         "the FFT convolution instead of the direct products); empty for none")
    ap.add_argument("--theta-path", default="auto", choices=["auto", "general", "stream", "fft"],
                    help="Theta kernel of the main leg (torus workloads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain device copies of the state size (for counter scaling)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU slab "
              "decomposition is a design, not implemented here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2511_11354_amd import inputs as I
    from paper_2511_11354_amd import wig2

    torch.cuda.set_device(0)
    if a.workload == "ensemble":
        a.precision = a.precision or "fp32"
        os.makedirs(os.path.dirname(os.path.abspath(a.tune_cache)), exist_ok=True)
        return bench_ensemble(a)
    if a.workload == "surrogate":
        return bench_surrogate(a)
    if a.workload == "accuracy":
        return bench_accuracy(a)
    box = a.workload in ("box", "box-pair", "box-meanfield")
    a.precision = a.precision or ("fp32" if a.workload == "box" else "fp64")
    if box:
        w = I.box_sem(129, 16, 16, a.potential, pair_u=None if a.workload == "box" else 1.0)
    elif a.workload in ("landau", "two-stream"):
        w = I.plasma(a.workload, 256, 128)
    else:
        w = I.large_periodic(u=1.0) if a.workload == "large" else I.tiny_periodic()
    probe = make_solver(w, box, a.scheme, "fp64")
    x, p, _ = probe.nodes()
    probe.close()
    if a.workload == "large":
        f0 = I.mixture(x, p, seed=0, period=w.x_max - w.x_min)
    elif a.workload in ("landau", "two-stream"):
        f0 = I.plasma_state(x, p, w.extra["kind"], w.extra["eps"], w.extra["k"])
    elif box:
        f0 = I.symmetrised_pair(x, p, a=(-2.0, 2.0), q=(0.0, 0.0))
    else:
        f0 = I.symmetrised_pair(x, p)

    forms = [f for f in a.forms.split(",") if f] if (a.workload == "large" and a.precision == "fp64") else []
    main_leg = run_form(w, f0, box, a.scheme, a.precision, a.steps, a.warmup,
                        lam=1.0 if a.workload == "box-meanfield" else 0.0, keep_state=bool(forms),
                        theta_path=None if box or a.theta_path == "auto" else a.theta_path,
                        copy_calibration=a.copy_calibration,
                        gpu_samples=not a.no_cpu and a.workload == "large" and a.precision == "fp64")
    cpu = None
    if not a.no_cpu and a.workload == "large" and a.precision == "fp64":
        cpu = cpu_baseline(w, f0, gpu_theta=main_leg.pop("gpu_theta"), gpu_advect=main_leg.pop("gpu_advect"))
    main_leg.pop("gpu_theta", None)
    main_leg.pop("gpu_advect", None)
    ref_state = main_leg.pop("state", None)
    ref_obs = main_leg.pop("obs")
    legs = {}
    for form in forms:
        prec, lam = ("fp64", 1.0) if form == "hartree" else ("fp64", 0.0) if form == "fft" else (form, 0.0)
        leg = run_form(w, f0, box, a.scheme, prec, a.steps, a.warmup, lam=lam, keep_state=lam == 0.0,
                       theta_path="fft" if form == "fft" else None)
        ob = leg.pop("obs")
        st = leg.pop("state", None)
        if st is not None:
            e_inf, e_2 = state_errors(st, ref_state)
            leg["error_vs_fp64"] = {
                "eps_inf": e_inf, "eps_2": e_2,
                "n1": rel_max(ob["n1"], ref_obs["n1"]), "n12": rel_max(ob["n12"], ref_obs["n12"]),
                "mass": abs(ob["mass"] - ref_obs["mass"]) / abs(ref_obs["mass"]),
                "after_steps": a.warmup + a.steps,
                "definition": "max|x - x_fp64| / max|x_fp64| (eps_2: rms); the FP64 leg's final state"}
        else:
            leg["note"] = ("Hartree mean field lambda = 1 rebuilt from the density each Theta "
                           "sub-step: dense single-body band, general Theta kernel")
        del st
        legs[form] = leg
    out = {
        "metric": METRIC, "value": main_leg["value"], "unit": "point-updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[a.precision], "data": "synthetic",
        "config": {"workload": w.name + ("-meanfield" if a.workload == "box-meanfield" else ""), "nx": w.nx, "nk": w.nk, "points": w.points, "dt": w.dt,
                   "scheme": a.scheme, "precision": a.precision, "V12_U": w.extra.get("U", 1.0),
                   "single_body_band": main_leg["band"], "theta_kernel": main_leg["theta_kernel"],
                   "seed": 0},
        "error": ({"vs": "FP64 CPU oracle", **cpu["error_vs_oracle"]} if cpu and cpu.get("error_vs_oracle")
                  else None),
        "roofline": main_leg["roofline"], "cpu_baseline": cpu, "kernels": main_leg["kernels"],
        "observables": {k: ref_obs[k] for k in ("mass", "energy", "entropy", "step")},
        "forms": legs,
    }
    print(json.dumps(out))


def make_solver(w, box, scheme, precision, lam=0.0):
    from paper_2511_11354_amd import wig2

    if box:
        return wig2.Solver(w.nx, w.nk, periodic=False, sem_cells=w.cells, x_min=w.x_min,
                           x_max=w.x_max, k_max=w.k_max, dt=w.dt, scheme=scheme, precision=precision,
                           meanfield_lambda=lam)
    if "hartree" in w.extra:  # the plasma workloads: their own mean field
        s = wig2.Solver(w.nx, w.nk, x_min=w.x_min, x_max=w.x_max, dt=w.dt, scheme=scheme,
                        precision=precision, meanfield_lambda=w.extra["lam"])
        s.set_hartree(w.extra["hartree"])
        return s
    return wig2.Solver(w.nx, w.nk, x_min=w.x_min, x_max=w.x_max, dt=w.dt, scheme=scheme,
                       precision=precision, meanfield_lambda=lam)


def rel_max(a, b):
    import numpy as np

    return float(np.abs(a - b).max() / np.abs(b).max())


def state_errors(f, r):
    """eps_inf and eps_2 of f against r, one x1 slab at a time."""
    import numpy as np

    mx = num = dmax = 0.0
    for i in range(f.shape[0]):
        d = f[i] - r[i]
        dmax = max(dmax, float(np.abs(d).max()))
        num += float(np.sum(d * d))
        mx = max(mx, float(np.abs(r[i]).max()))
    return dmax / mx, math.sqrt(num / f.size) / mx


def run_form(w, f0, box, scheme, precision, steps, warmup, lam=0.0, keep_state=False,
             copy_calibration=False, gpu_samples=False, theta_path=None):
    """One form of the workload: warm-up, then `steps` timed steps with the
    per-kernel-class HIP event timing on the context stream."""
    import torch

    s = make_solver(w, box, scheme, precision, lam)
    s.set_potentials(w.vext, w.v12)
    if theta_path:
        s.set_theta_path(theta_path)
    s.set_state(f0)
    band = s.band()
    res = {}
    if gpu_samples:
        # the FP64 path's Theta and x1 sweep of the initial state, checked
        # against the oracle on the CPU-baseline sample
        fin = torch.from_numpy(f0).cuda()
        out = torch.empty_like(fin)
        s.theta(fin, out)
        res["gpu_theta"] = out.cpu().numpy()
        s.advect(1, 0.5 * w.dt, fin, out)
        res["gpu_advect"] = out.cpu().numpy()
        del fin, out
    s.step(warmup)
    torch.cuda.synchronize()
    s.profile(True)
    s.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = s.profile_read(reset=True)
    s.profile(False)
    ob = s.observables()
    if copy_calibration:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE
        # counters calibrate the byte counts read for the method's kernels
        src = torch.empty(w.points * (8 if precision == "fp64" else 4), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    npts = w.points
    elem = 8 if precision == "fp64" else 4
    dense_band = w.nk - 1 if (lam != 0.0 or "hartree" in w.extra) else band
    pair = box and w.v12 is not None
    path = s.theta_path()
    fft = path == "fft"
    kernels = {}
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        by, fl = kernel_model(name, npts, elem, w.nk, dense_band, precision, dense=box, pair=pair, fft=fft)
        avg = ms / cnt / 1e3
        kernels[name] = {"avg_ms": ms / cnt, "launches": cnt, "GB/s": by / avg / 1e9,
                         "TFLOP/s": fl / avg / 1e12}
    # the box's pair operator (nested inside the Theta stages) is the hot
    # kernel class whenever it runs
    dom = "pair_sem" if prof.get("pair_sem", (0, 0))[1] else max(prof, key=lambda k: prof[k][0])
    ms, cnt = prof[dom]
    by, fl = kernel_model(dom, npts, elem, w.nk, dense_band, precision, dense=box, pair=pair, fft=fft)
    avg = ms / cnt / 1e3
    pk_fl = PEAK["fp64" if precision == "fp64" else ("fp32" if precision == "fp32" else "bf16")]
    t_hbm = by / (PEAK["hbm_gbs"] * 1e9)
    t_fl = fl / (pk_fl * 1e12)
    if fft and dom.startswith("theta"):
        # the transforms run on the vector ALUs; FP64 / FP32 vector peaks
        # equal the dense matrix peaks used above (78.6 / 157.3 TFLOP/s)
        roof = {"bound": "alu", "achieved": fl / avg / 1e12, "peak": pk_fl, "unit": "TFLOP/s"}
    elif (dom.startswith("theta") or dom == "pair_sem") and t_fl > t_hbm:
        roof = {"bound": "mfma", "achieved": fl / avg / 1e12, "peak": pk_fl, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": by / avg / 1e9, "peak": PEAK["hbm_gbs"], "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    theta_file = ("theta_fft.hip" if fft else "theta_panel.hip" if path == "panel" else
                  "theta_stream.hip" if path == "stream" else "theta.hip")
    kfile = os.path.join("paper_2511_11354_amd", "csrc",
                         "theta12_sem.hip" if dom == "pair_sem" else
                         theta_file if dom.startswith("theta") else "advect.hip")
    roof["traffic"] = load_traffic(kfile, dom, w.name, precision)
    roof["kernel"] = dom
    roof["algorithmic_bytes_per_launch"] = by
    roof["algorithmic_flops_per_launch"] = fl
    roof["avg_launch_ms"] = ms / cnt
    res.update({"value": npts * steps / dt, "ms_per_step": dt / steps * 1e3, "roofline": roof,
                "kernels": kernels, "theta_kernel": path, "band": band, "obs": ob,
                "precision": precision, "meanfield_lambda": lam})
    if keep_state:
        res["state"] = s.get_state()
    s.close()
    del s
    torch.cuda.synchronize()
    return res


if __name__ == "__main__":
    main()
