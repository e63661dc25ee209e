"""Turn rocprofv3 output into the short text summaries kept with the project.

    python -m paper_2511_11354_amd.profiling stats DIR --command "..." [--out FILE]
        Markdown table of a `rocprofv3 --kernel-trace --stats` run (the
        kernel_stats.csv under DIR): calls, average / min / max duration.

    python -m paper_2511_11354_amd.profiling traffic --fetch DIR --write DIR
            --copy-bytes N --workload NAME --precision P [--json FILE] [--out FILE]
        HBM bytes per dispatch of each kernel from two counter runs
        (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`).  Both counters are
        scaled by what they read for the plain device copy of N bytes that
        the same run performs (the kernel whose name contains "copy"):
        factor_fetch = N / FETCH(copy), factor_write = N / WRITE(copy).
        With --json the per-class figures are merged into that file, keyed
        "class/workload/precision" and stamped with the digest of the
        kernel's source file, so a later change to the kernel voids them.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join("paper_2511_11354_amd", "csrc")


def short_name(name: str) -> str:
    n = name.replace("void ", "").replace("wig2::(anonymous namespace)::", "")
    return re.sub(r"\(.*", "", n).strip()


def kernel_class(name: str):
    """(class, source file) of a kernel of this library, or None."""
    n = short_name(name)
    m = re.match(r"k_theta_stream<(\w+), (\d+), (\w+), (\d)(?:, \d+)?>", n)
    if m:
        form = int(m.group(4))
        cls = {0: "theta_apply", 1: "theta_stage1", 2: "theta_stage2", 3: "theta_heun"}[form]
        return cls, os.path.join(CSRC, "theta_stream.hip")
    m = re.match(r"k_theta_panel(?:_bf16)?<(?:\w+, )?(\d+), (\d)>", n)
    if m:
        cls = {0: "theta_apply", 1: "theta_stage1", 2: "theta_stage2"}[int(m.group(2))]
        return cls, os.path.join(CSRC, "theta_panel.hip")
    if n.startswith("k_theta_heun<"):
        return "theta_heun", os.path.join(CSRC, "theta.hip")
    if n.startswith("k_theta_fft<"):
        return "theta_fft", os.path.join(CSRC, "theta_fft.hip")
    if n.startswith("k_fft_symbols"):
        return "theta_fft_symbols", os.path.join(CSRC, "theta_fft.hip")
    m = re.match(r"k_theta<(\w+), (\d+), (\w+), (\w+), (\d)>", n)
    if m:
        return ("theta_stage1" if m.group(5) == "0" else "theta_stage2"), os.path.join(CSRC, "theta.hip")
    if re.match(r"k_advect_reg<\w+, \d+, \w+, 2>", n):
        return "advect_x1x1", os.path.join(CSRC, "advect.hip")
    if n.startswith("k_advect"):
        return "advect", os.path.join(CSRC, "advect.hip")
    return None


def source_digest(*rel) -> str:
    h = hashlib.sha256()
    for r in rel:
        with open(os.path.join(ROOT, r), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(d, fname):
    paths = glob.glob(os.path.join(d, "**", fname), recursive=True)
    if not paths:
        raise SystemExit(f"no {fname} under {d}")
    out = []
    for p in paths:
        with open(p) as fh:
            out.extend(csv.DictReader(fh))
    return out


def stats(d, command, out=None):
    rows = _rows(d, "*kernel_stats.csv")
    lines = [f"Command (from the repository root): `{command}`", "",
             "| kernel | calls | avg ms | min ms | max ms | total ms | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                     f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} |")
    text = "\n".join(lines) + "\n"
    if out:
        with open(out, "w") as fh:
            fh.write(text)
    return text


def _counter_values(d, counter):
    acc = defaultdict(list)
    for r in _rows(d, "*counter_collection.csv"):
        if r["Counter_Name"] == counter:
            acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return acc


def traffic(fetch_dir, write_dir, copy_bytes, workload, precision, json_path=None, out=None,
            commands=None):
    fv = _counter_values(fetch_dir, "FETCH_SIZE")
    wv = _counter_values(write_dir, "WRITE_SIZE")
    copies = [k for k in fv if "copy" in k.lower()]
    if not copies:
        raise SystemExit("no copy kernel in the FETCH_SIZE run")
    # the calibration copy is the largest copy dispatch of the run
    ck = max(copies, key=lambda k: max(fv[k]))
    cf, cw = max(fv[ck]), max(wv[ck])
    ffac = copy_bytes / (cf * 1024.0)
    wfac = copy_bytes / (cw * 1024.0)
    fetch = {k: sum(v) / len(v) for k, v in fv.items()}
    write = {k: sum(v) / len(v) for k, v in wv.items()}
    nf = {k: len(v) for k, v in fv.items()}
    lines = [f"Commands (from the repository root): {' ; '.join(f'`{c}`' for c in commands)}", ""] if commands else []
    lines += [f"Calibration: the largest dispatch of `{short_name(ck)}` copies {copy_bytes} bytes and reads "
             f"FETCH_SIZE {cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB -> scale factors {ffac:.3f} (fetch), "
             f"{wfac:.3f} (write).  Per-kernel rows are means over dispatches.", "",
             "| kernel | dispatches | FETCH KiB | WRITE KiB | scaled GB read | scaled GB written | GB total |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    rec = {}
    if json_path and os.path.exists(json_path):
        rec = json.load(open(json_path))
    for k in sorted(fetch, key=lambda k: -fetch[k]):
        if k not in write:
            continue
        rd, wr = fetch[k] * 1024.0 * ffac, write[k] * 1024.0 * wfac
        lines.append(f"| `{short_name(k)}` | {nf[k]} | {fetch[k]:.0f} | {write[k]:.0f} | {rd / 1e9:.3f} | "
                     f"{wr / 1e9:.3f} | {(rd + wr) / 1e9:.3f} |")
        kc = kernel_class(k)
        if kc and json_path:
            cls, src = kc
            keys = [cls] if cls != "advect" else ["advect_x1", "advect_x2"]
            for c in keys:
                rec[f"{c}/{workload}/{precision}"] = {
                    "bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr,
                    "fetch_kib": fetch[k], "write_kib": write[k], "fetch_factor": ffac,
                    "write_factor": wfac, "kernel": short_name(k), "source": src,
                    "source_sha": source_digest(src)}
    if json_path:
        with open(json_path, "w") as fh:
            json.dump(rec, fh, indent=1, sort_keys=True)
    text = "\n".join(lines) + "\n"
    if out:
        with open(out, "w") as fh:
            fh.write(text)
    return text


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--command", required=True)
    a.add_argument("--out")
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--workload", required=True)
    b.add_argument("--precision", required=True)
    b.add_argument("--json")
    b.add_argument("--out")
    b.add_argument("--command", action="append", help="counter run command (repeat per run)")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        sys.stdout.write(stats(args.dir, args.command, args.out))
    else:
        sys.stdout.write(traffic(args.fetch, args.write, args.copy_bytes, args.workload,
                                 args.precision, args.json, args.out, args.command))


if __name__ == "__main__":
    main()
