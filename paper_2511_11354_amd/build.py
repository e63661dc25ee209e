"""Build libwig2.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

    python -m paper_2511_11354_amd.build        # or build() from Python

Every translation unit is compiled to an object under ``_build/`` (in
parallel), then linked into ``paper_2511_11354_amd/libwig2.so``.  Device code
is built with packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libwig2.so")
BUILD = os.path.join(HERE, "_build")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
          f"-I{INCLUDE}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast"]
# Matrix-core accumulators in ordinary VGPRs (no AGPR copies around the loops):
# the box two-body GEMM otherwise copies its accumulators into AGPRs every K
# stage (122 against 132 ms per operator application at 129^2 x 256^2 FP64);
# bitwise the same results, neutral to slightly faster for the Theta kernels.
DEVICE_EXTRA = {
    "theta12_sem.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "theta.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "theta_stream.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def _sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip", *DEVICE, *DEVICE_EXTRA.get(os.path.basename(src), []), *COMMON, "-c", src,
               "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, "-pthread", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
