"""Build the gfx950 FDETD library in-tree: paper_2605_12132_amd/_build/libfdetd.so.

hipcc cross-compiles for gfx950 without a GPU.  Packed-FP32 instruction selection is disabled for all
device code.  Objects are built in parallel and linked into one shared library exporting the C-ABI
declared in include/fdetd.h.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libfdetd.so")

# (source, object name, extra defines): the row-marching kernels are instantiated per range of the stencil
# half width N_D in separate compiler processes
ND_RANGES = [(1, 3), (4, 6), (7, 8), (9, 10), (11, 12), (13, 14), (15, 15), (16, 16)]
SOURCES = ([("fdetd_march.hip", f"fdetd_march_nd{lo}_{hi}", [f"-DFDETD_ND_LO={lo}", f"-DFDETD_ND_HI={hi}"])
            for lo, hi in ND_RANGES]
           + [("fdetd_march.hip", f"fdetd_march_any{a}", ["-DFDETD_ND_LO=1", "-DFDETD_ND_HI=0", f"-DFDETD_ANY_WIDTH={a}"])
              for a in (0, 1, 2)]  # launches that mix stencil widths: FP64, FP32, FP32 compensated last stage
           + [(f, f, []) for f in ("fdetd_kernels.hip", "fdetd_noalloc.hip", "fdetd_plan.cpp", "fdetd_coeffs.cpp",
                                   "fdetd_dispatch.cpp")])
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _compile(entry) -> str:
    src, name, defines = entry
    obj = os.path.join(OUT_DIR, name + ".o")
    cmd = [_hipcc(), *COMMON, *defines]
    if src.endswith(".hip"):
        cmd += ["-x", "hip", *DEVICE]
    else:
        cmd += ["-D__HIP_PLATFORM_AMD__"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    workers = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    for stale in os.listdir(OUT_DIR):
        if stale.endswith(".o") and os.path.join(OUT_DIR, stale) not in objs:
            os.remove(os.path.join(OUT_DIR, stale))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
