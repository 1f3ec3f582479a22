"""Build libpic.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Always recompiles every translation unit (in parallel), then links
``paper_2303_12873_amd/libpic.so`` in place.  Usage: ``python -m
paper_2303_12873_amd.build`` or ``build()`` from Python.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpic.so")
BUILD_DIR = os.path.join(ROOT, "_build")
ARCH = os.environ.get("PIC_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # never emit packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}",
]

# pic_particles.hip once per (shape order, precision, part): part 0 the
# direct / straggler / split-call kernels, 1 the fused tiled kernels, 2 the
# fused persistent kernels; compiled in parallel.
UNITS = [
    ("libpic.hip", "libpic.o", []),
    ("pic_aux.hip", "pic_aux.o", []),
    ("pic_slab.hip", "pic_slab.o", []),
    ("pic_bound.hip", "pic_bound.o", []),
    ("pic_es.hip", "pic_es.o", []),
] + [
    ("pic_particles.hip", f"pic_particles_o{o}_p{p}_t{t}.o",
     [f"-DPIC_ORDER={o}", f"-DPIC_PREC={p}", f"-DPIC_PART={t}"])
    for o in (3, 2, 1) for p in (1, 0) for t in (2, 1, 0)
]


def _compile(unit, extra_flags=()):
    src, obj, flags = unit
    out = os.path.join(BUILD_DIR, obj)
    cmd = [HIPCC, *COMMON, *flags, *extra_flags, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


MB_OUT = os.path.join(HERE, "libpic_mb.so")


def build_microbench(extra_flags=()) -> str:
    """The hardware-rate microbenchmarks, a library of their own."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = _compile(("pic_microbench.hip", "pic_microbench.o", []), extra_flags)
    tmp = MB_OUT + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, obj],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, MB_OUT)
    return MB_OUT


def build(verbose: bool = False, extra_flags=()) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = min(len(UNITS), max(1, min(16, os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, extra_flags), UNITS))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    build_microbench(extra_flags)
    if verbose:
        print("built", OUT, "and", MB_OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, extra_flags=sys.argv[1:])
