"""Build libfftbf.so in-tree with hipcc for gfx950.

    python -m paper_1710_08591_amd.build        (or __graft_entry__.build())

Each source under csrc/ is compiled to an object in _build/ (in parallel),
then linked into paper_1710_08591_amd/libfftbf.so; csrc/bench_main.cpp
becomes the C-ABI driver paper_1710_08591_amd/fftbf_bench.  Packed FP32 VALU ops
are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfftbf.so")
ROOT = os.path.dirname(HERE)

ARCH = "gfx950"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")   # roctx ranges (rocprofiler-sdk-roctx)
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-command-line-argument",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-mfma-vgpr-form",     # MFMA results straight into VGPRs (no AGPR copies)
    "-I", CSRC, "-I", os.path.join(ROOT, "include"),
]


BENCH_SRC = os.path.join(CSRC, "bench_main.cpp")
BENCH = os.path.join(HERE, "fftbf_bench")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")) and os.path.join(CSRC, f) != BENCH_SRC)


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(src)}:\n{msgs}")
    if msgs.strip():
        print(msgs, file=sys.stderr)
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
           f"-L{ROCM_LIB}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    # the C-ABI driver (no Python), linked against the library next to it
    # compiled as HIP for gfx950: the driver has a small kernel of its own (the voltage fill)
    cmd = [HIPCC, "-x", "hip", f"--offload-arch={ARCH}", "-O2", "-std=c++17", "-Wno-unused-command-line-argument",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), BENCH_SRC, "-o", BENCH + ".tmp",
           f"-L{HERE}", "-lfftbf", "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("fftbf_bench build failed:\n" + r.stdout + r.stderr)
    os.replace(BENCH + ".tmp", BENCH)
    if verbose:
        print(f"built {LIB} and {BENCH}")
    return LIB


if __name__ == "__main__":
    build()
