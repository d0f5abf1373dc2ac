"""Build ``libqsim.so`` (HIP kernels for gfx950 + host runtime + compiler).

Every HIP source is compiled with hipcc for gfx950 only; the pure C++ compiler
pass is compiled with g++.  Objects are built in parallel and linked into
``paper_2010_09746_amd/libqsim.so``.  Run ``python -m paper_2010_09746_amd.build``.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libqsim.so")
OBJDIR = os.path.join(PKG, "_build")

# the tile-pass units first: they take minutes each and compile in parallel
HIP_SOURCES = ["tile_f64.hip", "tile_f64_plain.hip", "tile_f64_z.hip", "tile_f32.hip", "tile_f32_plain.hip",
               "tile_f32_z.hip", "batch_f64.hip", "batch_f32.hip", "api.cpp", "batch_api.cpp", "server_api.cpp",
               "gates.hip", "readout.hip", "noalloc.hip"]
CXX_SOURCES = ["compiler.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep the per-slot branches of the tile kernel separate, so register
    # arrays are indexed with constants and stay in VGPRs
    "-mllvm", "-simplifycfg-sink-common=false",
    # Branches on uniform values (operation kind, register slot, register
    # controls) stay plain scalar branches instead of being rewritten into a
    # structured form, and FP64 multiply-adds use the three-address form: with
    # both, every variant of the tile kernel's op loop updates the register
    # array in place instead of copying it at each iteration.
    "-mllvm", "-structurizecfg-skip-uniform-regions=true",
    "-Xclang", "-target-feature", "-Xclang", "-fmacf64-inst",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l and "fmacf64-inst" not in l)
    if p.returncode != 0:
        raise RuntimeError("build step failed: " + " ".join(cmd) + "\n" + out)
    return out


def _obj(src):
    return os.path.join(OBJDIR, os.path.basename(src) + ".o")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    steps = []
    for s in HIP_SOURCES:
        src = os.path.join(CSRC, s)
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        steps.append([HIPCC] + HIP_FLAGS + lang + ["-c", src, "-o", _obj(src)])
    for s in CXX_SOURCES:
        src = os.path.join(CSRC, s)
        steps.append(["g++"] + CXX_FLAGS + ["-c", src, "-o", _obj(src)])
    jobs = jobs or min(len(steps), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, out in zip(steps, ex.map(_run, steps)):
            if verbose:
                print(" ".join(cmd), flush=True)
                if out.strip():
                    print(out, flush=True)
    objs = [_obj(os.path.join(CSRC, s)) for s in HIP_SOURCES + CXX_SOURCES]
    tmp = OUT + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
