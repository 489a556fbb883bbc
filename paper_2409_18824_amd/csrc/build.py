"""Build libj3d.so for gfx950 (MI355X) in-tree.

Usage: python -m paper_2409_18824_amd.csrc.build  (or call build()).

The device code (kernels.hip) is compiled by hipcc for gfx950 only; the host
runtime (*.cpp) by clang++ against the HIP runtime headers.  Every object is
compiled with floating-point contraction off, correctly rounded FP32
division and square root, no FP32 denormal flushing, and packed FP32
instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libj3d.so")
BUILD = os.path.join(PKG, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=off", "-I", INCLUDE, "-I", HERE]
DEVICE = ["--offload-arch=" + ARCH, "-fhip-fp32-correctly-rounded-divide-sqrt",
          "-fno-gpu-flush-denormals-to-zero",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_SOURCES = ["runtime.cpp", "capi.cpp", "solve.cpp", "batch.cpp", "serve.cpp", "jacobi2d.cpp",
                "advect.cpp"]
DEVICE_SOURCES = ["kernels.hip", "kernels_f64.hip", "kernels_f32.hip", "kernels_sweep2.hip",
                  "kernels_sweep2_f32.hip", "kernels_sweep3.hip", "kernels_sweep3_f32.hip", "kernels_2d.hip",
                  "kernels_advect.hip", "noalloc.hip"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n%s\n%s" % (" ".join(cmd), r.stdout))
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clangxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    jobs = []
    for src in DEVICE_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([hipcc, "-c", *COMMON, *DEVICE, os.path.join(HERE, src), "-o", obj])
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([clangxx, "-c", "-x", "c++", *COMMON, "-D__HIP_PLATFORM_AMD__",
                     "-I", os.path.join(ROCM, "include"), os.path.join(HERE, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(BUILD, s + ".o") for s in DEVICE_SOURCES + HOST_SOURCES]
    tmp = OUT + ".tmp%d" % os.getpid()
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp,
          "-Wl,--no-undefined", "-lpthread"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
