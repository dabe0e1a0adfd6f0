"""Build libmpchol.so (the gfx950 HIP library behind include/mpchol.h) and
libspdgen.so (the seeded input generator) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmpchol.so")
GENLIB = os.path.join(HERE, "libspdgen.so")
ARCH = os.environ.get("MPCHOL_ARCH", "gfx950")

SOURCES = ["k_quant.hip", "k_gemm.hip", "k_gemm_f32f64.hip", "k_leaf.hip", "k_trsm_inv.hip", "k_solve.hip",
           "k_batched.hip", "k_policy.hip", "k_check.hip", "plan.cpp", "capi.cpp"]
# the leaf kernels round every a*b and every subtraction separately, in the
# order of the textbook elimination; their elimination chains are latency
# bound, and the ILP-oriented scheduler starts each column's square root before
# the updates that the next column does not need
EXTRA = {"k_leaf.hip": ["-ffp-contract=off", "-mllvm", "-amdgpu-sched-strategy=iterative-ilp"],
         "k_trsm_inv.hip": ["-ffp-contract=off"], "k_batched.hip": ["-ffp-contract=off"],
         # FP32 / FP64 GEMMs: VGPR-form MFMAs keep the 128-tile kernels at two
         # waves per SIMD with the accumulators in place
         "k_gemm_f32f64.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}
GEN_SOURCES = ["spdgen.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          # keep the compiler from emitting packed FP32 arithmetic
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def _compile(src: str, extra: list[str]) -> str:
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [_hipcc()] + COMMON + extra + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _link(objs: list[str], out: str) -> None:
    tmp = out + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed for {out}:\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> tuple[str, str]:
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, EXTRA.get(s, [])), SOURCES))
        gobjs = list(ex.map(lambda s: _compile(s, ["-ffp-contract=off"]), GEN_SOURCES))
    _link(objs, LIB)
    _link(gobjs, GENLIB)
    if verbose:
        print(f"built {LIB}\nbuilt {GENLIB}", flush=True)
    return LIB, GENLIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
