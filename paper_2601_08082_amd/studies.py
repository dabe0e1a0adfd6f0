"""Sub-kernel and depth studies on one MI355X (the paper's Sections 4.2 and 4.4).

    python -m paper_2601_08082_amd.studies subkernels [--sizes 8192,16384,...]
    python -m paper_2601_08082_amd.studies depth [--sizes ...] [--max-depth 6]
    python -m paper_2601_08082_amd.studies step [--sizes 65536] [--steps 3] [--workload large|single]
    python -m paper_2601_08082_amd.studies e4m3 [--sizes 32768,65536]

subkernels: Tree-SYRK and Tree-TRSM on their own (mpchol_syrk / mpchol_trsm),
at the shapes the outermost Tree-POTRF level issues for an order-n matrix
(A21 of n/2 x n/2 against L11 of n/2; A22 of n/2 updated by n/2 columns), for
the precision lists of Section 4.2, each against the recursion of the same
schedule run entirely in its diagonal (last) precision.
depth: the whole factorization (mpchol_factor) for precision lists of
increasing depth, [F16] * d + [F32] and [F16] * d + [F64], leaf 256, against
the all-F32 / all-F64 tree of the same schedule: time, speedup, backward error.
step: the benchmark's step on its own (large: factor with [F16,F32,F64] over a
leaf of 256 in FP64, then the FP64-refined solve of 16 right-hand sides,
dominance ratio 1.2; single: [F16,F16,F32,F32,F32,F32], 1 right-hand side,
ratio 1.5), a few times, with nothing else in the process: the command a
kernel-trace profiler wraps.
e4m3: the factorization with the level-0 updates in E4M3 (per-block power-of-two
scales both ways, scale_mode 1) against the same tree with FP16 there,
[p0, F32, F64] over a leaf of 256 in FP64, dominance ratio 1.2: time, backward
error, and per launch class the time and rate (the level-0 GEMM class against
the dense FP8 / FP16 MFMA peak).

Inputs are the synthetic diagonally dominant SPD matrices of the benchmark
(dominance ratio 1.5) generated on the device; times are the medians of five
calls after two warm-ups (HIP events inside the library).  One JSON line per
measurement.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _label(M, lst):
    return "[" + ",".join(M.PREC_LABELS[p] for p in lst) + "]"


def _time(fn, reps=5, warm=2):
    for _ in range(warm):
        fn()
    ms = [fn() for _ in range(reps)]
    return float(np.median(ms))


def subkernels(sizes):
    import torch
    from paper_2601_08082_amd import mpchol as M
    from paper_2601_08082_amd import spdgen_gpu
    ctx = M.Context(0)
    F16, F32, F64 = M.F16, M.F32, M.F64
    lists = [[F64], [F32], [F16, F32], [F16, F16, F32], [F16, F16, F16, F16, F32],
             [F16] * 12 + [F32]]
    for n in sizes:
        h = n // 2
        A0 = spdgen_gpu.gen_spd(n, 1.5, 0.0, 8, n)
        # L11 = Cholesky factor of the leading block, so the TRSM is the
        # factorization's own level-0 solve
        ctx.factor(A0, h, M.Tree(leaf=256, offdiag=[F64]), L_cm=A0)
        base = {}
        for lst in lists:
            leaf_prec = F32 if lst[-1] == F32 else F64
            t = M.Tree(leaf=256, offdiag=lst, leaf_prec=leaf_prec)
            A = torch.empty_like(A0)
            for op in ("syrk", "trsm"):
                def run():
                    A.copy_(A0)
                    fn = ctx.syrk if op == "syrk" else ctx.trsm
                    return fn(A, h, h, t)["ms_factor"]
                ms = _time(run)
                flops = h * h * h   # SYRK: h(h+1)/2 outputs x 2h; TRSM: h x h^2
                key = (op, lst[-1])
                if len(set(lst)) == 1:
                    base[key] = ms
                rec = {"study": "subkernel", "op": op, "n_matrix": n, "m": h, "k": h,
                       "list": _label(M, lst), "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12}
                if key in base:
                    rec["speedup_vs_" + M.PREC_LABELS[lst[-1]]] = base[key] / ms
                print(json.dumps(rec), flush=True)
            del A
        del A0
        torch.cuda.empty_cache()
    ctx.close()


def depth(sizes, max_depth):
    import torch
    from paper_2601_08082_amd import mpchol as M
    from paper_2601_08082_amd import spdgen_gpu
    ctx = M.Context(0)
    F16, F32, F64 = M.F16, M.F32, M.F64
    for n in sizes:
        A = spdgen_gpu.gen_spd(n, 1.5, 0.0, 8, n)
        L = torch.empty_like(A)
        for diag in (F32, F64):
            t0 = M.Tree(leaf=256, offdiag=[diag], leaf_prec=diag)
            ms0 = _time(lambda: ctx.factor(A, n, t0, L_cm=L)[1]["ms_factor"])
            # the device check is an O(n^3) FP64 product: skipped at the largest order
            be0 = ctx.backward_error(A, L, n)[0] if n <= 32768 else None
            print(json.dumps({"study": "depth", "n": n, "list": _label(M, [diag]), "ms": ms0,
                              "tflops": n ** 3 / 3 / (ms0 * 1e-3) / 1e12, "backward_error": be0}),
                  flush=True)
            for d in range(1, max_depth + 1):
                if n >> d < 512:
                    break
                lst = [F16] * d + [diag]
                t = M.Tree(leaf=256, offdiag=lst, leaf_prec=diag)
                ms = _time(lambda: ctx.factor(A, n, t, L_cm=L)[1]["ms_factor"])
                be = ctx.backward_error(A, L, n)[0] if n <= 32768 else None
                print(json.dumps({"study": "depth", "n": n, "list": _label(M, lst), "ms": ms,
                                  "tflops": n ** 3 / 3 / (ms * 1e-3) / 1e12,
                                  "speedup_vs_" + M.PREC_LABELS[diag]: ms0 / ms,
                                  "backward_error": be}), flush=True)
        del A, L
        torch.cuda.empty_cache()
    ctx.close()


def step(sizes, steps, workload):
    import torch
    from paper_2601_08082_amd import mpchol as M
    from paper_2601_08082_amd import spdgen_gpu
    ctx = M.Context(0)
    if workload == "large":
        levels, ratio, nrhs = [M.F16, M.F32, M.F64], 1.2, 16
    else:
        levels, ratio, nrhs = [M.F16, M.F16, M.F32, M.F32, M.F32, M.F32], 1.5, 1
    tree = M.Tree(leaf=256, offdiag=levels, leaf_prec=M.F64)
    for n in sizes:
        A = spdgen_gpu.gen_spd(n, ratio, 0.0, seed=8, lda=n)
        B = spdgen_gpu.gen_rhs(n, nrhs, seed=108, ldb=n)
        L = torch.empty_like(A)
        X = torch.empty_like(B)
        for i in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.factor(A, n, tree, L_cm=L, sync=False)
            _, s = ctx.solve(L, B, n, A_cm=A, tol=1e-13, max_iter=20, X_cm=X)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            print(json.dumps({"study": "step", "n": n, "step": i, "ms": ms,
                              "ir_iters": s["ir_iters"], "status": s["status"]}), flush=True)
        del A, B, L, X
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    ctx.close()


def e4m3(sizes):
    import torch
    from paper_2601_08082_amd import mpchol as M
    from paper_2601_08082_amd import spdgen_gpu
    peaks = {"gemm_e4m3": 5000.0, "gemm_f16": 2500.0, "gemm_f32": 157.3, "gemm_f64": 78.6}
    ctx = M.Context(0)
    for n in sizes:
        A = spdgen_gpu.gen_spd(n, 1.2, 0.0, 8, n)
        L = torch.empty_like(A)
        for p0, sm in ((M.E4M3, 1), (M.F16, 0)):
            t = M.Tree(leaf=256, offdiag=[p0, M.F32, M.F64], leaf_prec=M.F64, scale_mode=sm)
            ms = _time(lambda: ctx.factor(A, n, t, L_cm=L)[1]["ms_factor"], reps=3, warm=1)
            ctx.profile(M.PROF_KINDS)
            ctx.factor(A, n, t, L_cm=L)
            torch.cuda.synchronize()
            prof = ctx.profile_read()
            ctx.profile([])
            be = ctx.backward_error(A, L, n)[0] if n <= 32768 else None
            classes = {}
            for k, (cms, work, nl) in prof.items():
                if not nl:
                    continue
                rec = {"ms": cms, "launches": nl}
                if k in peaks and cms > 0:
                    rec["tflops"] = work / (cms * 1e-3) / 1e12
                    rec["frac_of_peak"] = rec["tflops"] / peaks[k]
                classes[k] = rec
            print(json.dumps({"study": "e4m3", "n": n, "level0": M.PREC_LABELS[p0],
                              "scale_mode": sm, "ms_factor": ms,
                              "tflops": n ** 3 / 3 / (ms * 1e-3) / 1e12, "backward_error": be,
                              "classes": classes}), flush=True)
        del A, L
        torch.cuda.empty_cache()
    ctx.close()


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["subkernels", "depth", "step", "e4m3"])
    ap.add_argument("--sizes", default="8192,16384,32768,65536")
    ap.add_argument("--max-depth", type=int, default=6)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--workload", choices=["large", "single"], default="large")
    a = ap.parse_args()
    sizes = [int(x) for x in a.sizes.split(",")]
    if a.study == "subkernels":
        subkernels(sizes)
    elif a.study == "step":
        step(sizes, a.steps, a.workload)
    elif a.study == "e4m3":
        e4m3(sizes)
    else:
        depth(sizes, a.max_depth)
    return 0


if __name__ == "__main__":
    sys.exit(main())
