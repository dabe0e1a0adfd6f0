"""Benchmark: mixed-precision nested recursive Cholesky factor + FP64-refined
solve on one MI355X.

A step is the whole hot path on one synthetic system.  The default workload
is the largest single-GPU configuration: the 65536 x 65536 SPD matrix with
dominance ratio 1.2 (34 GB in FP64), Tree-POTRF with Tree-TRSM / Tree-SYRK in
the three-level tree [F16, F32, F64] (level 0 FP16, level 1 FP32, deeper
levels and the leaves of 256 FP64), then the substitution solve and
FP64-residual iterative refinement of 16 right-hand sides to
||d||_inf <= 1e-13 ||x||_inf.  value = effective TFLOP/s = (n^3/3) / time to
solution.  Inputs are generated in device memory before the timed region.
`--workload single` runs the n=16384 configuration (ratio 1.5, tree
[F16,F16,F32,F32,F32,F32], 1 right-hand side), `--workload batched` the
4096-system batch.

Prints ONE JSON line (rank 0).  Extra fields: the same step on the all-FP64
tree (time-to-solution speedup), factor-only rate, the roofline of the
dominant kernel measured with HIP events inside the timed region, and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks: dense MFMA by operand type, FP64 vector = matrix, HBM3E
PEAKS = {"gemm_e4m3": (5000.0, "TFLOP/s", "mfma"), "gemm_f16": (2500.0, "TFLOP/s", "mfma"),
         "gemm_f32": (157.3, "TFLOP/s", "mfma"), "gemm_f64": (78.6, "TFLOP/s", "mfma"),
         "potrf": (78.6, "TFLOP/s", "alu"), "trsm": (78.6, "TFLOP/s", "alu"),
         "cast": (8000.0, "GB/s", "hbm"), "maxabs": (8000.0, "GB/s", "hbm"),
         "trsv": (8000.0, "GB/s", "hbm"), "residual": (8000.0, "GB/s", "hbm"),
         "trinv": (78.6, "TFLOP/s", "alu")}
# committed rocprofv3 --pmc summaries of the FP16 GEMM, per workload
TRAFFIC_FILES = {"large": os.path.join(ROOT, "profiles", "gemm_f16_n65536_pmc.md"),
                 "single": os.path.join(ROOT, "profiles", "gemm_f16_n16384_pmc.md")}
GEMM_SRC = [os.path.join(ROOT, "paper_2601_08082_amd", "csrc", f) for f in ("k_gemm.hip", "dev_gemm.h")]


def _sha(paths) -> str:
    """sha256 over the concatenated sources of the kernel."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per FP16 GEMM launch from the committed rocprofv3 --pmc
    summary of this workload (FETCH_SIZE and WRITE_SIZE, scaled by the
    copy-kernel calibration); None when the summary is missing or the GEMM
    source has changed since."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILES[workload]):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip().lstrip("- ")] = v.strip()
        if kv.get("kernel_source_sha256") != _sha(GEMM_SRC):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def class_roofline(kind: str, ms: float, work: float, launches: int) -> dict:
    peak, unit, bound = PEAKS[kind]
    scale = 1e12 if unit == "TFLOP/s" else 1e9
    achieved = (work / launches) / (ms / launches * 1e-3) / scale if launches and ms > 0 else 0.0
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "launches": launches, "ms": ms}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(n_full: int, ratio: float, offdiag, leaf: int, nrhs: int, budget_s: float) -> dict:
    """The CPU oracle (factor + refined solve) on a bounded sample: the same
    generator, ratio, tree and right-hand-side count at a smaller n chosen to
    take ~budget_s."""
    import oracle as O
    from paper_2601_08082_amd import spdgen

    def run(n):
        A = spdgen.gen_spd(n, ratio, 0.0, seed=8)
        B = spdgen.gen_rhs(n, nrhs, seed=108)
        t0 = time.perf_counter()
        L, st, _ = O.factor(A, tree=O.Tree(leaf=leaf, offdiag=list(offdiag)))
        X, st2, it, _ = O.solve(L, B, A=A, tol=1e-13, max_iter=20)
        dt = time.perf_counter() - t0
        assert st == O.OK and st2 == O.OK
        return dt

    # grow the sample until one run takes at least half the budget
    n, t = 1024, run(1024)
    while t < 0.5 * budget_s and n < n_full:
        grow = min(2.0, max(1.1, (budget_s / max(t, 1e-3)) ** (1.0 / 3.0)))
        n = min(n_full, int(n * grow) // 256 * 256)
        t = run(n)
    return {"value": (n ** 3 / 3) / t / 1e12, "unit": "TFLOP/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"oracle factor + refined solve at n={n}, {nrhs} rhs (same generator, ratio, "
                      f"tree), "
                      f"{t:.1f} s on {_cpu_model()}"}


def bench_batched(args) -> dict:
    """4096 systems, sizes log-uniform in [64, 2048], dominance ratios uniform
    in [1.05, 4], 4 right-hand sides each, all-FP16 off-diagonal tree with FP64
    leaves and split alignment 32, leaf/tile per size from the tune table:
    one persistent launch per step factors, solves and refines all of them."""
    import numpy as np
    import torch

    from paper_2601_08082_amd import mpchol as M
    from paper_2601_08082_amd import spdgen
    from paper_2601_08082_amd.workloads import DeviceBatch, batch_recipe

    ns, ratios, seeds = batch_recipe(args.batch, 64, 2048, 1.05, 4.0, seed=4)
    db = DeviceBatch(ns, ratios, seeds, 4)
    ctx = M.Context(0)
    tune = os.path.join(ROOT, "paper_2601_08082_amd", "tune_mi355x.json")
    tuned = os.path.exists(tune)
    if tuned:
        ctx.load_tune_table(tune)
    tree = M.Tree(leaf=64, offdiag=[M.F16], leaf_prec=M.F64, split_align=32)
    flops = db.flops()

    def step():
        st, infos = ctx.factor_batched(db.A, db.L, db.ns, tree, db.B, db.X, tol=1e-13, max_iter=20)
        return st, infos

    for _ in range(args.warmup):
        step()
    ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, infos = step()
        ms.append(infos[0]["ms_factor"])
        if st != 0:
            bad = [i for i, x in enumerate(infos) if x["status"] != 0]
            raise RuntimeError(f"batched step: {len(bad)} systems failed, first {infos[bad[0]]}")
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    kern_ms = float(np.median(ms))
    iters = np.array([x["ir_iters"] for x in infos])

    # one more step with the task classes timed inside the kernel (outside the timed region)
    ctx.profile(M.PROF_KINDS)
    step()
    breakdown = {k: {"wg_ms": v[0], "tasks": v[2]} for k, v in ctx.profile_read().items() if v[2]}
    ctx.profile([])

    # Gershgorin certificate on a sample of systems (FP64 residual on the CPU)
    worst = 0.0
    for i in list(range(0, len(ns), max(1, len(ns) // 32))):
        n = ns[i]
        Ah = M.from_device_cm(db.A[i])
        x = M.from_device_cm(db.X[i])[:n]
        b = M.from_device_cm(db.B[i])[:n]
        lam = spdgen.gershgorin_lower_bound(n, ratios[i], 0.0, Ah)
        r = b - Ah @ x
        worst = max(worst, float(np.max(np.linalg.norm(r, axis=0) / lam / np.linalg.norm(x, axis=0))))
    ctx.close()
    achieved = flops / (kern_ms * 1e-3) / 1e12
    return {
        "metric": "effective TFLOP/s (sum n^3/3) of batched factor + refined solve",
        "value": flops / (ms_step * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16 MFMA (f32 acc) + f64 leaves, f64 in/out", "data": "synthetic",
        "config": {"workload": f"{len(ns)} SPD systems, n log-uniform [64, 2048], ratio U[1.05, 4], "
                               f"4 rhs, tree [F16] leaf FP64 split_align 32, "
                               f"{'tuned' if tuned else 'untuned (leaf 64)'} per-size leaf/tile",
                   "batch": len(ns), "total_flops": flops, "nrhs": 4,
                   "parallelism": "single GPU, one persistent launch"},
        "ir_iters_max": int(iters.max()), "ir_iters_mean": float(iters.mean()),
        "solution_error_certificate_sample": worst,
        "task_breakdown_workgroup_ms": breakdown,
        "roofline": {"bound": "mfma", "kernel": "k_batched (persistent, whole path)",
                     "achieved": achieved, "peak": PEAKS["gemm_f16"][0], "unit": "TFLOP/s",
                     "frac": achieved / PEAKS["gemm_f16"][0], "traffic": None,
                     "ms_per_launch": kern_ms},
        "cpu_baseline": None,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["large", "single", "batched"], default="large",
                    help="large: n=65536 ratio 1.2 [F16,F32,F64] 16 rhs (default); single: n=16384 "
                         "ratio 1.5 [F16,F16,F32x4] 1 rhs; batched: 4096 uneven systems")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=None, help="order (default: the workload's)")
    ap.add_argument("--ratio", type=float, default=None, help="dominance ratio (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=16.0)
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the single-matrix path is not sharded "
              "across GPUs in this build (see the design notes on sharding)", file=sys.stderr)
        return 2

    if args.workload == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return 0

    import numpy as np
    import torch

    from paper_2601_08082_amd import mpchol as M
    from paper_2601_08082_amd import spdgen, spdgen_gpu

    leaf = 256
    if args.workload == "large":
        n, ratio, nrhs = 65536, 1.2, 16
        mixed_levels = [M.F16, M.F32, M.F64]
    else:
        n, ratio, nrhs = 16384, 1.5, 1
        mixed_levels = [M.F16, M.F16, M.F32, M.F32, M.F32, M.F32]
    full_size = args.n is None and args.ratio is None
    n = args.n if args.n is not None else n
    ratio = args.ratio if args.ratio is not None else ratio
    tree = M.Tree(leaf=leaf, offdiag=mixed_levels, leaf_prec=M.F64)
    tree64 = M.Tree(leaf=leaf, offdiag=[M.F64], leaf_prec=M.F64)
    flops = n ** 3 / 3.0

    ctx = M.Context(0)
    A = spdgen_gpu.gen_spd(n, ratio, 0.0, seed=8, lda=n)
    B = spdgen_gpu.gen_rhs(n, nrhs, seed=108, ldb=n)
    L = torch.empty_like(A)
    X = torch.empty_like(B)
    torch.cuda.synchronize()

    def step(tr):
        _, finfo = ctx.factor(A, n, tr, L_cm=L, sync=False)
        _, sinfo = ctx.solve(L, B, n, A_cm=A, tol=1e-13, max_iter=20, X_cm=X)
        return sinfo

    for _ in range(args.warmup):
        s = step(tree)
    torch.cuda.synchronize()
    ctx.profile(["gemm_f16"])
    iters = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = step(tree)
        iters.append(s["ir_iters"])
        if s["status"] != 0:
            raise RuntimeError(f"solve failed: {s}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ms_step = (t1 - t0) * 1e3 / args.steps

    # one more step with every launch class timed (outside the timed region)
    ctx.profile(M.PROF_KINDS)
    step(tree)
    torch.cuda.synchronize()
    breakdown = {k: class_roofline(k, v[0], v[1], v[2]) for k, v in ctx.profile_read().items()
                 if v[2]}
    ctx.profile([])

    # factor-only rate and info (outside the timed region)
    _, finfo = ctx.factor(A, n, tree, L_cm=L, sync=True)
    fms = []
    for _ in range(3):
        torch.cuda.synchronize()
        a = time.perf_counter()
        ctx.factor(A, n, tree, L_cm=L, sync=False)
        torch.cuda.synchronize()
        fms.append((time.perf_counter() - a) * 1e3)
    factor_ms = float(np.median(fms))

    # solution check (outside the timed region): Gershgorin certificate
    # ||x - x*|| <= ||b - A x|| / lambda_min with the FP64 residual, and the
    # factor's backward error, both computed on the device
    s = step(tree)
    torch.cuda.synchronize()
    with torch.no_grad():
        Acm = A[:n, :n]                      # A symmetric: the stored block is A itself
        R = B[:nrhs, :n] - X[:nrhs, :n] @ Acm
        dg = torch.diagonal(Acm)
        lam = float(torch.min(dg - (Acm.abs().sum(dim=1) - dg.abs())).item())
        cert = float(torch.max(torch.linalg.vector_norm(R, dim=1) / lam /
                               torch.linalg.vector_norm(X[:nrhs, :n], dim=1)).item())
        del R
    be_factor = ctx.backward_error(A, L, n)[0]

    fp64 = None
    if not args.no_fp64:
        step(tree64)
        torch.cuda.synchronize()
        a = time.perf_counter()
        k64 = max(1, min(args.steps, 3))
        for _ in range(k64):
            s64 = step(tree64)
        torch.cuda.synchronize()
        fp64_ms = (time.perf_counter() - a) * 1e3 / k64
        fp64 = {"tts_ms": fp64_ms, "ir_iters": s64["ir_iters"],
                "speedup_mixed_vs_fp64": fp64_ms / ms_step}

    ms16, work16, n16 = prof["gemm_f16"]
    achieved = (work16 / n16) / (ms16 / n16 * 1e-3) / 1e12 if n16 else 0.0
    roof = {"bound": "mfma", "kernel": "k_gemm_q<f16> (grouped FP16 GEMM/SYRK)",
            "achieved": achieved, "peak": PEAKS["gemm_f16"][0], "unit": "TFLOP/s",
            "frac": achieved / PEAKS["gemm_f16"][0],
            "traffic": measured_traffic(args.workload) if full_size else None,
            "launches_per_step": n16 / args.steps, "ms_per_step": ms16 / args.steps,
            "flops_per_launch": work16 / n16 if n16 else 0.0}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(n, ratio, mixed_levels, leaf, nrhs, args.cpu_budget)

    stats = M.plan_stats(n, tree)
    out = {
        "metric": "effective TFLOP/s (n^3/3) + time-to-solution at 1e-12 rel err vs FP64 path",
        "value": flops / (ms_step * 1e-3) / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f16/f32 MFMA (f32 acc) + f64 MFMA levels and leaves, f64 in/out"
                  if M.F64 in mixed_levels else "f16/f32 MFMA (f32 acc) + f64 leaves, f64 in/out"),
        "data": "synthetic",
        "config": {"workload": f"SPD n={n} dominance ratio {ratio}, tree "
                               f"[{','.join(M.PREC_LABELS[p] for p in mixed_levels)}] "
                               f"leaf {leaf} FP64, {nrhs} rhs, FP64-residual refinement to 1e-13 "
                               f"correction",
                   "n": n, "leaf": leaf, "nrhs": nrhs, "parallelism": "single GPU"},
        "time_to_solution_ms": ms_step,
        "factor_ms": factor_ms,
        "factor_tflops": flops / (factor_ms * 1e-3) / 1e12,
        "ir_iters": int(np.median(iters)),
        "solution_error_certificate": cert,
        "backward_error": be_factor,
        "fp64_path": fp64,
        "plan": {"launches": stats["launches"], "ws_gb": stats["ws_bytes"] / 1e9,
                 "flop_share": {k: v / flops for k, v in stats["flops"].items()}},
        "kernel_breakdown_one_step": breakdown,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    # release the device memory while the process is still fully up (a
    # profiler attached to the run writes its output at exit)
    del A, B, L, X
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
