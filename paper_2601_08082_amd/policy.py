"""Training and use of the learned per-node precision policy.

Every step runs in the library's kernels (mpchol_policy_features,
mpchol_policy_labels, mpchol_mlp_train_step, mpchol_policy_choose); this
module only generates the synthetic training matrices, shuffles minibatches
on the host and strings the calls together.

Training set (one row per internal Tree-POTRF node): `count` seeded matrices
with n log-uniform in [nmin, nmax] (multiples of 256) from two families:
diagonally dominant ones with dominance ratio log-uniform in [rmin, rmax],
and squared-exponential covariance matrices (length scale uniform in
[0.1, 0.5], nugget log-uniform in [1e-3, 1]) that are not dominant and are
ill-conditioned; leaf size 64, 128 or 256.  Features from A, labels from an
FP64 factor of A: the cheapest precision, not below MIN_PREC, whose
quantization error of the node's L21 block fits the node's share of the
budget tau * g (g the factor's pivot ratio, at most 1 / the conditioning).

Inference: the perceptron picks each node's precision; the factor runs with
scale_mode 2 (E4M3 blocks scaled up to the format's range, FP16 and FP32
blocks only down, so their casts stay single-pass).  If the factor or the
refined solve fails, the fallback chain retries with the fixed paper tree
and then with the all-FP64 tree.

    python -m paper_2601_08082_amd.policy --count 3000 --out paper_2601_08082_amd/policy_mi355x.npy
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time
from dataclasses import dataclass

import numpy as np

from . import mpchol as M

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "policy_mi355x.npy")


SCALE_MODE = 2
TAU = 1e-2
# cheapest format a label may name: on MI355X with these kernels E4M3 is not
# faster than FP16 (two-pass casts with upward scales, 128-row GEMM tiles)
MIN_PREC = M.F16


@dataclass(frozen=True)
class MatrixSpec:
    """One seeded synthetic system: kind "dominance" (a = ratio, b = shift)
    or "kernel" (a = length scale, b = nugget)."""
    kind: str
    n: int
    a: float
    b: float
    seed: int

    def generate(self, device="cuda"):
        from . import spdgen_gpu
        if self.kind == "dominance":
            return spdgen_gpu.gen_spd(self.n, self.a, self.b, seed=self.seed, device=device)
        if self.kind == "kernel":
            return spdgen_gpu.gen_kernel(self.n, self.a, self.b, seed=self.seed, device=device)
        raise ValueError(f"unknown matrix family {self.kind!r}")


def policy_tree(leaf: int = 256, split_align: int = 1) -> "M.Tree":
    """Descriptor the policy's node numbering refers to (per-node override on top)."""
    return M.Tree(leaf=leaf, offdiag=[M.F16], leaf_prec=M.F64, split_align=split_align,
                  scale_mode=SCALE_MODE)


def init_params(seed: int = 0) -> np.ndarray:
    """He-initialised float32 parameter vector (mu = 0, sigma = 1)."""
    rng = np.random.default_rng(seed)
    k = M.MLP_IN
    p = np.zeros(M.MLP_PARAMS, dtype=np.float32)
    p[0:k] = 0.0
    p[k:2 * k] = 1.0
    o = 2 * k
    for fan_out, fan_in in ((64, k), (64, 64), (4, 64)):
        p[o:o + fan_out * fan_in] = rng.normal(0, math.sqrt(2.0 / fan_in), fan_out * fan_in)
        o += fan_out * fan_in + fan_out
    return p


def training_recipe(count: int, nmin: int = 1024, nmax: int = 8192, rmin: float = 1.05,
                    rmax: float = 10.0, seed: int = 5, kernel_frac: float = 0.4):
    """`count` MatrixSpecs: a kernel_frac share of covariance matrices, the
    rest diagonally dominant."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))
    ns = np.clip(np.rint(ns / 256.0) * 256, nmin, nmax).astype(np.int64)
    ratios = np.exp(rng.uniform(math.log(rmin), math.log(rmax), count))
    ells = rng.uniform(0.1, 0.5, count)
    nuggets = np.exp(rng.uniform(math.log(1e-3), math.log(1.0), count))
    kern = rng.uniform(0.0, 1.0, count) < kernel_frac
    out = []
    for i in range(count):
        sd = seed * 100_003 + i
        if kern[i]:
            out.append(MatrixSpec("kernel", int(ns[i]), float(ells[i]), float(nuggets[i]), sd))
        else:
            out.append(MatrixSpec("dominance", int(ns[i]), float(ratios[i]), 0.0, sd))
    return out


def leaf_mix(count: int, seed: int = 7, leaves=(64, 128, 256)):
    """Leaf size per training matrix: smaller leaves put deep nodes (depth up
    to 6-7 at n = 8192) into the training set, as deep as the leaf-256 tree of
    an n = 32768 system goes."""
    rng = np.random.default_rng(seed)
    return [int(b) for b in rng.choice(leaves, count)]


def build_dataset(ctx, specs, tree, tau: float = TAU, log_every: int = 0, leaves=None):
    """Features (rows, 5) float32 and labels (rows,) int32, as device tensors.
    leaves: optional per-matrix leaf sizes (else the tree's)."""
    import dataclasses

    import torch
    feats, labs = [], []
    t0 = time.time()
    base = tree
    for i, sp in enumerate(specs):
        tree = dataclasses.replace(base, leaf=leaves[i]) if leaves else base
        t64 = M.Tree(leaf=tree.leaf, offdiag=[M.F64], leaf_prec=M.F64, split_align=tree.split_align)
        A = sp.generate()
        L, info = ctx.factor(A, sp.n, t64)
        if info["status"] != 0:
            raise RuntimeError(f"training matrix {i} ({sp}): FP64 factor failed {info}")
        feats.append(ctx.policy_features(A, sp.n, tree))
        lab, _ = ctx.policy_labels(A, L, sp.n, tree, tau=tau, scale_mode=SCALE_MODE,
                                   min_prec=MIN_PREC)
        labs.append(lab)
        del A, L
        if log_every and (i + 1) % log_every == 0:
            print(f"[policy] dataset {i + 1}/{len(specs)} matrices, {time.time() - t0:.1f} s",
                  flush=True)
    X = torch.cat(feats)
    y = torch.cat(labs)
    torch.cuda.synchronize()
    return X, y


def train(ctx, X, y, epochs: int = 30, batch: int = 1024, lr: float = 3e-3, seed: int = 0,
          params0: np.ndarray | None = None, log_every: int = 0):
    """Adam on the mean cross-entropy; returns (params device tensor, per-epoch mean losses)."""
    import torch
    dev = X.device
    Xh = X.cpu().numpy().astype(np.float64)
    p = init_params(seed) if params0 is None else params0.astype(np.float32).copy()
    # standardization from the data (host, MLP_IN numbers each)
    mu = Xh.mean(axis=0)
    sd = Xh.std(axis=0)
    sd[sd < 1e-6] = 1.0
    p[0:M.MLP_IN] = mu
    p[M.MLP_IN:2 * M.MLP_IN] = sd
    params = torch.from_numpy(p).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    rng = np.random.default_rng(seed + 1)
    rows = X.shape[0]
    Xc, yc = X.cpu(), y.cpu()
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(rows))
        Xs = Xc[perm].contiguous().to(dev)
        ys = yc[perm].contiguous().to(dev)
        losses = []
        for b0 in range(0, rows, batch):
            b1 = min(rows, b0 + batch)
            step += 1
            loss, _ = ctx.mlp_train_step(Xs[b0:b1], ys[b0:b1], params, m, v, step, lr)
            losses.append(loss)
        hist.append(float(torch.stack(losses).mean().item()))
        if log_every and (ep + 1) % log_every == 0:
            print(f"[policy] epoch {ep + 1}/{epochs} loss {hist[-1]:.4f}", flush=True)
    return params, hist


def accuracy(ctx, X, y, params) -> float:
    _, cls = ctx.mlp_forward(X, params)
    return float((cls == y).float().mean().item())


def load_params(path: str = DEFAULT_WEIGHTS, device="cuda"):
    import torch
    p = np.load(path)
    if p.shape != (M.MLP_PARAMS,) or p.dtype != np.float32:
        raise ValueError(f"{path}: expected float32[{M.MLP_PARAMS}]")
    return torch.from_numpy(p).to(device)


def fixed_tree(leaf: int = 256, split_align: int = 1) -> "M.Tree":
    """The paper's fixed tree the policy is compared with: FP16 off-diagonal
    blocks at every level, FP64 leaves (Section 3.3)."""
    return M.Tree(leaf=leaf, offdiag=[M.F16], leaf_prec=M.F64, split_align=split_align)


def fp64_tree(leaf: int = 256, split_align: int = 1) -> "M.Tree":
    return M.Tree(leaf=leaf, offdiag=[M.F64], split_align=split_align)


def three_level_tree(leaf: int = 256, split_align: int = 1) -> "M.Tree":
    """The paper's three-level layering (Section 4.2): FP16 at the outermost
    level, FP32 at the next, FP64 below, FP64 leaves."""
    return M.Tree(leaf=leaf, offdiag=[M.F16, M.F32, M.F64], leaf_prec=M.F64,
                  split_align=split_align)


def learned_tree(tree, choice) -> "M.Tree":
    return M.Tree(leaf=tree.leaf, offdiag=list(tree.offdiag), leaf_prec=tree.leaf_prec,
                  split_align=tree.split_align, scale_mode=SCALE_MODE, node_prec=list(choice))


def run_chain(ctx, A, B, n: int, chain, tol: float, max_iter: int, L=None, X=None):
    """Factor and refine with each (name, tree) of `chain` until one succeeds.
    Returns (X, info dict with the tree used and the number of fallbacks)."""
    fallbacks = 0
    for name, t in chain:
        L, finfo = ctx.factor(A, n, t, L_cm=L)
        if finfo["status"] != 0:
            fallbacks += 1
            continue
        X, sinfo = ctx.solve(L, B, n, A_cm=A, tol=tol, max_iter=max_iter, X_cm=X)
        if sinfo["status"] == 0:
            return X, {"used": name, "fallbacks": fallbacks, "ir_iters": sinfo["ir_iters"],
                       "solve": sinfo}
        fallbacks += 1
    raise RuntimeError("every tree of the fallback chain failed")


def solve_with_policy(ctx, A, B, n: int, params, tree=None, tol: float = 1e-12,
                      max_iter: int = 20, L=None, X=None):
    """Factor with the learned per-node precisions and refine; on failure fall
    back to the fixed tree, then to all-FP64.  Returns (X, info dict)."""
    tree = tree or policy_tree()
    choice = ctx.policy_choose(A, n, tree, params)
    chain = [("learned", learned_tree(tree, choice)),
             ("fixed", fixed_tree(tree.leaf, tree.split_align)),
             ("fp64", fp64_tree(tree.leaf, tree.split_align))]
    X, info = run_chain(ctx, A, B, n, chain, tol, max_iter, L, X)
    info["node_prec"] = choice
    return X, info


def measure(ctx, A, B, n: int, params, tree, tol: float = 1e-12, max_iter: int = 20,
            reps: int = 3):
    """Measured time to a refined solution (correction below `tol`), inputs
    resident on the device, median of `reps` after one warm-up, for: the
    learned tree (choice of precisions included) with its fallback chain, the
    fixed all-FP16 tree and the paper's three-level tree (each falling back
    to FP64), and the all-FP64 tree."""
    import torch
    L = torch.empty_like(A)
    X = torch.empty_like(B)
    fx = [("fixed", fixed_tree(tree.leaf, tree.split_align)),
          ("fp64", fp64_tree(tree.leaf, tree.split_align))]
    three = [("three_level", three_level_tree(tree.leaf, tree.split_align)), fx[1]]
    runs = {
        "learned": lambda: solve_with_policy(ctx, A, B, n, params, tree, tol, max_iter, L, X),
        "fixed": lambda: run_chain(ctx, A, B, n, fx, tol, max_iter, L, X),
        "three_level": lambda: run_chain(ctx, A, B, n, three, tol, max_iter, L, X),
        "fp64": lambda: run_chain(ctx, A, B, n, fx[1:], tol, max_iter, L, X),
    }
    out = {}
    for name, fn in runs.items():
        ms = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Xr, info = fn()
            torch.cuda.synchronize()
            if r:
                ms.append((time.perf_counter() - t0) * 1e3)
        rec = {"tts_ms": float(np.median(ms)), "used": info["used"],
               "fallbacks": info["fallbacks"], "ir_iters": info["ir_iters"],
               "correction": info["solve"]["final_rel_corr"]}
        if name == "learned":
            ch = info["node_prec"]
            rec["choice_counts"] = {nm: ch.count(p) for p, nm in
                                    enumerate(("E4M3", "F16", "F32", "F64"))}
            rec["node_prec"] = ch
        out[name] = rec
    out["gain_vs_fixed"] = out["fixed"]["tts_ms"] / out["learned"]["tts_ms"]
    out["gain_vs_three_level"] = out["three_level"]["tts_ms"] / out["learned"]["tts_ms"]
    out["gain_vs_fp64"] = out["fp64"]["tts_ms"] / out["learned"]["tts_ms"]
    return out


def evaluate(ctx, params, spec: MatrixSpec, leaf: int = 256, reps: int = 3, tol: float = 1e-12):
    """`measure` on one seeded system, plus its labels (from its FP64 factor)
    against the network's choice."""
    A = spec.generate()
    n = spec.n
    B = spdgen_rhs(n, spec.seed + 100)
    tree = policy_tree(leaf)
    out = {"system": {"kind": spec.kind, "n": n, "a": spec.a, "b": spec.b, "seed": spec.seed},
           "leaf": leaf, "tol": tol}
    out.update(measure(ctx, A, B, n, params, tree, tol, reps=reps))
    L64, _ = ctx.factor(A, n, fp64_tree(leaf))
    lab, _ = ctx.policy_labels(A, L64, n, tree, tau=TAU, scale_mode=SCALE_MODE,
                               min_prec=MIN_PREC)
    lab = lab.cpu().numpy().tolist()
    out["label_counts"] = {nm: lab.count(p) for p, nm in enumerate(("E4M3", "F16", "F32", "F64"))}
    out["choice_matches_labels"] = float(np.mean(np.array(lab) ==
                                                 np.array(out["learned"]["node_prec"])))
    del out["learned"]["node_prec"]
    return out


def spdgen_rhs(n: int, seed: int):
    from . import spdgen_gpu
    return spdgen_gpu.gen_rhs(n, 1, seed=seed)


# (system, refinement tolerance): a dominant system and a covariance matrix
# at 1e-12, and a covariance matrix whose conditioning (about 3e4) leaves the
# FP16 tree's refinement diverging, at 1e-10 (FP64 refinement stalls near
# kappa u64 ~ 3e-12 there)
EVAL_SYSTEMS = [(MatrixSpec("dominance", 32768, 1.1, 0.0, 55), 1e-12),
                (MatrixSpec("kernel", 32768, 0.1, 0.1, 56), 1e-12),
                (MatrixSpec("kernel", 16384, 0.1, 0.01, 57), 1e-10)]


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=3000)
    ap.add_argument("--nmin", type=int, default=1024)
    ap.add_argument("--nmax", type=int, default=16384)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--tau", type=float, default=TAU)
    ap.add_argument("--leaf", type=int, default=256)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--eval-only", action="store_true", help="evaluate the saved weights")
    ap.add_argument("--mixed-leaves", type=int, default=1,
                    help="1: leaf 64/128/256 per training matrix; 0: the --leaf of every matrix")
    args = ap.parse_args(argv)
    import json
    import torch
    ctx = M.Context(0)
    if not args.eval_only:
        tree = policy_tree(args.leaf)
        specs = training_recipe(args.count, args.nmin, args.nmax)
        t0 = time.time()
        X, y = build_dataset(ctx, specs, tree, args.tau, log_every=max(1, args.count // 20),
                             leaves=leaf_mix(args.count) if args.mixed_leaves else None)
        counts = np.bincount(y.cpu().numpy(), minlength=4)
        print(f"[policy] {X.shape[0]} nodes, label counts E4M3/F16/F32/F64 = {counts.tolist()}, "
              f"{time.time() - t0:.1f} s", flush=True)
        nv = max(1, args.count // 10)
        vspecs = training_recipe(nv, args.nmin, args.nmax, seed=6)
        Xv, yv = build_dataset(ctx, vspecs, tree, args.tau,
                               leaves=leaf_mix(nv, seed=8) if args.mixed_leaves else None)
        params, hist = train(ctx, X, y, args.epochs, args.batch, args.lr,
                             log_every=max(1, args.epochs // 10))
        print(f"[policy] train accuracy {accuracy(ctx, X, y, params):.4f}, validation accuracy "
              f"{accuracy(ctx, Xv, yv, params):.4f} ({Xv.shape[0]} nodes of {nv} held-out "
              f"matrices), final loss {hist[-1]:.4f}", flush=True)
        np.save(args.out, params.cpu().numpy().astype(np.float32))
        print(f"[policy] wrote {args.out}", flush=True)
        del X, y, Xv, yv
    params = load_params(args.out)
    for sp, tol in EVAL_SYSTEMS:
        print(json.dumps(evaluate(ctx, params, sp, args.leaf, tol=tol)), flush=True)
        torch.cuda.empty_cache()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
