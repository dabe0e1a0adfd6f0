"""Training and use of the learned per-node precision policy.

Every step runs in the library's kernels (mpchol_policy_features,
mpchol_policy_labels, mpchol_mlp_train_step, mpchol_policy_choose); this
module only generates the synthetic training matrices, shuffles minibatches
on the host and strings the calls together.

Training set (one row per internal Tree-POTRF node): `count` matrices of the
seeded generator with n log-uniform in [nmin, nmax] (multiples of 256),
dominance ratio log-uniform in [rmin, rmax] and leaf size 64, 128 or 256;
features from A, labels from an FP64 factor of A (the cheapest precision
whose quantization error of the node's L21 block fits the node's share of the
error budget tau).

Inference: the perceptron picks each node's precision; the factor runs with
scale_mode 1 (power-of-two scaling both ways, needed by E4M3).  If the
factor or the refined solve fails, the fallback chain retries with the fixed
paper tree and then with the all-FP64 tree.

    python -m paper_2601_08082_amd.policy --count 20000 --out paper_2601_08082_amd/policy_mi355x.npy
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

from . import mpchol as M

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "policy_mi355x.npy")


def policy_tree(leaf: int = 256, split_align: int = 1) -> "M.Tree":
    """Descriptor the policy's node numbering refers to (per-node override on top)."""
    return M.Tree(leaf=leaf, offdiag=[M.F16], leaf_prec=M.F64, split_align=split_align,
                  scale_mode=1)


def init_params(seed: int = 0) -> np.ndarray:
    """He-initialised float32 parameter vector (mu = 0, sigma = 1)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(M.MLP_PARAMS, dtype=np.float32)
    o = 0
    p[o:o + 5] = 0.0
    p[o + 5:o + 10] = 1.0
    o = 10
    for fan_out, fan_in in ((64, 5), (64, 64), (4, 64)):
        p[o:o + fan_out * fan_in] = rng.normal(0, math.sqrt(2.0 / fan_in), fan_out * fan_in)
        o += fan_out * fan_in + fan_out
    return p


def training_recipe(count: int, nmin: int = 1024, nmax: int = 8192, rmin: float = 1.05,
                    rmax: float = 10.0, seed: int = 5):
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))
    ns = np.clip(np.rint(ns / 256.0) * 256, nmin, nmax).astype(np.int64)
    ratios = np.exp(rng.uniform(math.log(rmin), math.log(rmax), count))
    return [int(n) for n in ns], [float(r) for r in ratios], [seed * 100_003 + i for i in range(count)]


def leaf_mix(count: int, seed: int = 7, leaves=(64, 128, 256)):
    """Leaf size per training matrix: smaller leaves put deep nodes (depth up
    to 6-7 at n = 8192) into the training set, as deep as the leaf-256 tree of
    an n = 32768 system goes."""
    rng = np.random.default_rng(seed)
    return [int(b) for b in rng.choice(leaves, count)]


def build_dataset(ctx, ns, ratios, seeds, tree, tau: float = 1e-4, log_every: int = 0,
                  leaves=None):
    """Features (rows, 5) float32 and labels (rows,) int32, as device tensors.
    leaves: optional per-matrix leaf sizes (else the tree's)."""
    import dataclasses

    import torch
    from . import spdgen_gpu
    feats, labs = [], []
    t0 = time.time()
    base = tree
    for i, (n, r, sd) in enumerate(zip(ns, ratios, seeds)):
        tree = dataclasses.replace(base, leaf=leaves[i]) if leaves else base
        t64 = M.Tree(leaf=tree.leaf, offdiag=[M.F64], leaf_prec=M.F64, split_align=tree.split_align)
        A = spdgen_gpu.gen_spd(n, r, 0.0, seed=sd)
        L, info = ctx.factor(A, n, t64)
        if info["status"] != 0:
            raise RuntimeError(f"training matrix {i} (n={n}, ratio={r}): FP64 factor failed {info}")
        feats.append(ctx.policy_features(A, n, tree))
        lab, _ = ctx.policy_labels(A, L, n, tree, tau=tau, scale_mode=1)
        labs.append(lab)
        del A, L
        if log_every and (i + 1) % log_every == 0:
            print(f"[policy] dataset {i + 1}/{len(ns)} matrices, {time.time() - t0:.1f} s", flush=True)
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
    # standardization from the data (host, 5 numbers each)
    mu = Xh.mean(axis=0)
    sd = Xh.std(axis=0)
    sd[sd < 1e-6] = 1.0
    p[0:5] = mu
    p[5:10] = sd
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


def solve_with_policy(ctx, A, B, n: int, params, tree=None, tol: float = 1e-13,
                      max_iter: int = 20, fixed=None):
    """Factor with the learned per-node precisions and refine; on failure fall
    back to the fixed tree, then to all-FP64.  Returns (X, info dict)."""
    tree = tree or policy_tree()
    fixed = fixed or M.Tree(leaf=tree.leaf, offdiag=[M.F16], leaf_prec=M.F64,
                            split_align=tree.split_align)
    choice = ctx.policy_choose(A, n, tree, params)
    learned = M.Tree(leaf=tree.leaf, offdiag=list(tree.offdiag), leaf_prec=tree.leaf_prec,
                     split_align=tree.split_align, scale_mode=1, node_prec=choice)
    chain = [("learned", learned), ("fixed", fixed),
             ("fp64", M.Tree(leaf=tree.leaf, offdiag=[M.F64], split_align=tree.split_align))]
    fallbacks = 0
    for name, t in chain:
        L, finfo = ctx.factor(A, n, t)
        if finfo["status"] == 0:
            X, sinfo = ctx.solve(L, B, n, A_cm=A, tol=tol, max_iter=max_iter)
            if sinfo["status"] == 0:
                return X, {"used": name, "fallbacks": fallbacks, "node_prec": choice,
                           "ir_iters": sinfo["ir_iters"], "factor": finfo, "solve": sinfo}
        fallbacks += 1
    raise RuntimeError("every tree of the fallback chain failed")


def evaluate(ctx, params, n: int = 32768, ratio: float = 1.1, leaf: int = 256, reps: int = 3,
             seed: int = 55):
    """Time to a refined solution (1e-13 correction) of one seeded system
    with the learned tree, the fixed all-FP16 tree and the all-FP64 tree;
    the learned tree's fallbacks counted.  Times are medians over `reps`
    after one warm-up, inputs resident on the device."""
    import torch
    from . import spdgen_gpu
    A = spdgen_gpu.gen_spd(n, ratio, 0.0, seed=seed)
    B = spdgen_gpu.gen_rhs(n, 1, seed=seed + 100)
    L = torch.empty_like(A)
    X = torch.empty_like(B)
    tree = policy_tree(leaf)
    t0 = time.perf_counter()
    choice = ctx.policy_choose(A, n, tree, params)
    torch.cuda.synchronize()
    choose_ms = (time.perf_counter() - t0) * 1e3
    # fixed_f16_scaled scales blocks the way the learned tree does (scale_mode
    # 1, also up); fixed_f16 uses scale_mode 0, whose FP16 casts are one pass
    trees = {
        "learned": M.Tree(leaf=leaf, offdiag=[M.F16], scale_mode=1, node_prec=choice),
        "fixed_f16_scaled": M.Tree(leaf=leaf, offdiag=[M.F16], scale_mode=1),
        "fixed_f16": M.Tree(leaf=leaf, offdiag=[M.F16]),
        "fp64": M.Tree(leaf=leaf, offdiag=[M.F64]),
    }
    out = {"n": n, "ratio": ratio, "leaf": leaf, "choose_ms": choose_ms,
           "choice_counts": {nm: choice.count(p) for p, nm in enumerate(("E4M3", "F16", "F32", "F64"))}}
    for name, t in trees.items():
        ms = []
        info = None
        for r in range(reps + 1):
            torch.cuda.synchronize()
            a = time.perf_counter()
            _, fi = ctx.factor(A, n, t, L_cm=L, sync=False)
            _, si = ctx.solve(L, B, n, A_cm=A, tol=1e-13, max_iter=20, X_cm=X)
            torch.cuda.synchronize()
            if r:
                ms.append((time.perf_counter() - a) * 1e3)
            info = si
        fl = 0
        if name == "learned" and info["status"] != 0:
            fl = 1
        be = ctx.backward_error(A, ctx.factor(A, n, t, L_cm=L)[0], n)[0]
        out[name] = {"tts_ms": float(np.median(ms)), "ir_iters": info["ir_iters"],
                     "status": info["status"], "backward_error": be, "fallback": fl,
                     "flops_share": {k: v / (n ** 3 / 3) for k, v in M.plan_stats(n, t)["flops"].items()}}
    # the labels of this matrix (from its FP64 factor) against the network's choice
    L64, _ = ctx.factor(A, n, trees["fp64"], L_cm=L)
    lab, _ = ctx.policy_labels(A, L64, n, tree, tau=1e-4, scale_mode=1)
    lab = lab.cpu().numpy().tolist()
    out["label_counts"] = {nm: lab.count(p) for p, nm in enumerate(("E4M3", "F16", "F32", "F64"))}
    out["choice_matches_labels"] = float(np.mean(np.array(lab) == np.array(choice)))
    out["speedup_learned_vs_fp64"] = out["fp64"]["tts_ms"] / out["learned"]["tts_ms"]
    out["speedup_learned_vs_fixed"] = out["fixed_f16"]["tts_ms"] / out["learned"]["tts_ms"]
    out["speedup_learned_vs_fixed_scaled"] = (out["fixed_f16_scaled"]["tts_ms"] /
                                              out["learned"]["tts_ms"])
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--nmin", type=int, default=1024)
    ap.add_argument("--nmax", type=int, default=8192)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--tau", type=float, default=1e-4)
    ap.add_argument("--leaf", type=int, default=256)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--eval-only", action="store_true", help="evaluate the saved weights")
    ap.add_argument("--mixed-leaves", type=int, default=1,
                    help="1: leaf 64/128/256 per training matrix; 0: the --leaf of every matrix")
    ap.add_argument("--eval-n", type=int, default=32768)
    ap.add_argument("--eval-ratio", type=float, default=1.1)
    args = ap.parse_args(argv)
    import json
    import torch
    ctx = M.Context(0)
    if args.eval_only:
        res = evaluate(ctx, load_params(args.out), args.eval_n, args.eval_ratio, args.leaf)
        print(json.dumps(res), flush=True)
        ctx.close()
        return 0
    tree = policy_tree(args.leaf)
    ns, ratios, seeds = training_recipe(args.count, args.nmin, args.nmax)
    t0 = time.time()
    X, y = build_dataset(ctx, ns, ratios, seeds, tree, args.tau, log_every=max(1, args.count // 20),
                         leaves=leaf_mix(args.count) if args.mixed_leaves else None)
    counts = np.bincount(y.cpu().numpy(), minlength=4)
    print(f"[policy] {X.shape[0]} nodes, label counts E4M3/F16/F32/F64 = {counts.tolist()}, "
          f"{time.time() - t0:.1f} s", flush=True)
    nv = max(1, args.count // 10)
    vns, vr, vs = training_recipe(nv, args.nmin, args.nmax, seed=6)
    Xv, yv = build_dataset(ctx, vns, vr, vs, tree, args.tau,
                           leaves=leaf_mix(nv, seed=8) if args.mixed_leaves else None)
    params, hist = train(ctx, X, y, args.epochs, args.batch, args.lr,
                         log_every=max(1, args.epochs // 10))
    print(f"[policy] train accuracy {accuracy(ctx, X, y, params):.4f}, validation accuracy "
          f"{accuracy(ctx, Xv, yv, params):.4f} ({Xv.shape[0]} nodes of {nv} held-out matrices), "
          f"final loss {hist[-1]:.4f}", flush=True)
    np.save(args.out, params.cpu().numpy().astype(np.float32))
    print(f"[policy] wrote {args.out}", flush=True)
    ctx.close()
    torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
