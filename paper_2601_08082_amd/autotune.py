"""Autotuner for the batched path: per size bucket, the leaf size, split
alignment and GEMM tile with the shortest measured time to solution.

For each of `buckets` log-spaced size ranges in [nmin, nmax], a batch of
`per_bucket` systems (sizes log-uniform inside the range, dominance ratios
uniform in [1.05, 4], nrhs right-hand sides) is factored, solved and refined
by mpchol_factor_batched under every candidate; the candidate with the
smallest median time over `reps` runs among those whose systems all
converge wins.  Candidates: leaf in {32, 64, 128, 256} (those below the
bucket's top size, at least the smallest) x tile in {64, 128} at the
descriptor's split alignment, then the winner's leaf and tile with split
alignment 16 and 64.  Writes a JSON table for Context.load_tune_table.

    python -m paper_2601_08082_amd.autotune --out paper_2601_08082_amd/tune_mi355x.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

LEAVES = (32, 64, 128, 256)
TILES = (64, 128)
ALIGNS = (16, 64)


def bucket_edges(nmin: int, nmax: int, buckets: int):
    e = [int(round(math.exp(math.log(nmin) + (math.log(nmax) - math.log(nmin)) * i / buckets)))
         for i in range(buckets + 1)]
    return [(max(nmin, e[i - 1] + 1) if i > 1 else nmin, e[i]) for i in range(1, buckets + 1)]


def run(args) -> dict:
    import torch
    from . import mpchol as M
    from .workloads import DeviceBatch, batch_recipe

    ctx = M.Context(0)
    tree = M.Tree(leaf=64, offdiag=[M.F16], leaf_prec=M.F64, split_align=args.split_align)
    entries = []
    for bi, (lo, hi) in enumerate(bucket_edges(args.nmin, args.nmax, args.buckets)):
        ns, ratios, seeds = batch_recipe(args.per_bucket, lo, hi, 1.05, 4.0, seed=900 + bi)
        db = DeviceBatch(ns, ratios, seeds, args.nrhs)

        def timed(leaf, align, tile):
            ctx.set_tune_table([(1 << 20, leaf, align, tile)])
            ms = []
            for r in range(args.reps + 1):
                st, infos = ctx.factor_batched(db.A, db.L, db.ns, tree, db.B, db.X,
                                               tol=1e-13, max_iter=20)
                ms.append(infos[0]["ms_factor"])          # HIP events around the launch
                if st != 0:
                    return None
            ms = sorted(ms[1:])
            return ms[len(ms) // 2]

        cands = {}
        leaves = [b for b in LEAVES if b < hi] or [LEAVES[0]]
        for leaf in leaves:
            for tile in TILES:
                cands[(leaf, args.split_align, tile)] = timed(leaf, args.split_align, tile)
        ok = {k: v for k, v in cands.items() if v is not None}
        if not ok:
            raise RuntimeError(f"bucket {lo}..{hi}: no candidate converged")
        leaf, _, tile = min(ok, key=ok.get)
        for al in ALIGNS:
            cands[(leaf, al, tile)] = timed(leaf, al, tile)
        ok = {k: v for k, v in cands.items() if v is not None}
        best = min(ok, key=ok.get)
        entries.append({"nmin": lo, "nmax": hi, "leaf": best[0], "split_align": best[1],
                        "tile": best[2], "ms": ok[best],
                        "candidates": {f"b{k[0]}_a{k[1]}_t{k[2]}": v for k, v in cands.items()}})
        print(f"[autotune] {lo}..{hi}: leaf {best[0]} align {best[1]} tile {best[2]} "
              f"{ok[best]:.3f} ms", flush=True)
        del db
        torch.cuda.empty_cache()
    ctx.set_tune_table([])
    ctx.close()
    return {"device": torch.cuda.get_device_name(0), "per_bucket": args.per_bucket,
            "nrhs": args.nrhs, "reps": args.reps, "tree": "offdiag [F16], leaf FP64",
            "entries": entries}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "tune_mi355x.json"))
    ap.add_argument("--nmin", type=int, default=64)
    ap.add_argument("--nmax", type=int, default=2048)
    ap.add_argument("--buckets", type=int, default=16)
    ap.add_argument("--per-bucket", type=int, default=256)
    ap.add_argument("--nrhs", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--split-align", type=int, default=32)
    args = ap.parse_args(argv)
    tab = run(args)
    with open(args.out, "w") as f:
        json.dump(tab, f, indent=1)
    print(f"[autotune] wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
