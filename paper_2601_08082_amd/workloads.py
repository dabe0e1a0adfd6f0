"""Synthetic batched workloads: many SPD systems of uneven sizes, generated
directly into device memory with the seeded generator (input generation only).

batch_recipe(count, nmin, nmax, rmin, rmax, seed): sizes log-uniform in
[nmin, nmax] (n = round(exp(U[ln nmin, ln nmax]))), dominance ratios uniform
in [rmin, rmax]; the per-system matrix seed is seed * 1_000_003 + i, the
right-hand-side seed that plus 500_000.
"""
from __future__ import annotations

import math

import numpy as np


def batch_recipe(count: int, nmin: int = 64, nmax: int = 2048, rmin: float = 1.05,
                 rmax: float = 4.0, seed: int = 4):
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))).astype(np.int64)
    ns = np.clip(ns, nmin, nmax)
    ratios = rng.uniform(rmin, rmax, count)
    seeds = [seed * 1_000_003 + i for i in range(count)]
    return [int(n) for n in ns], [float(r) for r in ratios], seeds


class DeviceBatch:
    """A, L (n_i x n_i, ld n_i) and B, X (n_i x nrhs, ld n_i) for every system,
    carved out of four device buffers; lists of per-system tensor views in the
    (cols, ld) layout of mpchol.to_device_cm."""

    def __init__(self, ns, ratios, seeds, nrhs: int, device="cuda"):
        import torch
        from . import spdgen_gpu
        lib = spdgen_gpu._get()
        self.ns = list(ns)
        self.nrhs = nrhs
        tot = sum(n * n for n in ns)
        totb = sum(n for n in ns) * max(nrhs, 1)
        self.Abuf = torch.empty(tot, dtype=torch.float64, device=device)
        self.Lbuf = torch.zeros(tot, dtype=torch.float64, device=device)
        self.Bbuf = torch.empty(totb, dtype=torch.float64, device=device)
        self.Xbuf = torch.zeros(totb, dtype=torch.float64, device=device)
        s = torch.cuda.current_stream().cuda_stream
        self.A, self.L, self.B, self.X = [], [], [], []
        oa = ob = 0
        for n, r, sd in zip(ns, ratios, seeds):
            a = self.Abuf[oa:oa + n * n].view(n, n)
            if lib.spdgen_fill(n, n, r, 0.0, sd, a.data_ptr(), s) != 0:
                raise RuntimeError("spdgen_fill failed")
            self.A.append(a)
            self.L.append(self.Lbuf[oa:oa + n * n].view(n, n))
            b = self.Bbuf[ob:ob + n * max(nrhs, 1)].view(max(nrhs, 1), n)
            if nrhs and lib.spdgen_rhs(n, nrhs, n, sd + 500_000, b.data_ptr(), s) != 0:
                raise RuntimeError("spdgen_rhs failed")
            self.B.append(b)
            self.X.append(self.Xbuf[ob:ob + n * max(nrhs, 1)].view(max(nrhs, 1), n))
            oa += n * n
            ob += n * max(nrhs, 1)
        torch.cuda.synchronize()

    def flops(self) -> float:
        return float(sum(n ** 3 for n in self.ns)) / 3.0
