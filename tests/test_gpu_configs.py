"""GPU parity at the sizes and trees of the benchmarked workloads.

* n = 16384, ratio 1.5, tree [F16, F16, F32 x 4], leaf 256 (the 16384
  benchmark): the GPU factor against the oracle's emulation of the same tree:
  backward error within 2x (0.5 <= be_gpu / be_emu <= 2) and
  ||L - L_emu||_F <= 1/4 ||L_emu - L_64||_F, with L_64 the FP64 Cholesky factor
  (LAPACK through numpy, equal to the oracle's FP64 tree to ~n u); refined
  solution within 1e-12 of the FP64 solution.
* n = 16384, ratio 1.2, tree [F16, F32, F64], leaf 256, 16 right-hand sides
  (the three-level tree of the 65536 benchmark at a size the oracle finishes):
  the same bars.
* n = 65536 with that tree (the benchmark itself, too large for the CPU
  oracle): the device backward error (checked against an independent FP64
  product computed with torch), the element-wise bound below on sampled
  entries, and the Gershgorin certificate of the refined solution of all 16
  right-hand sides <= 1e-12.

Element-wise bound for a tree whose lowest precision is FP16 (scale 1): every
product L_ik L_jk of the update of entry (i, j) uses operands rounded to FP16
(relative error <= u16 = 2^-11 each, or absolute 2^-25 in FP16's subnormal
range) and is summed in FP32 over at most K = n / 2 terms, so
  |A - L L^T|_ij <= (2 u16 + K u32) (|L| |L|^T)_ij + 2^-25 (||L_i||_1 + ||L_j||_1)
up to FP64 terms (the leaves, the FP64 epilogue), which the slack covers.

Backward errors and the products behind them are computed with torch (FP64
matrix products on the GPU), the same function for the GPU factor and the
emulated one.
"""
import numpy as np
import pytest

import oracle as O
from paper_2601_08082_amd import spdgen

pytestmark = pytest.mark.gpu

U16, U32 = 2.0 ** -11, 2.0 ** -24


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2601_08082_amd import mpchol
    return mpchol


@pytest.fixture(scope="module")
def ctx(M):
    c = M.Context(0)
    yield c
    c.close()


def _true_lower(Ld, n):
    """The lower triangle of a column-major device factor as a row-major
    torch matrix (the buffer's upper triangle is not part of the factor)."""
    return Ld[:n, :n].T.contiguous().tril_()


def _be(A, L):
    """||A - L L^T||_F / ||A||_F in FP64 on the GPU (A full symmetric)."""
    import torch
    E = A - L @ L.T
    return float(torch.linalg.norm(E) / torch.linalg.norm(A))


def _elementwise_ratio(A, L, n, sample=None):
    """max over (i, j) of |A - L L^T|_ij / bound_ij (bound in the module
    docstring); sample: None = all entries, else (I, J) index arrays."""
    import torch
    cu = 2 * U16 + (n // 2) * U32 + 1e-12
    if sample is None:
        aL = L.abs()
        s = aL.sum(dim=1)
        E = (A - L @ L.T).abs()
        bound = cu * (aL @ aL.T) + 2.0 ** -25 * (s[:, None] + s[None, :])
        return float((E / bound).max())
    I, J = sample
    Ii = torch.as_tensor(I, device=A.device)
    Jj = torch.as_tensor(J, device=A.device)
    Li, Lj = L[Ii], L[Jj]
    llt = (Li * Lj).sum(dim=1)
    E = (A[Ii, Jj] - llt).abs()
    si, sj = Li.abs().sum(dim=1), Lj.abs().sum(dim=1)
    bound = cu * (Li.abs() * Lj.abs()).sum(dim=1) + 2.0 ** -25 * (si + sj)
    return float((E / bound).max())


def _relerr(X, Xs):
    return float(np.max(np.linalg.norm(X - Xs, axis=0) / np.linalg.norm(Xs, axis=0)))


@pytest.mark.parametrize("name,ratio,levels,nrhs", [
    ("16384 benchmark tree", 1.5, [1, 1, 2, 2, 2, 2], 1),
    ("three-level tree", 1.2, [1, 2, 3], 16),
])
def test_n16384_against_emulation(M, ctx, name, ratio, levels, nrhs):
    import torch
    n, leaf = 16384, 256
    print(f"[gpu] n={n} {name}: generating and emulating on the CPU", flush=True)
    A = spdgen.gen_spd(n, ratio, 0.0, seed=8)
    B = spdgen.gen_rhs(n, nrhs, seed=108)
    Le, so, _ = O.factor(A, tree=O.Tree(leaf=leaf, offdiag=list(levels)))
    assert so == O.OK
    L64 = np.linalg.cholesky(A)            # lower; the unique FP64 factor
    print(f"[gpu] n={n} {name}: GPU factor + refined solve", flush=True)
    Ad = M.to_device_cm(A)
    Ld, info = ctx.factor(Ad, n, M.Tree(leaf=leaf, offdiag=list(levels), leaf_prec=M.F64))
    assert info["status"] == 0
    Xd, sinfo = ctx.solve(Ld, M.to_device_cm(B), n, A_cm=Ad, tol=1e-13, max_iter=20)
    assert sinfo["status"] == 0, sinfo
    X = M.from_device_cm(Xd)[:n]
    dev = torch.device("cuda")
    At = torch.as_tensor(A, device=dev)    # symmetric: layout does not matter
    Lg = _true_lower(Ld, n)
    Lem = torch.tril(torch.as_tensor(np.ascontiguousarray(Le), device=dev))
    L64t = torch.as_tensor(np.ascontiguousarray(L64), device=dev)
    be_g, be_e = _be(At, Lg), _be(At, Lem)
    print(f"[gpu]   backward error gpu {be_g:.3e} emulation {be_e:.3e}", flush=True)
    assert 0.5 <= be_g / be_e <= 2.0, (be_g, be_e)
    d_ge = float(torch.linalg.norm(Lg - Lem))
    d_e64 = float(torch.linalg.norm(Lem - L64t))
    assert d_ge <= 0.25 * d_e64, (d_ge, d_e64)
    if levels[0] == M.F16:
        r = _elementwise_ratio(At, Lg, n)
        print(f"[gpu]   element-wise |A - LL^T| / bound max {r:.3e}", flush=True)
        assert r <= 1.0
    from scipy.linalg import cho_solve
    Xs = cho_solve((L64, True), B)         # the FP64 solution
    assert _relerr(X, Xs) <= 1e-12


def test_n65536_three_level_tree(M, ctx):
    """The 65536 benchmark: ratio 1.2, [F16, F32, F64], leaf 256, 16 rhs."""
    import torch
    from paper_2601_08082_amd import spdgen_gpu
    n, ratio, nrhs = 65536, 1.2, 16
    print(f"[gpu] n={n}: generate, factor, refined solve", flush=True)
    Ad = spdgen_gpu.gen_spd(n, ratio, 0.0, 8, n)
    Bd = spdgen_gpu.gen_rhs(n, nrhs, 108, n)
    Ld, info = ctx.factor(Ad, n, M.Tree(leaf=256, offdiag=[M.F16, M.F32, M.F64], leaf_prec=M.F64))
    assert info["status"] == 0
    Xd, sinfo = ctx.solve(Ld, Bd, n, A_cm=Ad, tol=1e-13, max_iter=20)
    assert sinfo["status"] == 0, sinfo
    torch.cuda.synchronize()
    # device backward error against an independent FP64 product (torch), by
    # row blocks of the factor (torch kernels take at most 2^31 elements)
    be_dev, _, _ = ctx.backward_error(Ad, Ld, n)
    print(f"[gpu]   device backward error {be_dev:.3e}", flush=True)
    A = Ad[:n, :n]                          # symmetric
    R0 = 4096
    L = torch.empty((n, n), dtype=torch.float64, device=Ad.device)
    for r0 in range(0, n, R0):               # rows of L = columns of the buffer, lower part
        L[r0:r0 + R0] = torch.tril(Ld[:n, r0:r0 + R0].T, diagonal=r0)
    del Ld
    torch.cuda.empty_cache()
    ss = aa = 0.0
    rowabs = torch.empty(n, dtype=torch.float64, device=A.device)
    for r0 in range(0, n, R0):
        Ab = A[r0:r0 + R0]
        E = Ab - L[r0:r0 + R0] @ L.T
        ss += float((E * E).sum())
        aa += float((Ab * Ab).sum())
        rowabs[r0:r0 + R0] = Ab.abs().sum(dim=1)
        del E
    be_t = float(np.sqrt(ss / aa))
    print(f"[gpu]   torch backward error {be_t:.3e}", flush=True)
    assert abs(be_dev - be_t) <= 1e-3 * be_t
    assert 1e-12 < be_t <= 1e-7
    # element-wise bound on sampled entries (diagonal and off-diagonal)
    rng = np.random.default_rng(1)
    I = rng.integers(0, n, 4000)
    J = rng.integers(0, n, 4000)
    I[:200] = J[:200]
    r = _elementwise_ratio(A, L, n, sample=(np.maximum(I, J), np.minimum(I, J)))
    print(f"[gpu]   sampled element-wise ratio {r:.3e}", flush=True)
    assert r <= 1.0
    # Gershgorin certificate ||x - x*|| <= ||b - A x|| / lambda_min (FP64)
    X = Xd[:nrhs, :n]                      # row c = right-hand side c
    R = Bd[:nrhs, :n] - X @ A
    dg = torch.diagonal(A)
    lam = float(torch.min(dg - (rowabs - dg.abs())))
    assert lam > 0
    cert = torch.linalg.vector_norm(R, dim=1) / lam / torch.linalg.vector_norm(X, dim=1)
    print(f"[gpu]   certificate {float(cert.max()):.3e}", flush=True)
    assert float(cert.max()) <= 1e-12


@pytest.mark.parametrize("e", [0, 22])
def test_integer_bitwise_n16384_256_tiles(M, ctx, e):
    """n = 16384 with leaf 256: the level-0 FP16 groups run the 256 x 256 tile
    kernel.  A = 4^e L0 L0^T (L0 integer, off-diagonal in [-3, 3]) has the
    factor 2^e L0 bit for bit: every FP16 operand (scaled by a power of two
    when 3 * 2^e exceeds the format's range, e = 22: the kernel's path that
    quantizes from the factor on the way in) and every FP32 partial sum is
    exact."""
    import torch
    n = 16384
    print(f"[gpu] integer L0 n={n} scale 2^{e}", flush=True)
    assert M.plan_stats(n, M.Tree(leaf=256, offdiag=[M.F16]))["launches"] > 0
    g = torch.Generator(device="cpu").manual_seed(99)
    L0 = torch.tril(torch.randint(-3, 4, (n, n), generator=g, dtype=torch.int8), -1).to(torch.float64)
    L0 += torch.diag(torch.randint(n // 2, n + 1, (n,), generator=g).to(torch.float64))
    L0d = torch.ldexp(L0.cuda(), torch.tensor(e, dtype=torch.float64, device="cuda"))
    del L0
    A = (L0d @ L0d.T.contiguous()).contiguous()   # exact: entries < 2^53
    t = M.Tree(leaf=256, offdiag=[M.F16], leaf_trsm=1)
    L, info = ctx.factor(A, n, t)
    assert info["status"] == M.OK, info
    assert torch.equal(torch.tril(L.T), L0d)


def _tuned(n, table):
    for e in table:
        if n <= e["nmax"]:
            return e
    return None


@pytest.mark.parametrize("nrhs", [4, 5, 16])
def test_batched_tuned_sizes_against_oracle(M, ctx, nrhs):
    """Systems across the whole batched size range [64, 2048] (every bucket of
    the committed tune table at nrhs 4, a few sizes at 5 and 16 rhs), solved by
    the persistent batched launch under that table: each against the oracle
    run with its tuned leaf and split alignment."""
    import json
    import os
    import torch
    path = os.path.join(os.path.dirname(M.__file__), "tune_mi355x.json")
    table = json.load(open(path))["entries"]
    if nrhs == 4:
        sizes = []
        for e in table:
            sizes += sorted({e["nmin"], (e["nmin"] + e["nmax"]) // 2, e["nmax"]})
        sizes = sorted(set(sizes))
    else:
        sizes = [64, 333, 1100, 1700, 2048]
    rng = np.random.default_rng(nrhs)
    ratios = rng.uniform(1.05, 4.0, len(sizes))
    print(f"[gpu] batched tuned sizes nrhs={nrhs}: {len(sizes)} systems up to {max(sizes)}",
          flush=True)
    mats = [spdgen.gen_spd(n, float(r), 0.0, seed=700 + i) for i, (n, r) in enumerate(zip(sizes, ratios))]
    rhs = [spdgen.gen_rhs(n, nrhs, seed=900 + i) for i, n in enumerate(sizes)]
    A = [M.to_device_cm(a) for a in mats]
    L = [torch.zeros_like(a) for a in A]
    B = [M.to_device_cm(b) for b in rhs]
    X = [torch.zeros_like(b) for b in B]
    t = M.Tree(leaf=64, offdiag=[M.F16], leaf_prec=M.F64, split_align=32)
    ctx.load_tune_table(path)
    try:
        st, infos = ctx.factor_batched(A, L, sizes, t, B, X, tol=1e-13, max_iter=20)
    finally:
        ctx.set_tune_table([])
    assert st == 0, [x for x in infos if x["status"]]
    for i, n in enumerate(sizes):
        e = _tuned(n, table)
        ot = O.Tree(leaf=e["leaf"], offdiag=[O.F16], split_align=e["split_align"] or 32)
        Le, so, _ = O.factor(mats[i], tree=ot)
        assert so == O.OK
        L64 = np.linalg.cholesky(mats[i])
        Lg = np.tril(M.from_device_cm(L[i]))
        if n > e["leaf"]:
            # mixed work: backward error within 2x, factor distance bar
            be_g, be_e = O.backward_error(mats[i], Lg), O.backward_error(mats[i], Le)
            assert 0.5 <= be_g / be_e <= 2.0, (n, e["leaf"], be_g, be_e)
            assert np.linalg.norm(Lg - np.tril(Le)) <= 0.25 * np.linalg.norm(np.tril(Le) - L64), n
        else:
            # a single FP64 leaf: the FP64 factor
            assert np.linalg.norm(Lg - np.tril(Le)) <= 1e-13 * np.linalg.norm(L64), n
        xs = np.linalg.solve(mats[i], rhs[i])
        x = M.from_device_cm(X[i])[:n]
        assert _relerr(x, xs) <= 1e-12, (n, infos[i])
