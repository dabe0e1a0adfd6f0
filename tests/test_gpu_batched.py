"""GPU parity of the persistent batched factor + refined solve (one launch for
many systems of uneven sizes) against the CPU oracle.

Bars: integer-exact systems bit for bit; FP64 tree within 1e-13 of the oracle;
mixed trees: backward error within 2x of the oracle's emulation of the same
tree, factor distance at most a quarter of the emulation's distance to FP64;
refined solutions within 1e-12 of the FP64 solution; a non-SPD member reports
its own pivot index without disturbing the others.
"""
import numpy as np
import pytest

import oracle as O
from paper_2601_08082_amd import spdgen

pytestmark = pytest.mark.gpu


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


def _batch(M, mats, nrhs, seed=0):
    import torch
    A = [M.to_device_cm(a) for a in mats]
    L = [torch.zeros_like(a) for a in A]
    B, X, Bh = [], [], []
    for i, a in enumerate(mats):
        n = a.shape[1]
        b = spdgen.gen_rhs(n, nrhs, seed=500 + seed + i)
        Bh.append(b)
        B.append(M.to_device_cm(b))
        X.append(torch.zeros_like(B[-1]))
    return A, L, B, X, Bh


def _otree(t, leaf=None):
    return O.Tree(leaf=leaf or t.leaf, offdiag=list(t.offdiag), leaf_prec=t.leaf_prec,
                  split_align=t.split_align, syrk_leaf_mode=t.syrk_leaf_mode,
                  scale_mode=t.scale_mode)


def test_batched_mixed_ragged(M, ctx):
    print("[gpu] batched mixed ragged", flush=True)
    rng = np.random.default_rng(3)
    sizes = [1, 7, 33, 64, 65, 100, 129, 200, 257, 300, 511] + list(rng.integers(20, 400, 9))
    ratios = list(rng.uniform(1.05, 4.0, len(sizes)))
    mats = [spdgen.gen_spd(int(n), float(r), 0.5, seed=40 + i) for i, (n, r) in enumerate(zip(sizes, ratios))]
    t = M.Tree(leaf=64, offdiag=[M.F16], split_align=32)
    A, L, B, X, Bh = _batch(M, mats, 4)
    st, infos = ctx.factor_batched(A, L, sizes, t, B, X, tol=1e-13, max_iter=20)
    assert st == 0, infos
    for i, n in enumerate(sizes):
        n = int(n)
        Lg = M.from_device_cm(L[i])
        Le, so, _ = O.factor(mats[i], tree=_otree(t))
        L64, _, _ = O.factor(mats[i], tree=O.Tree(leaf=64, offdiag=[O.F64]))
        be_g, be_e = O.backward_error(mats[i], Lg), O.backward_error(mats[i], Le)
        if be_e > 1e-15:
            assert 0.5 <= be_g / be_e <= 2.0, (n, be_g, be_e)
            assert np.linalg.norm(np.tril(Lg) - np.tril(Le)) <= 0.25 * np.linalg.norm(np.tril(Le) - np.tril(L64)), n
        xs = np.linalg.solve(mats[i][:n, :n], Bh[i][:n])
        x = M.from_device_cm(X[i])[:n]
        err = np.max(np.linalg.norm(x - xs, axis=0) / np.linalg.norm(xs, axis=0))
        assert err <= 1e-12, (n, err, infos[i])
        assert infos[i]["status"] == 0


def test_batched_fp64_and_integer(M, ctx):
    print("[gpu] batched fp64 + integer", flush=True)
    sizes = [5, 90, 130, 260]
    mats = [spdgen.gen_spd(n, 1.3, 0.5, seed=n) for n in sizes]
    t = M.Tree(leaf=64, offdiag=[M.F64])
    A, L, B, X, Bh = _batch(M, mats, 1)
    st, infos = ctx.factor_batched(A, L, sizes, t, B, X)
    assert st == 0
    for i, n in enumerate(sizes):
        Lo, _, _ = O.factor(mats[i], tree=_otree(t))
        Lg = M.from_device_cm(L[i])
        assert np.linalg.norm(np.tril(Lg) - np.tril(Lo)) <= 1e-13 * np.linalg.norm(np.tril(Lo))
    # integer-exact systems: every tree returns L0 bit for bit
    rng = np.random.default_rng(9)
    L0s, As = [], []
    for n in (3, 70, 150):
        L0 = np.tril(rng.integers(-3, 4, (n, n)), -1).astype(np.int64)
        L0[np.arange(n), np.arange(n)] = rng.integers(max(1, n // 2), n + 1, n)
        L0s.append(L0.astype(np.float64))
        As.append(np.asfortranarray((L0 @ L0.T).astype(np.float64)))
    for t in (M.Tree(leaf=32, offdiag=[M.F16, M.F32]), M.Tree(leaf=16, offdiag=[M.E4M3], scale_mode=1)):
        A, L, _, _, _ = _batch(M, As, 1)
        st, infos = ctx.factor_batched(A, L, [a.shape[1] for a in As], t)
        assert st == 0
        for i, L0 in enumerate(L0s):
            np.testing.assert_array_equal(np.tril(M.from_device_cm(L[i])), L0)


def test_batched_not_spd_member(M, ctx):
    sizes = [100, 120, 80]
    mats = [spdgen.gen_spd(n, 1.5, 0.0, seed=n) for n in sizes]
    mats[1][57, 57] = -3.0
    t = M.Tree(leaf=32, offdiag=[M.F16])
    A, L, B, X, Bh = _batch(M, mats, 2)
    st, infos = ctx.factor_batched(A, L, sizes, t, B, X)
    _, so, fi = O.factor(mats[1], tree=_otree(t))
    assert st == M.NOT_SPD and so == O.NOT_SPD
    assert infos[1]["status"] == M.NOT_SPD and infos[1]["failed_index"] == fi == 58
    assert infos[0]["status"] == 0 and infos[2]["status"] == 0


def test_batched_tune_table_and_replay(M, ctx):
    sizes = [60, 150, 300, 40]
    mats = [spdgen.gen_spd(n, 2.0, 0.0, seed=n + 1) for n in sizes]
    t = M.Tree(leaf=64, offdiag=[M.F16], split_align=32)
    ctx.set_tune_table([(64, 32, 0, 0), (200, 48, 16, 64)])
    try:
        A, L, B, X, Bh = _batch(M, mats, 3)
        for rep in range(2):                     # second call replays the captured graph
            st, infos = ctx.factor_batched(A, L, sizes, t, B, X)
            assert st == 0
        for i, n in enumerate(sizes):
            leaf, al = (32, 32) if n <= 64 else ((48, 16) if n <= 200 else (64, 32))
            ot = _otree(t, leaf)
            ot.split_align = al
            Le, _, _ = O.factor(mats[i], tree=ot)
            Lg = M.from_device_cm(L[i])
            be_g, be_e = O.backward_error(mats[i], Lg), O.backward_error(mats[i], Le)
            assert 0.5 <= be_g / be_e <= 2.0, (n, leaf, be_g, be_e)
    finally:
        ctx.set_tune_table([])
