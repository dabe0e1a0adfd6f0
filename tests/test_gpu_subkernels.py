"""GPU parity of Tree-TRSM and Tree-SYRK run on their own (mpchol_trsm /
mpchol_syrk) against the oracle's orc_tree_trsm / orc_tree_syrk.

* Integer-exact inputs: every precision list returns the exact result bit for
  bit (substitution leaf TRSMs); with the inverse-based FP64 leaf TRSM within
  1e-13 relative.  Sizes span several output tiles with ragged tails, and one
  SYRK is large enough for the 256 x 256 FP16 tile kernel.
* Random inputs: the all-FP64 list within 1e-13 of the oracle; mixed lists
  within a quarter of the emulation's own distance from the FP64 result (the
  GPU and the emulation share the operand quantization and differ only in the
  FP32 accumulation order).
"""
import numpy as np
import pytest

import oracle as O

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


LISTS = [[3], [1], [1, 2], [1, 1, 2], [0, 1, 2]]   # F64, F16, [F16,F32], [F16,F16,F32], [E4M3,F16,F32]


def _tree(M, offdiag, leaf, leaf_trsm=0, mode=0):
    lp = M.F32 if offdiag[-1] == M.F32 else M.F64
    return M.Tree(leaf=leaf, offdiag=list(offdiag), leaf_prec=lp, leaf_trsm=leaf_trsm,
                  syrk_leaf_mode=mode, scale_mode=1 if offdiag[0] == M.E4M3 else 0)


def _otree(t):
    return O.Tree(leaf=t.leaf, offdiag=list(t.offdiag), leaf_prec=t.leaf_prec,
                  syrk_leaf_mode=t.syrk_leaf_mode, scale_mode=t.scale_mode)


def _trsm_input(m, k, seed, integer):
    rng = np.random.default_rng(seed)
    A = np.zeros((k + m, k + m), order="F")
    if integer:
        L0 = np.tril(rng.integers(-3, 4, (k, k)), -1).astype(np.float64)
        L0[np.arange(k), np.arange(k)] = rng.integers(max(1, k // 2), k + 1, k)
        X0 = rng.integers(-3, 4, (m, k)).astype(np.float64)
        A[:k, :k] = L0
        A[k:, :k] = X0 @ L0.T
        return A, X0
    L = np.tril(rng.uniform(-1, 1, (k, k)) / np.sqrt(k))
    L[np.arange(k), np.arange(k)] = rng.uniform(1, 2, k)
    A[:k, :k] = L
    A[k:, :k] = rng.uniform(-1, 1, (m, k))
    return A, None


@pytest.mark.parametrize("li", range(len(LISTS)))
@pytest.mark.parametrize("m,k,leaf", [(1500, 1100, 128), (777, 2100, 256), (300, 129, 64)])
def test_trsm_integer_exact(M, ctx, li, m, k, leaf):
    print(f"[gpu] trsm integer m={m} k={k} leaf={leaf} list={LISTS[li]}", flush=True)
    A, X0 = _trsm_input(m, k, seed=m + k + li, integer=True)
    for leaf_trsm in (1, 0):
        t = _tree(M, LISTS[li], leaf, leaf_trsm=leaf_trsm)
        Ad = M.to_device_cm(A)
        info = ctx.trsm(Ad, m, k, t)
        assert info["status"] == M.OK, info
        R = M.from_device_cm(Ad)
        np.testing.assert_array_equal(R[:k, :k], A[:k, :k])
        if leaf_trsm == 1 or t.leaf_prec == M.F32:
            np.testing.assert_array_equal(R[k:, :k], X0)
        else:
            assert np.abs(R[k:, :k] - X0).max() <= 1e-13 * np.abs(X0).max()


@pytest.mark.parametrize("li", range(len(LISTS)))
@pytest.mark.parametrize("n,k,leaf", [(1300, 700, 128), (2100, 333, 256), (8192, 1024, 256)])
def test_syrk_integer_exact(M, ctx, li, n, k, leaf):
    if n == 8192 and li not in (1, 2):
        pytest.skip("the 256-tile case runs for the FP16 lists")
    print(f"[gpu] syrk integer n={n} k={k} leaf={leaf} list={LISTS[li]}", flush=True)
    rng = np.random.default_rng(n + k + li)
    A = np.asfortranarray(rng.integers(-40, 41, (k + n, k + n)).astype(np.float64))
    A[k:, :k] = rng.integers(-3, 4, (n, k))
    want = A[k:, k:] - A[k:, :k] @ A[k:, :k].T       # exact integers
    t = _tree(M, LISTS[li], leaf)
    Ad = M.to_device_cm(A)
    info = ctx.syrk(Ad, n, k, t)
    assert info["status"] == M.OK, info
    R = M.from_device_cm(Ad)
    np.testing.assert_array_equal(np.tril(R[k:, k:]), np.tril(want))
    np.testing.assert_array_equal(np.triu(R[k:, k:], 1), np.triu(A[k:, k:], 1))
    np.testing.assert_array_equal(R[:, :k], A[:, :k])


@pytest.mark.parametrize("li", range(len(LISTS)))
def test_trsm_random_against_oracle(M, ctx, li):
    m, k, leaf = 1200, 900, 128
    print(f"[gpu] trsm random m={m} k={k} list={LISTS[li]}", flush=True)
    A, _ = _trsm_input(m, k, seed=40 + li, integer=False)
    t = _tree(M, LISTS[li], leaf)
    Ad = M.to_device_cm(A)
    assert ctx.trsm(Ad, m, k, t)["status"] == M.OK
    Bg = M.from_device_cm(Ad)[k:, :k]
    E, st = O.tree_trsm(A, m, k, _otree(t))
    assert st == O.OK
    Be = E[k:, :k]
    B64 = O.tree_trsm(A, m, k, O.Tree(leaf=leaf, offdiag=[O.F64]))[0][k:, :k]
    if LISTS[li] == [3]:
        assert np.linalg.norm(Bg - Be) <= 1e-13 * np.linalg.norm(Be)
    else:
        assert np.linalg.norm(Bg - Be) <= 0.25 * np.linalg.norm(Be - B64)


@pytest.mark.parametrize("li", range(len(LISTS)))
@pytest.mark.parametrize("mode", [0, 1])
def test_syrk_random_against_oracle(M, ctx, li, mode):
    n, k, leaf = 1100, 500, 128
    print(f"[gpu] syrk random n={n} k={k} list={LISTS[li]} mode={mode}", flush=True)
    rng = np.random.default_rng(60 + li + 7 * mode)
    A = np.asfortranarray(rng.uniform(-1, 1, (k + n, k + n)))
    t = _tree(M, LISTS[li], leaf, mode=mode)
    Ad = M.to_device_cm(A)
    assert ctx.syrk(Ad, n, k, t)["status"] == M.OK
    Cg = np.tril(M.from_device_cm(Ad)[k:, k:])
    E, st = O.tree_syrk(A, n, k, _otree(t))
    assert st == O.OK
    Ce = np.tril(E[k:, k:])
    C64 = np.tril(A[k:, k:] - A[k:, :k] @ A[k:, :k].T)
    if LISTS[li] == [3]:
        assert np.linalg.norm(Cg - Ce) <= 1e-13 * np.linalg.norm(Ce)
    else:
        assert np.linalg.norm(Cg - Ce) <= 0.25 * np.linalg.norm(Ce - C64)
