"""Pins for the oracle's Tree-TRSM and Tree-SYRK run on their own (CPU only).

The paper times the nested recursive TRSM and SYRK separately (Section 4.2),
with precision lists read by the depth of their own recursion.  Pins:
* integer-exact inputs: every precision list returns the exact result bit for
  bit (FP16 / E4M3 operands and FP32 partial sums are exact on them);
* the all-FP64 list equals the definition (LAPACK's triangular solve, the
  plain product) to a few ulps;
* a second formulation: the tile loop over the recursion's leaf blocks with
  each product in the precision of its lowest common ancestor's depth
  (oracle/tile_lca.py), on random inputs with scale-1 blocks, to 32 u32;
  and a wrong depth assignment moves the result far beyond that tolerance.
"""
import numpy as np
import pytest
from scipy.linalg import solve_triangular

import oracle as O
from oracle import tile_lca

U64 = 2.0 ** -53
U32 = 2.0 ** -24

LISTS = [[O.F64], [O.F16], [O.F16, O.F32], [O.F16, O.F16, O.F32], [O.F32], [O.E4M3, O.F16, O.F32]]


def _trsm_case(m, k, seed, integer):
    rng = np.random.default_rng(seed)
    A = np.zeros((k + m, k + m), order="F")
    if integer:
        L0 = np.tril(rng.integers(-3, 4, (k, k)), -1).astype(np.float64)
        L0[np.arange(k), np.arange(k)] = rng.integers(max(1, k // 2), k + 1, k)
        X0 = rng.integers(-3, 4, (m, k)).astype(np.float64)
        A[:k, :k] = L0
        A[k:, :k] = X0 @ L0.T           # exact: B L0^{-T} = X0
        return A, X0
    L = np.tril(rng.uniform(-1, 1, (k, k)) / k)
    L[np.arange(k), np.arange(k)] = rng.uniform(1, 2, k)
    A[:k, :k] = L
    A[k:, :k] = rng.uniform(-1, 1, (m, k))
    return A, None


@pytest.mark.parametrize("li", range(len(LISTS)))
@pytest.mark.parametrize("m,k,leaf", [(40, 37, 4), (64, 64, 8), (9, 100, 7)])
def test_trsm_integer_exact(li, m, k, leaf):
    A, X0 = _trsm_case(m, k, seed=m + k + li, integer=True)
    lp = O.F32 if LISTS[li][-1] == O.F32 else O.F64
    M, st = O.tree_trsm(A, m, k, O.Tree(leaf=leaf, offdiag=LISTS[li], leaf_prec=lp))
    assert st == O.OK
    np.testing.assert_array_equal(M[k:, :k], X0)
    np.testing.assert_array_equal(M[:k, :k], A[:k, :k])    # L untouched


@pytest.mark.parametrize("li", range(len(LISTS)))
@pytest.mark.parametrize("n,k,leaf", [(37, 20, 4), (64, 64, 8), (100, 9, 16)])
def test_syrk_integer_exact(li, n, k, leaf):
    rng = np.random.default_rng(n * 7 + k + li)
    A = np.asfortranarray(rng.integers(-40, 41, (k + n, k + n)).astype(np.float64))
    A[k:, :k] = rng.integers(-3, 4, (n, k))
    C0, P = A[k:, k:].copy(), A[k:, :k].copy()
    M, st = O.tree_syrk(A, n, k, O.Tree(leaf=leaf, offdiag=LISTS[li]))
    assert st == O.OK
    np.testing.assert_array_equal(np.tril(M[k:, k:]), np.tril(C0 - P @ P.T))
    np.testing.assert_array_equal(np.triu(M[k:, k:], 1), np.triu(C0, 1))   # upper untouched


def test_fp64_lists_equal_definitions():
    m, k = 90, 77
    A, _ = _trsm_case(m, k, seed=3, integer=False)
    M, _ = O.tree_trsm(A, m, k, O.Tree(leaf=6, offdiag=[O.F64]))
    X = solve_triangular(np.tril(A[:k, :k]), A[k:, :k].T, lower=True).T
    assert np.abs(M[k:, :k] - X).max() <= 16 * k * U64 * np.abs(X).max()
    n = 83
    rng = np.random.default_rng(4)
    A = np.asfortranarray(rng.uniform(-1, 1, (k + n, k + n)))
    M, _ = O.tree_syrk(A, n, k, O.Tree(leaf=5, offdiag=[O.F64]))
    want = np.tril(A[k:, k:] - A[k:, :k] @ A[k:, :k].T)
    assert np.abs(np.tril(M[k:, k:]) - want).max() <= 4 * k * U64 * k


@pytest.mark.parametrize("li", range(1, len(LISTS)))
@pytest.mark.parametrize("leaf,align", [(4, 1), (7, 1), (5, 4)])
def test_trsm_recursion_equals_lca_tile_loop(li, leaf, align):
    m, k = 33, 53
    A, _ = _trsm_case(m, k, seed=li * 10 + leaf, integer=False)
    lp = O.F32 if LISTS[li][-1] == O.F32 else O.F64
    M, _ = O.tree_trsm(A, m, k, O.Tree(leaf=leaf, offdiag=LISTS[li], leaf_prec=lp, split_align=align))
    T = tile_lca.trsm_lca(A, m, k, leaf, LISTS[li], leaf_prec=lp, align=align)
    assert np.abs(M[k:, :k] - T).max() <= 32 * U32 * np.abs(T).max()


@pytest.mark.parametrize("li", range(1, len(LISTS)))
@pytest.mark.parametrize("leaf,align,mode", [(4, 1, 0), (7, 1, 0), (5, 4, 1)])
def test_syrk_recursion_equals_lca_tile_loop(li, leaf, align, mode):
    n, k = 45, 30
    rng = np.random.default_rng(li * 3 + leaf)
    A = np.asfortranarray(rng.uniform(-1, 1, (k + n, k + n)))
    tr = O.Tree(leaf=leaf, offdiag=LISTS[li], split_align=align, syrk_leaf_mode=mode)
    M, _ = O.tree_syrk(A, n, k, tr)
    T = tile_lca.syrk_lca(A, n, k, leaf, LISTS[li], align=align, syrk_leaf_mode=mode)
    assert np.abs(np.tril(M[k:, k:]) - T).max() <= 32 * U32 * np.abs(T).max()


def test_depth_rule_is_sharp():
    """Reading the list by the wrong depth (one level shifted) moves both
    results far beyond the cross-check tolerance."""
    m, k, leaf = 33, 53, 4
    A, _ = _trsm_case(m, k, seed=5, integer=False)
    M, _ = O.tree_trsm(A, m, k, O.Tree(leaf=leaf, offdiag=[O.F64, O.F16, O.F64]))
    T = tile_lca.trsm_lca(A, m, k, leaf, [O.F16, O.F64])
    assert np.abs(M[k:, :k] - T).max() > 4 * 32 * U32 * np.abs(T).max()
    n = 45
    rng = np.random.default_rng(6)
    A = np.asfortranarray(rng.uniform(-1, 1, (k + n, k + n)))
    M, _ = O.tree_syrk(A, n, k, O.Tree(leaf=leaf, offdiag=[O.F64, O.F16, O.F64]))
    T = tile_lca.syrk_lca(A, n, k, leaf, [O.F16, O.F64])
    assert np.abs(np.tril(M[k:, k:]) - T).max() > 4 * 32 * U32 * np.abs(T).max()
