"""Second, independent formulation of the layered-precision factorization
(TEST INFRASTRUCTURE ONLY, for tiny inputs).

Unrolling Algorithms 1-3 (Section 3.2) shows that every update
``A_IJ -= L_IK L_JK^T`` between leaf blocks (K < J <= I) is issued by exactly one
Tree-POTRF node: the lowest common ancestor of leaf blocks I and K in the
recursion tree (K lies in that node's first half, I and J in its second half).
Section 3.3 gives that node's off-diagonal precision to the update.  So the
whole tree equals a right-looking tile Cholesky over the leaf blocks in which
the update of tile (I, J) by column block K runs in precision
``p(LCA(I, K))`` -- provided quantization is elementwise (all block scales 1),
and up to the grouping of the FP32 accumulation.

This module rebuilds the recursion tree in Python (its own split rule, its own
node numbering) and runs that tile loop with numpy.  It shares nothing with
``mpchol_oracle.c`` except the numeric format definitions, which it
re-implements here from the IEEE/OCP encodings.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

E4M3, F16, F32, F64 = 0, 1, 2, 3


def _split(m: int, align: int) -> int:
    h = m // 2
    if align > 1:
        h = -(-h // align) * align
    return min(max(h, 1), m - 1)


class Node:
    __slots__ = ("start", "size", "depth", "nid", "left", "right")

    def __init__(self, start, size, depth):
        self.start, self.size, self.depth = start, size, depth
        self.nid = -1
        self.left = self.right = None


def build_tree(n: int, leaf: int, align: int = 1) -> Tuple[Node, List[Node]]:
    """Recursion tree of Tree-POTRF; internal nodes numbered in preorder."""
    counter = [0]
    leaves: List[Node] = []

    def rec(start, size, depth):
        nd = Node(start, size, depth)
        if size <= leaf:
            leaves.append(nd)
            return nd
        nd.nid = counter[0]
        counter[0] += 1
        m1 = _split(size, align)
        nd.left = rec(start, m1, depth + 1)
        nd.right = rec(start + m1, size - m1, depth + 1)
        return nd

    root = rec(0, n, 0)
    return root, leaves


def _lca(root: Node, a: int, b: int) -> Node:
    """Deepest node whose range holds both row indices a and b."""
    nd = root
    while nd.left is not None:
        m = nd.left.start + nd.left.size
        if a < m and b < m:
            nd = nd.left
        elif a >= m and b >= m:
            nd = nd.right
        else:
            return nd
    return nd


def _q(x: np.ndarray, prec: int) -> np.ndarray:
    """Round to nearest even in the target format (scale 1)."""
    if prec == F64:
        return x.copy()
    if prec == F32:
        return x.astype(np.float32).astype(np.float64)
    if prec == F16:
        return x.astype(np.float16).astype(np.float64)
    # E4M3 (OCP e4m3fn): 3 fraction bits, smallest normal 2^-6, max 448
    out = np.empty_like(x)
    for idx, v in np.ndenumerate(x):
        if v == 0.0 or not math.isfinite(v):
            out[idx] = v
            continue
        e = max(math.floor(math.log2(abs(v))), -6)
        qn = 2.0 ** (e - 3)
        r = round(abs(v) / qn) * qn      # Python round(): ties to even
        out[idx] = math.copysign(r, v)
    return out


def _acc32(prod_terms: np.ndarray, prec: int) -> np.ndarray:
    """FP32 accumulation of one tile update's k-terms (shape (..., k))."""
    if prec == F32:
        acc = np.zeros(prod_terms.shape[:-1], dtype=np.float32)
        k = prod_terms.shape[-1]
        for q0 in range(0, k, 4):
            chunk = prod_terms[..., q0:q0 + 4].sum(axis=-1)
            acc = (acc.astype(np.float64) + chunk).astype(np.float32)
        return acc.astype(np.float64)
    return prod_terms.sum(axis=-1).astype(np.float32).astype(np.float64)


def factor_lca(A: np.ndarray, n: int, leaf: int, offdiag: Sequence[int],
               leaf_prec: int = F64, align: int = 1, syrk_leaf_mode: int = 0,
               node_prec: Optional[Sequence[int]] = None) -> np.ndarray:
    """Tile Cholesky with the LCA precision rule; returns the lower factor."""
    root, leaves = build_tree(n, leaf, align)
    M = np.array(A[:n, :n], dtype=np.float64)
    T = len(leaves)

    def prec_of(nd: Node) -> int:
        if node_prec is not None and 0 <= nd.nid < len(node_prec) and node_prec[nd.nid] >= 0:
            return node_prec[nd.nid]
        return offdiag[min(nd.depth, len(offdiag) - 1)]

    def sl(t):
        return slice(leaves[t].start, leaves[t].start + leaves[t].size)

    lp32 = leaf_prec == F32
    for K in range(T):
        # leaf POTRF of tile (K, K): Cholesky-Banachiewicz
        kk = sl(K)
        D = M[kk, kk]
        m = D.shape[0]
        Lk = np.zeros_like(D)
        for i in range(m):
            for j in range(i + 1):
                if lp32:
                    s = np.float32(D[i, j])
                    for q in range(j):
                        s = np.float32(s - np.float32(Lk[i, q]) * np.float32(Lk[j, q]))
                    Lk[i, j] = float(np.sqrt(s)) if i == j else float(np.float32(s / np.float32(Lk[j, j])))
                else:
                    s = D[i, j]
                    for q in range(j):
                        s = s - Lk[i, q] * Lk[j, q]
                    Lk[i, j] = math.sqrt(s) if i == j else s / Lk[j, j]
        M[kk, kk] = Lk
        # leaf TRSM of every tile below: x_j = (b_j - sum_q x_q L_jq) / L_jj
        for I in range(K + 1, T):
            ii = sl(I)
            Bt = M[ii, kk].copy()
            for j in range(m):
                if lp32:
                    col = Bt[:, j].astype(np.float32)
                    for q in range(j):
                        col = (col - Bt[:, q].astype(np.float32) * np.float32(Lk[j, q])).astype(np.float32)
                    Bt[:, j] = (col / np.float32(Lk[j, j])).astype(np.float64)
                else:
                    col = Bt[:, j].copy()
                    for q in range(j):
                        col = col - Bt[:, q] * Lk[j, q]
                    Bt[:, j] = col / Lk[j, j]
            M[ii, kk] = Bt
        # trailing updates from column block K
        for J in range(K + 1, T):
            jj = sl(J)
            for I in range(J, T):
                ii = sl(I)
                nd = _lca(root, leaves[I].start, leaves[K].start)
                p = prec_of(nd)
                if I == J and syrk_leaf_mode == 1:
                    p = leaf_prec
                X = M[ii, kk]
                Y = M[jj, kk]
                if p == F64:
                    upd = X @ Y.T
                else:
                    Xq, Yq = _q(X, p), _q(Y, p)
                    upd = _acc32(Xq[:, None, :] * Yq[None, :, :], p)
                if I == J:
                    upd = np.tril(upd)
                    M[ii, jj] = M[ii, jj] - upd
                else:
                    M[ii, jj] = M[ii, jj] - upd
    return np.tril(M)


# --------------------------------------------------------------------------
# Tree-TRSM and Tree-SYRK on their own, as tile loops over the leaf blocks of
# their own recursion tree (the precision list read by that tree's depth).
#
# Tree-TRSM splits only L's order k.  Column block j of B receives, from each
# ancestor node N of leaf j that holds j in its second half, one GEMM over all
# the column blocks of N's first half (the GEMM Algorithm 2 issues at N), in
# the precision of N's depth, outermost ancestor first; then the leaf solve.
# Tree-SYRK splits only C's order n.  Tile (I, J), I > J, of C receives one
# product P_I P_J^T from the GEMM issued at LCA(I, J); a diagonal tile from the
# leaf SYRK reached at its leaf's depth.  Equal to the recursions when every
# block scale is 1, up to the FP64 summation order inside a product.

def _leaf_of(leaves: List[Node], pos: int) -> int:
    for i, lf in enumerate(leaves):
        if lf.start <= pos < lf.start + lf.size:
            return i
    raise ValueError(pos)


def _product(X: np.ndarray, Y: np.ndarray, p: int) -> np.ndarray:
    """X Y^T in precision p (operands rounded, accumulation as in the header)."""
    if p == F64:
        return X @ Y.T
    Xq, Yq = _q(X, p), _q(Y, p)
    return _acc32(Xq[:, None, :] * Yq[None, :, :], p)


def trsm_lca(A: np.ndarray, m: int, k: int, leaf: int, offdiag: Sequence[int],
             leaf_prec: int = F64, align: int = 1) -> np.ndarray:
    """Returns B = A[k:k+m, :k] L^{-T} (L = lower A[:k, :k]) by the tile loop.
    Requires m > leaf (the recursion then splits k down to leaf-sized blocks)."""
    root, leaves = build_tree(k, leaf, align)
    L = np.tril(np.array(A[:k, :k], dtype=np.float64))
    B = np.array(A[k:k + m, :k], dtype=np.float64)
    lp32 = leaf_prec == F32
    for lf in leaves:
        jj = slice(lf.start, lf.start + lf.size)
        # ancestors of this leaf, outermost first, that hold it in their second half
        nd = root
        while nd.left is not None:
            mid = nd.left.start + nd.left.size
            if lf.start >= mid:
                p = offdiag[min(nd.depth, len(offdiag) - 1)]
                ll = slice(nd.left.start, mid)
                B[:, jj] = B[:, jj] - _product(B[:, ll], L[jj, ll], p)
                nd = nd.right
            else:
                nd = nd.left
        # leaf solve, column by column
        Lk = L[jj, jj]
        Bt = B[:, jj].copy()
        for j in range(lf.size):
            if lp32:
                col = Bt[:, j].astype(np.float32)
                for q in range(j):
                    col = (col - Bt[:, q].astype(np.float32) * np.float32(Lk[j, q])).astype(np.float32)
                Bt[:, j] = (col / np.float32(Lk[j, j])).astype(np.float64)
            else:
                col = Bt[:, j].copy()
                for q in range(j):
                    col = col - Bt[:, q] * Lk[j, q]
                Bt[:, j] = col / Lk[j, j]
        B[:, jj] = Bt
    return B


def syrk_lca(A: np.ndarray, n: int, k: int, leaf: int, offdiag: Sequence[int],
             leaf_prec: int = F64, align: int = 1, syrk_leaf_mode: int = 0) -> np.ndarray:
    """Returns the lower triangle of A[k:k+n, k:k+n] - P P^T, P = A[k:k+n, :k],
    by the tile loop (strictly upper triangle zero)."""
    root, leaves = build_tree(n, leaf, align)
    C = np.array(A[k:k + n, k:k + n], dtype=np.float64)
    P = np.array(A[k:k + n, :k], dtype=np.float64)
    for I, li in enumerate(leaves):
        ii = slice(li.start, li.start + li.size)
        for J in range(I + 1):
            lj = leaves[J]
            jj = slice(lj.start, lj.start + lj.size)
            if I == J:
                p = leaf_prec if syrk_leaf_mode else offdiag[min(li.depth, len(offdiag) - 1)]
                C[ii, jj] = C[ii, jj] - np.tril(_product(P[ii], P[jj], p))
            else:
                nd = _lca(root, li.start, lj.start)
                C[ii, jj] = C[ii, jj] - _product(P[ii], P[jj], offdiag[min(nd.depth, len(offdiag) - 1)])
    return np.tril(C)
