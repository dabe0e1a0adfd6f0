"""Python view of the CPU oracle (TEST INFRASTRUCTURE ONLY).

The oracle is plain C in ``mpchol_oracle.c``: Tree-POTRF / Tree-TRSM / Tree-SYRK
(Section 3.2, Algorithms 1-3) with the layered precision of Section 3.3 and the
per-block quantization of Section 3.4, plus substitution solves, FP64-residual
iterative refinement and the backward-error checker.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use it; the
GPU library never links or imports it.

Matrices are numpy arrays in Fortran (column-major) order, shape (lda, n).
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

E4M3, F16, F32, F64 = 0, 1, 2, 3
OK, NOT_SPD, NONFINITE, NOT_CONVERGED = 0, 1, 2, 3
PREC_NAMES = {E4M3: "E4M3", F16: "F16", F32: "F32", F64: "F64"}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Tree(ct.Structure):
    _fields_ = [
        ("leaf", ct.c_int32),
        ("split_align", ct.c_int32),
        ("nlevels", ct.c_int32),
        ("offdiag", ct.c_int32 * 24),
        ("leaf_prec", ct.c_int32),
        ("syrk_leaf_mode", ct.c_int32),
        ("scale_mode", ct.c_int32),
        ("node_prec", ct.POINTER(ct.c_int8)),
        ("n_nodes", ct.c_int64),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ct.CDLL(_LIB_PATH)
    dp = ct.POINTER(ct.c_double)
    i64 = ct.c_int64
    lib.orc_round.argtypes = [ct.c_double, ct.c_int32]
    lib.orc_round.restype = ct.c_double
    lib.orc_round_array.argtypes = [dp, ct.c_int64, ct.c_int32, dp]
    lib.orc_round_array.restype = None
    lib.orc_scale.argtypes = [ct.c_double, ct.c_int32, ct.c_int32]
    lib.orc_scale.restype = ct.c_double
    lib.orc_rmax.argtypes = [ct.c_int32]
    lib.orc_rmax.restype = ct.c_double
    lib.orc_split.argtypes = [i64, ct.c_int32]
    lib.orc_split.restype = i64
    lib.orc_factor.argtypes = [i64, dp, i64, ct.POINTER(_Tree), ct.POINTER(i64)]
    lib.orc_factor.restype = ct.c_int32
    lib.orc_tree_trsm.argtypes = [i64, i64, dp, i64, ct.POINTER(_Tree)]
    lib.orc_tree_trsm.restype = ct.c_int32
    lib.orc_tree_syrk.argtypes = [i64, i64, dp, i64, ct.POINTER(_Tree)]
    lib.orc_tree_syrk.restype = ct.c_int32
    lib.orc_potrf_unblocked.argtypes = [i64, dp, i64, ct.POINTER(i64)]
    lib.orc_potrf_unblocked.restype = ct.c_int32
    lib.orc_trsm_left_lower.argtypes = [i64, i64, dp, i64, dp, i64]
    lib.orc_trsm_left_lower_t.argtypes = [i64, i64, dp, i64, dp, i64]
    lib.orc_residual.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, dp, i64]
    lib.orc_solve.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, dp, i64,
                              ct.c_double, ct.c_int32, ct.POINTER(ct.c_int32),
                              ct.POINTER(ct.c_double)]
    lib.orc_solve.restype = ct.c_int32
    lib.orc_backward_error.argtypes = [i64, dp, i64, dp, i64]
    lib.orc_backward_error.restype = ct.c_double
    lib.orc_count_nodes.argtypes = [i64, ct.c_int32, ct.c_int32]
    lib.orc_count_nodes.restype = i64
    lib.orc_num_threads.restype = ct.c_int32
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and (a.flags.f_contiguous or a.ndim == 1)
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _ld(a: np.ndarray) -> int:
    return a.shape[0]


@dataclass
class Tree:
    """Precision-tree descriptor (mirrors the C-ABI's mpchol_tree).

    offdiag lists precisions outermost (depth 0) to innermost; depths beyond the
    list repeat its last entry (Section 4.2's list convention)."""
    leaf: int = 64
    offdiag: Sequence[int] = (F64,)
    leaf_prec: int = F64
    split_align: int = 1
    syrk_leaf_mode: int = 0
    scale_mode: int = 0
    node_prec: Optional[Sequence[int]] = None
    _keep: list = field(default_factory=list, repr=False)

    def c_struct(self) -> _Tree:
        t = _Tree()
        t.leaf = self.leaf
        t.split_align = self.split_align
        t.nlevels = len(self.offdiag)
        for i, p in enumerate(self.offdiag):
            t.offdiag[i] = p
        t.leaf_prec = self.leaf_prec
        t.syrk_leaf_mode = self.syrk_leaf_mode
        t.scale_mode = self.scale_mode
        if self.node_prec is not None:
            arr = (ct.c_int8 * max(1, len(self.node_prec)))(*self.node_prec)
            self._keep = [arr]
            t.node_prec = ct.cast(arr, ct.POINTER(ct.c_int8))
            t.n_nodes = len(self.node_prec)
        else:
            t.node_prec = None
            t.n_nodes = 0
        return t


def round_to(x: float, prec: int) -> float:
    return _load().orc_round(float(x), prec)


def round_array(x: np.ndarray, prec: int) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.float64).ravel()
    out = np.empty_like(a)
    _load().orc_round_array(_dp(a), a.size, prec, _dp(out))
    return out.reshape(np.shape(x))


def scale(maxabs: float, prec: int, scale_mode: int = 0) -> float:
    return _load().orc_scale(float(maxabs), prec, scale_mode)


def rmax(prec: int) -> float:
    return _load().orc_rmax(prec)


def split(m: int, align: int = 1) -> int:
    return _load().orc_split(m, align)


def count_nodes(n: int, leaf: int, align: int = 1) -> int:
    return _load().orc_count_nodes(n, leaf, align)


def num_threads() -> int:
    return _load().orc_num_threads()


def factor(A: np.ndarray, n: Optional[int] = None, tree: Optional[Tree] = None):
    """Tree-POTRF of the lower triangle; returns (L, status, failed_index).

    L is a new Fortran-ordered array of A's shape whose lower triangle holds the
    factor (upper triangle copied unchanged from A)."""
    lib = _load()
    n = A.shape[1] if n is None else n
    tree = Tree() if tree is None else tree
    L = np.array(A, dtype=np.float64, order="F", copy=True)
    fi = ct.c_int64(0)
    ts = tree.c_struct()
    st = lib.orc_factor(n, _dp(L), _ld(L), ct.byref(ts), ct.byref(fi))
    return L, int(st), int(fi.value)


def tree_trsm(A: np.ndarray, m: int, k: int, tree: Optional[Tree] = None):
    """Tree-TRSM on its own (Algorithm 2, the precision list read by its own
    recursion depth): A[k:k+m, :k] <- A[k:k+m, :k] L^{-T} with L the lower
    triangle of A[:k, :k].  Returns (new array, status)."""
    tree = Tree() if tree is None else tree
    M = np.array(A, dtype=np.float64, order="F", copy=True)
    ts = tree.c_struct()
    st = _load().orc_tree_trsm(m, k, _dp(M), _ld(M), ct.byref(ts))
    return M, int(st)


def tree_syrk(A: np.ndarray, n: int, k: int, tree: Optional[Tree] = None):
    """Tree-SYRK on its own (Algorithm 3): the lower triangle of A[k:k+n, k:k+n]
    <- itself - A[k:k+n, :k] A[k:k+n, :k]^T.  Returns (new array, status)."""
    tree = Tree() if tree is None else tree
    M = np.array(A, dtype=np.float64, order="F", copy=True)
    ts = tree.c_struct()
    st = _load().orc_tree_syrk(n, k, _dp(M), _ld(M), ct.byref(ts))
    return M, int(st)


def potrf_unblocked(A: np.ndarray, n: Optional[int] = None):
    lib = _load()
    n = A.shape[1] if n is None else n
    L = np.array(A, dtype=np.float64, order="F", copy=True)
    fi = ct.c_int64(0)
    st = lib.orc_potrf_unblocked(n, _dp(L), _ld(L), ct.byref(fi))
    return L, int(st), int(fi.value)


def solve(L: np.ndarray, B: np.ndarray, A: Optional[np.ndarray] = None,
          n: Optional[int] = None, tol: float = 1e-13, max_iter: int = 20):
    """Returns (X, status, iters, final_rel_corr)."""
    lib = _load()
    n = L.shape[1] if n is None else n
    B = np.asfortranarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B.reshape(-1, 1, order="F")
    nrhs = B.shape[1]
    X = np.zeros((max(n, 1), nrhs), dtype=np.float64, order="F")
    it = ct.c_int32(0)
    fc = ct.c_double(0.0)
    Ap = _dp(A) if A is not None else None
    lda = _ld(A) if A is not None else max(n, 1)
    st = lib.orc_solve(n, nrhs, Ap, lda, _dp(L), _ld(L), _dp(B), _ld(B), _dp(X), _ld(X),
                       tol, max_iter, ct.byref(it), ct.byref(fc))
    return X, int(st), int(it.value), float(fc.value)


def residual(A: np.ndarray, X: np.ndarray, B: np.ndarray, n: Optional[int] = None):
    lib = _load()
    n = A.shape[1] if n is None else n
    X = np.asfortranarray(X, dtype=np.float64)
    B = np.asfortranarray(B, dtype=np.float64)
    nrhs = X.shape[1]
    R = np.zeros((n, nrhs), dtype=np.float64, order="F")
    lib.orc_residual(n, nrhs, _dp(A), _ld(A), _dp(X), _ld(X), _dp(B), _ld(B), _dp(R), _ld(R))
    return R


def backward_error(A: np.ndarray, L: np.ndarray, n: Optional[int] = None) -> float:
    lib = _load()
    n = A.shape[1] if n is None else n
    return float(lib.orc_backward_error(n, _dp(np.asfortranarray(A)), _ld(A),
                                        _dp(np.asfortranarray(L)), _ld(L)))
