"""Seeded synthetic inputs: dense SPD matrices with a chosen diagonal-dominance
ratio, and right-hand sides.

This module is the one piece shared by the CPU oracle and the GPU path.  It holds
none of the factorization's arithmetic: it only turns (seed, index) pairs into
matrix entries, from a published counter-based generator (SplitMix64, Steele,
Lea and Flood, OOPSLA 2014).  The GPU generator kernel in ``csrc/spdgen.hip``
implements the same definition and produces bitwise-identical matrices (the
dominance family below; the kernel family agrees to an ulp or two).

Definition (0-based indices, column-major storage):

* off-diagonal, i > j:  h = mix(seed XOR mix((i << 32) | j)),  u = h >> 40
  (24 bits),  a_ij = (u - 2^23) * 2^-23,  uniform on [-1, 1) on a 2^-23 grid;
  a_ji = a_ij.
* diagonal:  S_i = sum_{j != i} |a_ij|  (exact in FP64 in any order: every term
  is a multiple of 2^-23 and S_i < 2^17),  a_ii = RN(RN(ratio * S_i) + shift).
  ratio > 1 makes the matrix strictly diagonally dominant, hence SPD.
* right-hand side column c, row r:  the same hash on (seed_rhs, key (c << 32) | r).

A second family, ``gen_kernel``, is not diagonally dominant: the covariance
matrix of a Gaussian process with a squared-exponential kernel at n points of
the square [-1, 1)^2, plus a nugget (the matrices Gaussian-process regression
factors).  Point i is (hash(seed, (i << 32) | K0), hash(seed, (i << 32) | K1))
with K0 = 0xFFFFFFF0, K1 = 0xFFFFFFF1;  a_ij = exp(-|p_i - p_j|^2 / (2 ell^2))
for i != j,  a_ii = 1 + nugget.  Its eigenvalues decay fast, so the smallest
is about the nugget and the conditioning is about lambda_max / nugget.  The
GPU fill evaluates the same formula with the device's exp (equal to numpy's
up to an ulp or two, not bitwise).

The paper evaluates on dense SPD matrices with uniform random entries and a
large diagonal (Section 4.1); the dominance-ratio form keeps that structure and
makes the conditioning a parameter.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
TWO23 = 8388608.0


def mix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to state ``x`` (uint64 array)."""
    with np.errstate(over="ignore"):
        z = x + GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def hash_unit(seed: int, hi: np.ndarray, lo: np.ndarray) -> np.ndarray:
    """Value in [-1, 1) on the 2^-23 grid for keys (hi << 32) | lo."""
    key = (hi.astype(np.uint64) << np.uint64(32)) | lo.astype(np.uint64)
    h = mix64(np.uint64(seed) ^ mix64(key))
    u = (h >> np.uint64(40)).astype(np.int64)
    return (u - 8388608).astype(np.float64) / TWO23


def gen_spd(n: int, ratio: float, shift: float = 0.0, seed: int = 1,
            lda: int | None = None) -> np.ndarray:
    """Full symmetric SPD matrix, column-major (Fortran order), shape (lda, n).

    Only ``[:n, :n]`` is meaningful; padding rows hold zeros.
    """
    lda = n if lda is None else lda
    if lda < n:
        raise ValueError("lda < n")
    A = np.zeros((lda, n), dtype=np.float64, order="F")
    if n == 0:
        return A
    S = np.zeros(n, dtype=np.float64)
    rows = np.arange(n, dtype=np.int64)
    for j in range(n):
        i = rows[j + 1:]
        if i.size:
            v = hash_unit(seed, i, np.full(i.shape, j, dtype=np.int64))
            A[j + 1:n, j] = v
            A[j, j + 1:n] = v
            S[j + 1:] += np.abs(v)
            S[j] += np.abs(v).sum()
    A[rows, rows] = (ratio * S) + shift
    return A


def gen_rhs(n: int, nrhs: int, seed: int = 101, ldb: int | None = None) -> np.ndarray:
    """Right-hand sides uniform on [-1, 1), column-major, shape (ldb, nrhs)."""
    ldb = n if ldb is None else ldb
    B = np.zeros((ldb, nrhs), dtype=np.float64, order="F")
    r = np.arange(n, dtype=np.int64)
    for c in range(nrhs):
        B[:n, c] = hash_unit(seed, np.full(r.shape, c, dtype=np.int64), r)
    return B


KEY_X = 0xFFFFFFF0
KEY_Y = 0xFFFFFFF1


def kernel_points(n: int, seed: int) -> np.ndarray:
    """(n, 2) points of ``gen_kernel``, uniform on [-1, 1)^2."""
    i = np.arange(n, dtype=np.int64)
    return np.stack([hash_unit(seed, i, np.full(n, KEY_X, dtype=np.int64)),
                     hash_unit(seed, i, np.full(n, KEY_Y, dtype=np.int64))], axis=1)


def gen_kernel(n: int, ell: float, nugget: float, seed: int = 1,
               lda: int | None = None) -> np.ndarray:
    """Squared-exponential covariance matrix plus nugget, column-major (lda, n)."""
    lda = n if lda is None else lda
    if lda < n:
        raise ValueError("lda < n")
    A = np.zeros((lda, n), dtype=np.float64, order="F")
    if n == 0:
        return A
    P = kernel_points(n, seed)
    dx = P[:, 0][:, None] - P[:, 0][None, :]
    dy = P[:, 1][:, None] - P[:, 1][None, :]
    K = np.exp(-(dx * dx + dy * dy) / (2.0 * ell * ell))
    K[np.arange(n), np.arange(n)] = 1.0 + nugget
    A[:n, :n] = K
    return A


def gershgorin_lower_bound(n: int, ratio: float, shift: float, A: np.ndarray) -> float:
    """min_i (a_ii - sum_{j != i} |a_ij|): a lower bound on lambda_min(A)."""
    d = np.diag(A[:n, :n])
    off = np.abs(A[:n, :n]).sum(axis=1) - np.abs(d)
    return float(np.min(d - off))
