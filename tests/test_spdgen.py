"""The seeded input generator: published SplitMix64 outputs, symmetry, exact
row sums, strict diagonal dominance (hence SPD)."""
import numpy as np

from paper_2601_08082_amd import spdgen


def test_splitmix64_published_sequence():
    # SplitMix64 seeded with 0: the first three outputs of the reference
    # generator (Steele, Lea, Flood 2014; Vigna's splitmix64.c)
    state = np.array([0], dtype=np.uint64)
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    with np.errstate(over="ignore"):
        got = [int(spdgen.mix64(state + np.uint64(k) * spdgen.GAMMA)[0]) for k in range(3)]
    assert got == want


def test_matrix_structure_and_exact_rowsums():
    n, ratio, shift = 300, 1.5, 0.0
    A = spdgen.gen_spd(n, ratio, shift, seed=2, lda=n + 7)
    M = A[:n, :n]
    assert A.shape == (n + 7, n) and A.flags.f_contiguous
    np.testing.assert_array_equal(M, M.T)
    off = M - np.diag(np.diag(M))
    assert np.all(np.abs(off) < 1.0) and np.all(off >= -1.0)
    assert np.all(off * 2 ** 23 == np.round(off * 2 ** 23))        # 2^-23 grid
    S = np.abs(off).sum(axis=1)
    np.testing.assert_array_equal(np.diag(M), ratio * S + shift)   # exact sums
    assert np.all(A[n:, :] == 0)
    assert np.linalg.eigvalsh(M).min() > (ratio - 1) * S.min() * 0.999


def test_deterministic_and_seed_dependent():
    a = spdgen.gen_spd(64, 1.2, 0.0, seed=5)
    b = spdgen.gen_spd(64, 1.2, 0.0, seed=5)
    c = spdgen.gen_spd(64, 1.2, 0.0, seed=6)
    np.testing.assert_array_equal(a, b)
    assert np.any(a != c)
    # a sub-matrix of a larger matrix has the same off-diagonal entries
    big = spdgen.gen_spd(100, 1.2, 0.0, seed=5)
    np.testing.assert_array_equal(np.tril(a, -1), np.tril(big[:64, :64], -1))


def test_rhs():
    B = spdgen.gen_rhs(50, 3, seed=101, ldb=53)
    assert B.shape == (53, 3)
    assert np.all(np.abs(B[:50]) <= 1.0) and np.all(B[50:] == 0)
    assert len(np.unique(B[:50])) == 150
