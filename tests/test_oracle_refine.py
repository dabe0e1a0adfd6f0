"""Pins of the oracle's refinement stopping rule on hand-built systems.

The refinement (x0 = L^-T L^-1 b; r = b - A x in FP64, d = L^-T L^-1 r,
x += d) stops when max over columns of ||d||_inf / ||x||_inf <= tol (status
OK), when the correction holds Inf/NaN (NONFINITE), when that ratio grew in two
consecutive steps (diverging: NOT_CONVERGED), or after max_iter steps
(NOT_CONVERGED).  The paper gives no refinement of its own (its related work,
Section 2.2, surveys mixed-precision refinement), so the rule itself is the
reading being pinned.  Each case below is chosen so that every step is exact
in FP64 and the whole iteration can be followed by hand.
"""
import numpy as np

import oracle as O


def _diag_system(adiag, ldiag, b):
    n = len(adiag)
    A = np.asfortranarray(np.diag(np.asarray(adiag, dtype=np.float64)))
    L = np.asfortranarray(np.diag(np.asarray(ldiag, dtype=np.float64)))
    B = np.asfortranarray(np.asarray(b, dtype=np.float64).reshape(n, -1))
    return A, L, B


def test_exact_factor_converges_after_one_step():
    # L L^T = A: x0 is exact, the first correction is 0 -> OK after one step
    A, L, B = _diag_system([4.0, 9.0, 1.0], [2.0, 3.0, 1.0], [1.0, 3.0, -2.0])
    X, st, it, corr = O.solve(L, B, A=A, tol=1e-13, max_iter=20)
    assert (st, it, corr) == (O.OK, 1, 0.0)
    np.testing.assert_array_equal(X[:, 0], [0.25, 1.0 / 3.0, -2.0])


def test_oscillation_runs_to_max_iter():
    # A = 2, L L^T = 1, b = 1: x alternates 1, 0, 1, 0, ...; every correction
    # has size 1 and ||d|| / ||x|| stays 1 (when x = 0 the ratio is ||d||): it
    # never grows, never reaches tol -> stop at max_iter
    A, L, B = _diag_system([2.0], [1.0], [1.0])
    for max_iter, xlast in ((5, 0.0), (6, 1.0)):
        X, st, it, corr = O.solve(L, B, A=A, tol=1e-13, max_iter=max_iter)
        assert (st, it, corr) == (O.NOT_CONVERGED, max_iter, 1.0)
        assert X[0, 0] == xlast


def test_divergence_stops_after_two_growths():
    # A = I, L L^T = diag(1, 1/4), b = (1, e), e = 2^-20: the first component is
    # exact; the second has x0 = 4e, then x = -8e, 28e, -80e (error times -3 per
    # step) with corrections -12e, 36e, -108e while ||x||_inf stays 1: the ratio
    # grows at steps 2 and 3 -> stop after step 3
    e = 2.0 ** -20
    A, L, B = _diag_system([1.0, 1.0], [1.0, 0.5], [1.0, e])
    X, st, it, corr = O.solve(L, B, A=A, tol=1e-13, max_iter=20)
    assert (st, it) == (O.NOT_CONVERGED, 3)
    assert corr == 108.0 * e
    np.testing.assert_array_equal(X[:, 0], [1.0, -80.0 * e])


def test_growth_once_then_shrink_keeps_going():
    # the growth counter resets when the ratio shrinks: the oscillating case
    # above grows at every other step and still runs to max_iter, while the
    # same divergence with max_iter = 2 stops at the limit, not as diverged
    e = 2.0 ** -20
    A, L, B = _diag_system([1.0, 1.0], [1.0, 0.5], [1.0, e])
    X, st, it, corr = O.solve(L, B, A=A, tol=1e-13, max_iter=2)
    assert (st, it) == (O.NOT_CONVERGED, 2)
    assert corr == 36.0 * e


def test_nonfinite_right_hand_side():
    # a NaN in b reaches the first correction -> NONFINITE after step 1
    A, L, B = _diag_system([4.0, 4.0], [2.0, 2.0], [1.0, np.nan])
    X, st, it, corr = O.solve(L, B, A=A, tol=1e-13, max_iter=20)
    assert (st, it) == (O.NONFINITE, 1)


def test_multiple_columns_worst_column_decides():
    # column 0 converges at once; column 1 diverges as above: the stopping
    # ratio is the max over columns
    e = 2.0 ** -20
    A = np.asfortranarray(np.eye(2))
    L = np.asfortranarray(np.diag([1.0, 0.5]))
    B = np.asfortranarray(np.array([[1.0, 1.0], [0.0, e]]))
    X, st, it, corr = O.solve(L, B, A=A, tol=1e-13, max_iter=20)
    assert (st, it) == (O.NOT_CONVERGED, 3)
    assert corr == 108.0 * e
