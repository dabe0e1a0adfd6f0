"""GPU backward-error check (mpchol_backward_error) against the oracle's
compensated CPU computation of ||A - L L^T||_F / ||A||_F.

Bars: within 1e-6 relative for mixed-precision factors (errors >= 1e-9);
at most 1e-13 for FP64 factors (the check's own rounding is ~sqrt(n) u);
the upper triangle of L is never read; L = 0 gives exactly 1."""
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


@pytest.mark.parametrize("n", [1, 63, 100, 777, 2000])
def test_backward_error_matches_oracle(M, ctx, n):
    print(f"[gpu] backward error n={n}", flush=True)
    A = spdgen.gen_spd(n, 1.2, 0.5, seed=n + 11)
    Ad = M.to_device_cm(A)
    L16, info = ctx.factor(Ad, n, M.Tree(leaf=32, offdiag=[M.F16]))
    assert info["status"] == 0
    Lh = M.from_device_cm(L16)
    be_o = O.backward_error(A, Lh)
    be_g, rn, an = ctx.backward_error(Ad, L16, n)
    if be_o >= 1e-9:
        assert be_g == pytest.approx(be_o, rel=1e-6)
    else:
        assert be_g <= 1e-13
    assert an == pytest.approx(np.linalg.norm(np.tril(A[:n, :n]) + np.tril(A[:n, :n], -1).T), rel=1e-13)
    L64, _ = ctx.factor(Ad, n, M.Tree(leaf=64, offdiag=[M.F64]))
    assert ctx.backward_error(Ad, L64, n)[0] <= 1e-13


def test_backward_error_ignores_upper_and_zero_factor(M, ctx):
    import torch
    n = 300
    A = spdgen.gen_spd(n, 1.5, 0.0, seed=3)
    Ad = M.to_device_cm(A)
    L, _ = ctx.factor(Ad, n, M.Tree(leaf=64, offdiag=[M.F16]))
    be1 = ctx.backward_error(Ad, L, n)[0]
    Lh = M.from_device_cm(L)
    Lh[np.triu_indices(n, 1)] = np.nan
    be2 = ctx.backward_error(Ad, M.to_device_cm(Lh), n)[0]
    assert be1 == be2
    Z = torch.zeros_like(Ad)
    assert ctx.backward_error(Ad, Z, n)[0] == 1.0
