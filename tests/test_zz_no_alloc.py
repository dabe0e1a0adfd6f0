"""The allocation-free solve entry point against mpchol_solve.

mpchol_solve_noalloc runs the kernels of mpchol_solve on the library's fixed
per-GPU scratch instead of context buffers; only its FP64 residual differs
(each tile of A read twice, summed in another order), so on the same factor
and right-hand sides both must reach the same status, the refinement counts
may differ by one step, and the solutions agree to the refinement tolerance
(both corrections end below 1e-13 of the solution).  Two calls in a row, the second with a smaller
system, check that nothing left in the shared scratch by the first call leaks
into the second; a third call at the maximum order checks the size limit, and
orders beyond it are refused.
"""
import numpy as np
import pytest

from paper_2601_08082_amd import spdgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2601_08082_amd import mpchol
    return mpchol


def _case(M, ctx, n, nrhs, seed, tree):
    import torch
    A = M.to_device_cm(spdgen.gen_spd(n, 1.5, 0.0, seed=seed))
    B = M.to_device_cm(spdgen.gen_rhs(n, nrhs, seed=seed + 100))
    L, info = ctx.factor(A, n, tree)
    assert info["status"] == M.OK
    Xref, iref = ctx.solve(L, B, n, A_cm=A, tol=1e-13, max_iter=20)
    X = torch.full_like(B, float("nan"))
    Xna, ina = M.solve_noalloc(L, B, n, A_cm=A, tol=1e-13, max_iter=20, X_cm=X, device=0)
    assert Xna.data_ptr() == X.data_ptr()
    return Xref, iref, Xna, ina


@pytest.mark.parametrize("calls", [[(1000, 4, 11), (300, 16, 12)], [(4100, 16, 13), (257, 1, 14)]])
def test_noalloc_matches_solve_twice(M, calls):
    import torch
    ctx = M.Context(0)
    tree = M.Tree(leaf=64, offdiag=[M.F16, M.F32], leaf_prec=M.F64)
    try:
        for n, nrhs, seed in calls:
            print(f"[gpu] noalloc n={n} nrhs={nrhs} seed={seed}", flush=True)
            Xref, iref, Xna, ina = _case(M, ctx, n, nrhs, seed, tree)
            assert ina["status"] == iref["status"] == M.OK
            assert abs(ina["ir_iters"] - iref["ir_iters"]) <= 1
            d = (Xna[:, :n] - Xref[:, :n]).abs().max(dim=1).values
            x = Xref[:, :n].abs().max(dim=1).values
            assert torch.all(d <= 1e-12 * x), (d / x).max().item()
    finally:
        ctx.close()


def test_noalloc_no_refinement_and_limits(M):
    import torch
    ctx = M.Context(0)
    try:
        n = M.NOALLOC_MAX_N
        print(f"[gpu] noalloc n={n} (the maximum), no refinement", flush=True)
        tree = M.Tree(leaf=256, offdiag=[M.F64], leaf_prec=M.F64)
        A = M.to_device_cm(spdgen.gen_spd(n, 1.5, 0.0, seed=21))
        B = M.to_device_cm(spdgen.gen_rhs(n, 2, seed=121))
        L, info = ctx.factor(A, n, tree)
        assert info["status"] == M.OK
        Xref, _ = ctx.solve(L, B, n, A_cm=None)
        Xna, ina = M.solve_noalloc(L, B, n, A_cm=None, X_cm=torch.empty_like(B))
        assert ina["status"] == M.OK and ina["ir_iters"] == 0
        assert torch.equal(Xna[:, :n], Xref[:, :n])
        with pytest.raises(ValueError):
            M.solve_noalloc(L, B, n + 1, A_cm=None, X_cm=torch.empty_like(B))
        B17 = torch.zeros((17, n), dtype=torch.float64, device=B.device)
        with pytest.raises(ValueError):
            M.solve_noalloc(L, B17, n, A_cm=None, X_cm=torch.empty_like(B17))
    finally:
        ctx.close()
