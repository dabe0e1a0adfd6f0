"""Host-side checks of libmpchol that need no GPU: the C-ABI loads and exports
every symbol include/mpchol.h declares, descriptor validation, and the
planner's bookkeeping against the analytic flop counts of Algorithms 1-3."""
import ctypes as ct
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "mpchol.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpchol_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = _declared_symbols()
    for s in ("mpchol_factor", "mpchol_solve", "mpchol_factor_batched", "mpchol_create",
              "mpchol_destroy"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2601_08082_amd import mpchol as M
    out = subprocess.run(["nm", "-D", "--defined-only", M.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mpchol_\w+)", out))
    missing = [s for s in _declared_symbols() if s not in exported]
    assert not missing, missing
    lib = ct.CDLL(M.LIB_PATH)
    for s in _declared_symbols():
        getattr(lib, s)


def test_gpu_code_object_is_gfx950():
    from paper_2601_08082_amd import mpchol as M
    data = open(M.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_null_context_rejected():
    from paper_2601_08082_amd import mpchol as M
    assert M.lib.mpchol_factor(None, 4, None, 4, None, 4, None, None, None) == -1
    assert M.lib.mpchol_solve(None, 4, 1, None, 4, None, 4, None, 4, None, 4, 1e-13, 5,
                              None, None) == -1


@pytest.mark.parametrize("field,value,code", [
    ("leaf", 0, -7), ("split_align", 0, -7), ("leaf_prec", 1, -7), ("scale_mode", 3, -7),
    ("abi_version", 99, -7), ("scale_tile", 8, 5), ("syrk_leaf_mode", 2, -7)])
def test_descriptor_validation(field, value, code):
    from paper_2601_08082_amd import mpchol as M
    t, keep = M.Tree().to_c()
    setattr(t, field, value)
    f4 = (ct.c_double * 4)()
    a, b = ct.c_double(), ct.c_double()
    c, d = ct.c_int64(), ct.c_int64()
    assert M.lib.mpchol_plan_stats(100, 100, ct.byref(t), f4, ct.byref(a), ct.byref(b),
                                   ct.byref(c), ct.byref(d)) == code


@pytest.mark.parametrize("n,leaf,offdiag,leafp,align", [
    (512, 64, (1, 1, 1), 3, 1), (1000, 64, (1, 2), 3, 1), (16384, 256, (1, 1, 2, 2, 2, 2), 3, 1),
    (65536, 256, (1, 2, 3), 3, 1), (777, 100, (0,), 2, 32), (64, 64, (1,), 3, 1), (1, 1, (1,), 3, 1)])
def test_plan_flops_match_cholesky(n, leaf, offdiag, leafp, align):
    """GEMM + leaf flops of the plan add up to the Cholesky count n^3/3 + O(n^2),
    and each precision gets the share its levels own."""
    from paper_2601_08082_amd import mpchol as M
    s = M.plan_stats(n, M.Tree(leaf=leaf, offdiag=list(offdiag), leaf_prec=leafp,
                               split_align=align))
    tot = sum(s["flops"].values()) + s["leaf_flops"]
    assert abs(tot - n ** 3 / 3) <= n * n * (1 + 64) , (tot, n ** 3 / 3)
    assert s["launches"] >= 1


def test_plan_precision_shares_of_the_16384_tree():
    """FP16 levels 0-1, FP32 levels 2-5, FP64 leaves of 256: per Algorithms 1-3
    the TRSM+SYRK flops of depth l are n^3 / 2^(2l+2), of which the leaf
    triangular solves (leaf precision) take n^2 b / 2^(l+2)."""
    from paper_2601_08082_amd import mpchol as M
    n, b = 16384, 256
    s = M.plan_stats(n, M.Tree(leaf=b, offdiag=[1, 1, 2, 2, 2, 2]))
    tot = n ** 3 / 3

    def level(l):
        return n ** 3 / 2 ** (2 * l + 2) - n * n * b / 2 ** (l + 2)

    f16 = level(0) + level(1)
    f32 = sum(level(l) for l in range(2, 6))
    assert s["flops"]["F16"] == pytest.approx(f16, rel=1e-3)
    assert s["flops"]["F32"] == pytest.approx(f32, rel=1e-2)
    assert s["flops"]["F16"] / tot == pytest.approx(0.92, abs=0.01)


def test_plan_node_precision_override_changes_only_that_node():
    from paper_2601_08082_amd import mpchol as M
    n = 1024
    base = M.plan_stats(n, M.Tree(leaf=128, offdiag=[1]))
    root64 = M.plan_stats(n, M.Tree(leaf=128, offdiag=[1], node_prec=[3]))
    # the root node issues n^3/4 TRSM + SYRK flops, minus its leaf solves n^2 b/4
    moved = base["flops"]["F16"] - root64["flops"]["F16"]
    assert moved == pytest.approx(n ** 3 / 4 - n * n * 128 / 4, rel=0.01)
    assert root64["flops"]["F64"] - base["flops"]["F64"] == pytest.approx(moved, rel=1e-12)
