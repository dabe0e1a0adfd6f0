"""GPU parity of the HIP factorization (through the C-ABI) against the CPU oracle.

Bars (derived in the design notes):
  * integer-exact inputs (A = L0 L0^T): L0 returned bit for bit, every tree;
  * tridiagonal inputs: the layered-precision closed form bit for bit (the cast
    at each node boundary, FP64 leaves without contraction);
  * FP64 tree: ||A - L L^T||_F / ||A||_F <= 1e-13 and
    ||L - L_oracle||_F / ||L_oracle||_F <= 4 n u64 kappa-free bound 1e-13;
  * mixed trees: backward error within a factor 2 of the oracle's emulation of
    the same tree, and, with FP64 leaves, ||L - L_emu|| at most a quarter of
    ||L_emu - L_64|| (the two differ only in FP32 accumulation order, far below
    the operand quantization error they share).  With FP32 leaves the FP32
    rounding of the leaf arithmetic itself dominates and its order differs
    (blocked MFMA updates vs. one product at a time), so there the bar is
    ||L - L_emu|| <= 2 ||L_emu - L_64||;
  * casts: bit-identical codes and scale.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2601_08082_amd import spdgen

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


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


def _gpu_factor(M, ctx, A, n, tree):
    Ad = M.to_device_cm(A)
    Ld, info = ctx.factor(Ad, n, tree)
    return M.from_device_cm(Ld), info


def _otree(M, t):
    return O.Tree(leaf=t.leaf, offdiag=list(t.offdiag), leaf_prec=t.leaf_prec,
                  split_align=t.split_align, syrk_leaf_mode=t.syrk_leaf_mode,
                  scale_mode=t.scale_mode, node_prec=t.node_prec)


def _integer_L0(n, seed):
    rng = np.random.default_rng(seed)
    L0 = np.tril(rng.integers(-3, 4, (n, n)), -1).astype(np.int64)
    L0[np.arange(n), np.arange(n)] = rng.integers(max(1, n // 2), n + 1, n)
    return (np.asfortranarray(L0.astype(np.float64)),
            np.asfortranarray((L0 @ L0.T).astype(np.float64)))


def _trees(M):
    return [
        M.Tree(leaf=64, offdiag=[M.F64]),
        M.Tree(leaf=64, offdiag=[M.F16, M.F16, M.F16]),
        M.Tree(leaf=32, offdiag=[M.F16, M.F32, M.F64]),
        M.Tree(leaf=64, offdiag=[M.E4M3], scale_mode=1),
        M.Tree(leaf=48, offdiag=[M.F32], leaf_prec=M.F32),
        M.Tree(leaf=100, offdiag=[M.F16, M.F16, M.F32], split_align=32),
        M.Tree(leaf=256, offdiag=[M.F16, M.F32]),
        M.Tree(leaf=16, offdiag=[M.F16], syrk_leaf_mode=1),
        M.Tree(leaf=32, offdiag=[M.E4M3, M.F16, M.F32], scale_mode=2),
    ]


@pytest.mark.parametrize("n", [1, 7, 64, 130, 300])
@pytest.mark.parametrize("ti", range(9))
def test_integer_factor_bitwise(M, ctx, n, ti):
    """Substitution leaf TRSM: L0 bit for bit.  Inverse-based leaf TRSM (the
    default for FP64 leaves): L0 up to the rounding of the leaf inverses."""
    import dataclasses
    print(f"[gpu] integer L0 n={n} tree={ti}", flush=True)
    L0, A = _integer_L0(n, seed=1000 + n + ti)
    t = _trees(M)[ti]
    L, info = _gpu_factor(M, ctx, A, n, dataclasses.replace(t, leaf_trsm=1))
    assert info["status"] == M.OK, info
    np.testing.assert_array_equal(np.tril(L[:n, :n]), L0)
    L, info = _gpu_factor(M, ctx, A, n, dataclasses.replace(t, leaf_trsm=0))
    assert info["status"] == M.OK, info
    assert np.max(np.abs(np.tril(L[:n, :n]) - L0)) <= 1e-13 * np.max(np.abs(L0))


@pytest.mark.parametrize("n,e", [(7, -772), (130, -780), (300, -900)])
def test_tiny_pivots_scale_exactly(M, ctx, n, e):
    """Pivots below 2^-767 take the rescaled square-root path of the leaf
    POTRF (the sizes and scales put them below, across and far below that
    bound): A = 2^e L0 L0^T has the factor 2^(e/2) L0 bit for bit with the
    substitution leaf TRSM, and within FP64 rounding with the leaf inverses."""
    import dataclasses
    print(f"[gpu] tiny pivots n={n} e={e}", flush=True)
    L0, A = _integer_L0(n, seed=3000 + n)
    As = np.asfortranarray(np.ldexp(A, e))
    Ls0 = np.ldexp(L0, e // 2)
    t = M.Tree(leaf=64, offdiag=[M.F64])
    L, info = _gpu_factor(M, ctx, As, n, dataclasses.replace(t, leaf_trsm=1))
    assert info["status"] == M.OK, info
    np.testing.assert_array_equal(np.tril(L[:n, :n]), Ls0)
    L, info = _gpu_factor(M, ctx, As, n, t)
    assert info["status"] == M.OK, info
    assert np.max(np.abs(np.tril(L[:n, :n]) - Ls0)) <= 1e-13 * np.max(np.abs(Ls0))


@pytest.mark.parametrize("n,leaf", [(5, 4), (100, 37), (300, 64), (700, 128), (1111, 200),
                                    (2600, 256), (3001, 128)])
def test_leaf_inverse_trsm_vs_substitution(M, ctx, n, leaf):
    """The two leaf-TRSM modes agree to FP64 rounding on ragged leaves; the
    last two sizes also solve strips of more than 1024 rows."""
    import dataclasses
    print(f"[gpu] leaf inverse vs substitution n={n} leaf={leaf}", flush=True)
    A = spdgen.gen_spd(n, 1.1, 0.0, seed=n + 5)
    t = M.Tree(leaf=leaf, offdiag=[M.F64])
    Ls, _ = _gpu_factor(M, ctx, A, n, dataclasses.replace(t, leaf_trsm=1))
    Li, info = _gpu_factor(M, ctx, A, n, t)
    assert info["status"] == M.OK
    assert np.linalg.norm(np.tril(Li[:n, :n] - Ls[:n, :n])) <= 1e-14 * np.linalg.norm(np.tril(Ls[:n, :n]))


@pytest.mark.parametrize("prec", ["F16", "E4M3"])
def test_integer_factor_bitwise_large_tiles(M, ctx, prec):
    """n = 8192 with leaf 256: multi-round grids of 128 x 128 MFMA tiles and
    K up to 4096 in the FP32 accumulators (sums stay below 2^24).  A = L0 L0^T
    is formed on the device in FP64 (exact: entries < 2^53)."""
    import torch
    n = 8192
    print(f"[gpu] integer L0 n={n} {prec}", flush=True)
    g = torch.Generator(device="cpu").manual_seed(77)
    L0 = torch.tril(torch.randint(-3, 4, (n, n), generator=g), -1).to(torch.float64)
    L0 += torch.diag(torch.randint(n // 2, n + 1, (n,), generator=g).to(torch.float64))
    L0d = L0.cuda()
    # column-major storage of A = L0 L0^T is the row-major storage of A^T = A
    A = (L0d @ L0d.T.contiguous()).contiguous()
    t = M.Tree(leaf=256, offdiag=[getattr(M, prec)], scale_mode=1 if prec == "E4M3" else 0,
               leaf_trsm=1)
    L, info = ctx.factor(A, n, t)
    assert info["status"] == M.OK, info
    # L is column-major: its (n, ld) tensor holds L^T row-major
    assert torch.equal(torch.tril(L.T), L0d)


def _tridiag(n, c, d):
    A = np.zeros((n, n), order="F")
    A[np.arange(n), np.arange(n)] = d
    A[np.arange(1, n), np.arange(n - 1)] = c
    A[np.arange(n - 1), np.arange(1, n)] = c
    return A


@pytest.mark.parametrize("ti", [1, 2, 3, 5, 7])
def test_tridiagonal_bitwise_vs_oracle(M, ctx, ti):
    print(f"[gpu] tridiagonal tree={ti}", flush=True)
    n = 333
    import dataclasses
    A = _tridiag(n, -1.0, 2.5)
    t = dataclasses.replace(_trees(M)[ti], leaf_trsm=1)
    L, info = _gpu_factor(M, ctx, A, n, t)
    Lo, st, _ = O.factor(A, tree=_otree(M, t))
    assert info["status"] == M.OK and st == O.OK
    np.testing.assert_array_equal(np.diag(L), np.diag(Lo))
    np.testing.assert_array_equal(np.diag(L, -1), np.diag(Lo, -1))


@pytest.mark.parametrize("n,leaf,align,lda_pad", [(1, 64, 1, 0), (37, 16, 1, 3), (256, 64, 1, 0),
                                                  (300, 64, 1, 64), (513, 64, 32, 7),
                                                  (1000, 128, 1, 0), (777, 200, 32, 1)])
def test_fp64_tree_vs_oracle(M, ctx, n, leaf, align, lda_pad):
    print(f"[gpu] fp64 n={n} leaf={leaf} align={align}", flush=True)
    A = spdgen.gen_spd(n, 1.2, 0.5, seed=n, lda=n + lda_pad)
    t = M.Tree(leaf=leaf, offdiag=[M.F64], split_align=align)
    L, info = _gpu_factor(M, ctx, A, n, t)
    Lo, st, _ = O.factor(A, n=n, tree=_otree(M, t))
    assert info["status"] == M.OK and st == O.OK
    Lg, Lr = np.tril(L[:n, :n]), np.tril(Lo[:n, :n])
    assert np.linalg.norm(Lg - Lr) <= 1e-13 * np.linalg.norm(Lr)
    assert O.backward_error(A, L, n=n) <= 1e-13
    # the strictly upper triangle of the output is never written
    assert np.all(np.triu(L[:n, :n], 1) == 0)


MIXED = [
    ("C1 [F16]x3 b64", 512, 1.0, 1.0, dict(leaf=64, offdiag=[1, 1, 1])),
    ("[F16,F32,F64] b32", 512, 1.2, 0.0, dict(leaf=32, offdiag=[1, 2, 3])),
    ("E4M3 pow2 b64", 512, 1.5, 0.0, dict(leaf=64, offdiag=[0], scale_mode=1)),
    ("F32 all b64", 512, 1.05, 0.0, dict(leaf=64, offdiag=[2], leaf_prec=2)),
    ("[F16,F16,F32] ragged", 1111, 1.5, 0.0, dict(leaf=100, offdiag=[1, 1, 2], split_align=32)),
    ("[F16,F32] b256", 1024, 1.5, 0.0, dict(leaf=256, offdiag=[1, 2])),
    ("F16 leafSYRK64", 700, 1.1, 0.0, dict(leaf=64, offdiag=[1], syrk_leaf_mode=1)),
    ("E4M3/F16/F32 node", 640, 1.3, 0.0, dict(leaf=40, offdiag=[0, 1, 2], scale_mode=1)),
    ("E4M3 up, F16 down", 640, 1.3, 0.0, dict(leaf=40, offdiag=[0, 1, 2], scale_mode=2)),
]


@pytest.mark.parametrize("name,n,ratio,shift,kw", MIXED, ids=[m[0] for m in MIXED])
def test_mixed_tree_vs_emulation(M, ctx, name, n, ratio, shift, kw):
    print(f"[gpu] mixed {name}", flush=True)
    A = spdgen.gen_spd(n, ratio, shift, seed=7 + n)
    t = M.Tree(**kw)
    L, info = _gpu_factor(M, ctx, A, n, t)
    assert info["status"] == M.OK, info
    Le, st, _ = O.factor(A, tree=_otree(M, t))
    L64, _, _ = O.factor(A, tree=O.Tree(leaf=t.leaf, offdiag=[O.F64]))
    be_gpu = O.backward_error(A, L)
    be_emu = O.backward_error(A, Le)
    assert 0.5 <= be_gpu / be_emu <= 2.0, (be_gpu, be_emu)
    d_ge = np.linalg.norm(np.tril(L) - np.tril(Le))
    d_e64 = np.linalg.norm(np.tril(Le) - np.tril(L64))
    bar = 2.0 if t.leaf_prec == M.F32 else 0.25
    assert d_ge <= bar * d_e64, (d_ge, d_e64)


def test_node_precision_policy_applied(M, ctx):
    n = 512
    A = spdgen.gen_spd(n, 1.5, 0.0, seed=3)
    nodes = O.count_nodes(n, 64, 1)
    rng = np.random.default_rng(1)
    npz = [int(v) for v in rng.integers(1, 4, nodes)]
    t = M.Tree(leaf=64, offdiag=[M.F16], node_prec=npz)
    L, info = _gpu_factor(M, ctx, A, n, t)
    Le, _, _ = O.factor(A, tree=_otree(M, t))
    L64, _, _ = O.factor(A, tree=O.Tree(leaf=64, offdiag=[O.F64]))
    assert np.linalg.norm(np.tril(L) - np.tril(Le)) <= 0.25 * np.linalg.norm(np.tril(Le) - np.tril(L64))


def test_not_spd_index_matches_oracle(M, ctx):
    n = 300
    A = spdgen.gen_spd(n, 1.5, 0.0, seed=2)
    A[123, 123] = -1.0
    for t in (M.Tree(leaf=64, offdiag=[M.F64]), M.Tree(leaf=32, offdiag=[M.F16, M.F32])):
        _, info = _gpu_factor(M, ctx, A, n, t)
        _, st, fi = O.factor(A, tree=_otree(M, t))
        assert info["status"] == M.NOT_SPD and st == O.NOT_SPD
        assert info["failed_index"] == fi == 124


def test_nan_input_reports_not_spd(M, ctx):
    n = 200
    A = spdgen.gen_spd(n, 1.5, 0.0, seed=4)
    A[150, 20] = np.nan
    t = M.Tree(leaf=32, offdiag=[M.F16])
    _, info = _gpu_factor(M, ctx, A, n, t)
    _, st, fi = O.factor(A, tree=_otree(M, t))
    assert info["status"] == M.NOT_SPD and st == O.NOT_SPD
    assert info["failed_index"] == fi


def test_in_place_factor(M, ctx):
    import torch
    n = 400
    A = spdgen.gen_spd(n, 1.5, 0.0, seed=5)
    Ad = M.to_device_cm(A)
    t = M.Tree(leaf=64, offdiag=[M.F16, M.F32])
    L1, _ = ctx.factor(Ad.clone(), n, t)
    L2, info = ctx.factor(Ad, n, t, L_cm=Ad)
    assert info["status"] == 0
    assert torch.equal(torch.tril(L1.T), torch.tril(L2.T))


def test_determinism(M, ctx):
    import torch
    n = 1500
    A = spdgen.gen_spd(n, 1.2, 0.0, seed=6)
    Ad = M.to_device_cm(A)
    t = M.Tree(leaf=128, offdiag=[M.F16, M.F16, M.F32])
    L1, _ = ctx.factor(Ad, n, t)
    L2, _ = ctx.factor(Ad, n, t)
    assert torch.equal(L1, L2)


def test_bad_arguments_rejected(M, ctx):
    import torch
    Ad = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        ctx.factor(Ad, 5, M.Tree())           # lda 4 < n 5
    with pytest.raises(ValueError):
        ctx.factor(Ad, 4, M.Tree(leaf=0))


def _e4m3_bits(v):
    if v == 0.0:
        return 0x80 if math.copysign(1.0, v) < 0 else 0x00
    s = 0x80 if v < 0 else 0
    a = abs(v)
    if a < 2.0 ** -6:
        return s | int(round(a / 2.0 ** -9))
    e = math.floor(math.log2(a))
    f = int(round((a / 2.0 ** e - 1.0) * 8))
    return s | ((e + 7) << 3) | f


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("shape,scale_pow", [((64, 64), 0), ((150, 77), -20), ((200, 130), 18),
                                             ((1, 1), 0), ((513, 17), -3)])
def test_cast_bitwise(M, ctx, prec, mode, shape, scale_pow):
    """GPU quantization == oracle RNE_p(x / s) bit for bit (random, subnormal
    range, exact ties, the double-rounding witness)."""
    print(f"[gpu] cast prec={prec} mode={mode} shape={shape}", flush=True)
    rows, cols = shape
    rng = np.random.default_rng(rows * 7 + cols + prec)
    X = rng.standard_normal((rows, cols)) * 10.0 ** rng.uniform(-6, 2, (rows, cols))
    X *= 2.0 ** scale_pow
    flat = X.reshape(-1)
    if flat.size > 8:
        flat[0] = (1.0 + 2.0 ** -11 + 2.0 ** -40) * 2.0 ** scale_pow
        flat[1] = (1.0 + 3 * 2.0 ** -11) * 2.0 ** scale_pow      # tie
        flat[2] = 3 * 2.0 ** -26 * 2.0 ** scale_pow
        flat[3] = -0.0
    X = np.asfortranarray(X)
    codes, s, st = ctx.quantize(M.to_device_cm(X), rows, cols, prec, mode)
    assert st == 0
    maxabs = np.abs(X).max()
    s_or = O.scale(maxabs, prec, mode)
    assert s == s_or
    want = O.round_array(X / s_or, prec)
    got = codes.cpu().numpy()
    if prec == 1:
        want_bits = want.astype(np.float16).view(np.int16)
        np.testing.assert_array_equal(got[:rows, :cols], want_bits)
    else:
        wb = np.vectorize(_e4m3_bits)(want).astype(np.uint8)
        np.testing.assert_array_equal(got[:rows, :cols], wb)
    assert np.all(got[:rows, cols:] == 0)


@pytest.mark.parametrize("n,leaf", [(500, 64), (1100, 128), (1024, 64)])
def test_large_magnitude_block_scales(M, ctx, n, leaf):
    """Entries far above the FP16 range: every quantized block needs a scale
    above 1 (the single-pass cast re-casts those blocks; at n = 1024 the
    operands of a launch also share their scale-1 copies); the result follows
    the oracle's per-block scaling to the mixed-precision bars."""
    print(f"[gpu] large-magnitude scales n={n}", flush=True)
    A = spdgen.gen_spd(n, 1.3, 0.0, seed=n + 21) * 2.0 ** 44   # exact scaling
    t = M.Tree(leaf=leaf, offdiag=[M.F16, M.F16, M.F32])
    L, info = _gpu_factor(M, ctx, A, n, t)
    assert info["status"] == M.OK, info
    Le, st, _ = O.factor(A, tree=_otree(M, t))
    L64, _, _ = O.factor(A, tree=O.Tree(leaf=leaf, offdiag=[O.F64]))
    assert st == O.OK
    assert np.max(np.abs(np.tril(L64[:n, :n], -1))) > 65504.0   # operands above the FP16 range
    be_g, be_e = O.backward_error(A, L), O.backward_error(A, Le)
    assert 0.5 <= be_g / be_e <= 2.0, (be_g, be_e)
    d_ge = np.linalg.norm(np.tril(L[:n, :n]) - np.tril(Le[:n, :n]))
    d_e64 = np.linalg.norm(np.tril(Le[:n, :n]) - np.tril(L64[:n, :n]))
    assert d_ge <= 0.25 * d_e64, (d_ge, d_e64)


def test_mixed_magnitude_shared_copies(M, ctx):
    """A = D A0 D with every other 64-row block of D at 2^30: operands that
    share one scale-1 copy (n = 1024, leaf 64, aligned splits) have block
    scales of 1 and above 1 side by side, so some read the shared copy and
    others their own re-cast copy."""
    n, leaf = 1024, 64
    print(f"[gpu] mixed-magnitude shared copies n={n}", flush=True)
    A0 = spdgen.gen_spd(n, 1.3, 0.0, seed=4242)
    d = np.where((np.arange(n) // 64) % 2 == 1, 2.0 ** 30, 1.0)
    A = np.asfortranarray(A0 * d[:, None] * d[None, :])   # exact scaling by powers of two
    t = M.Tree(leaf=leaf, offdiag=[M.F16, M.F16, M.F32])
    L, info = _gpu_factor(M, ctx, A, n, t)
    assert info["status"] == M.OK, info
    Le, st, _ = O.factor(A, tree=_otree(M, t))
    L64, _, _ = O.factor(A, tree=O.Tree(leaf=leaf, offdiag=[O.F64]))
    assert st == O.OK
    be_g, be_e = O.backward_error(A, L), O.backward_error(A, Le)
    assert 0.5 <= be_g / be_e <= 2.0, (be_g, be_e)
    d_ge = np.linalg.norm(np.tril(L[:n, :n]) - np.tril(Le[:n, :n]))
    d_e64 = np.linalg.norm(np.tril(Le[:n, :n]) - np.tril(L64[:n, :n]))
    assert d_ge <= 0.25 * d_e64, (d_ge, d_e64)
