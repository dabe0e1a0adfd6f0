"""Pins of the learned-policy oracle (oracle/policy.py) against closed forms,
hand-derived values and finite differences: node numbering, features,
quantization-error labels, the perceptron's gradient and the Adam step."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.policy as P


def test_nodes_preorder_hand():
    # n = 8, leaf 2: root [0,8) split 4, then [0,4) split 2, then [4,8) split 2
    assert P.nodes(8, 2) == [(0, 8, 4, 0), (0, 4, 2, 1), (4, 4, 2, 1)]
    # n = 7, leaf 2: root split 3; [0,3) split 1 (depth 1); [3,7) split 2 (depth 1)
    assert P.nodes(7, 2) == [(0, 7, 3, 0), (0, 3, 1, 1), (3, 4, 2, 1)]
    for n, b, al in [(1000, 64, 1), (777, 32, 32), (64, 64, 1), (65, 64, 1), (2048, 256, 1)]:
        assert len(P.nodes(n, b, al)) == O.count_nodes(n, b, al)


def _compound(n, a, beta):
    return np.asfortranarray(a * np.eye(n) + beta * np.ones((n, n)))


@pytest.mark.parametrize("n,leaf,a,beta", [(64, 8, 3.0, 0.25), (100, 16, 50.0, -0.5), (33, 4, 1.0, 2.0 ** -7)])
def test_features_compound_symmetry(n, leaf, a, beta):
    # A = a I + beta 1 1^T: every A21 entry is beta, every diagonal a + beta,
    # every off-diagonal row sum (n - 1) |beta|
    F = P.features(_compound(n, a, beta), n, leaf)
    nd = P.nodes(n, leaf)
    assert F.shape == (len(nd), 6)
    f1 = math.log2(abs(beta) / math.sqrt(a + beta))
    f3 = math.log2((a + beta) / ((n - 1) * abs(beta)))
    # every row: a_ii - max |a_ij| = a + beta - |beta|, over the mean diagonal a + beta
    f6 = math.log2((a + beta - abs(beta)) / (a + beta))
    for row, (i0, m, m1, d) in zip(F, nd):
        assert row[0] == pytest.approx(f1, abs=1e-12)
        assert row[1] == pytest.approx(0.0, abs=1e-12)
        assert row[2] == pytest.approx(f3, abs=1e-12)
        assert row[3] == d and row[4] == math.log2(m1)
        assert row[5] == pytest.approx(f6, abs=1e-12)


def test_features_diagonal_and_single_entry():
    n = 16
    A = np.asfortranarray(np.diag(np.arange(1.0, n + 1)))
    F = P.features(A, n, 4)
    assert np.all(F[:, 0] == -64.0) and np.all(F[:, 1] == 0.0) and np.all(F[:, 2] == 30.0)
    # f6 of a diagonal matrix: min diag / mean diag of the node (root: 1 / 8.5)
    for row, (i0, m, m1, d) in zip(F, P.nodes(n, 4)):
        assert row[5] == pytest.approx(math.log2((i0 + 1) / (i0 + (m + 1) / 2)), abs=1e-12)
    # one nonzero 0.5 in the root's A21 (rows 8..15, cols 0..7): 64 entries,
    # rms = 0.5 / 8, max / rms = 8; root mean diag = 8.5; row 9 ratio = 10 / 0.5
    A[9, 2] = A[2, 9] = 0.5
    F = P.features(A, n, 4)
    assert F[0, 0] == pytest.approx(math.log2((0.5 / 8) / math.sqrt(8.5)), abs=1e-12)
    assert F[0, 1] == pytest.approx(3.0, abs=1e-12)
    assert F[0, 2] == pytest.approx(math.log2(3.0 / 0.5), abs=1e-12)   # row 2: a_22 = 3
    # node [0, 8) holds row 2: a_22 - 0.5 = 2.5 > its min diag 1, so f6 keeps
    # 1 / 4.5; a 2 x 2 block [[1, 0.9], [0.9, 1]] on rows 0, 1 brings the
    # root's min gap to 0.1
    assert F[1, 5] == pytest.approx(math.log2(1.0 / 4.5), abs=1e-12)
    C = A.copy()
    C[0, 0] = C[1, 1] = 1.0
    C[1, 0] = C[0, 1] = 0.9
    assert P.features(C, n, 4)[0, 5] == pytest.approx(math.log2(0.1 / ((1 + 1 + sum(range(3, 17))) / 16)),
                                                      abs=1e-12)
    # the lower triangle alone decides: garbage above the diagonal is ignored
    B = A.copy()
    B[np.triu_indices(n, 1)] = 7.0
    np.testing.assert_array_equal(P.features(B, n, 4), F)


def _node_block(n, leaf, X):
    """A = I (so ||A_node||_F = sqrt(m)) and an L whose root L21 block is X."""
    A = np.asfortranarray(np.eye(n))
    L = np.zeros((n, n), order="F")
    i0, m, m1, _ = P.nodes(n, leaf)[0]
    L[i0 + m1:i0 + m, i0:i0 + m1] = X
    return A, L, m


def test_errors_closed_form():
    n, leaf = 16, 4
    # 1 + 2^-5: E4M3 (3 fraction bits) rounds it to 1 (error 2^-5 each),
    # exact in FP16 and FP32
    X = np.full((8, 8), 1.0 + 2.0 ** -5)
    A, L, m = _node_block(n, leaf, X)
    e = P.node_errors(A, L, n, leaf, scale_mode=1)[0]
    want = 2.0 * (8 * (1 + 2.0 ** -5)) * (8 * 2.0 ** -5) / math.sqrt(m)
    assert e[O.E4M3] == pytest.approx(want, rel=1e-14)
    assert e[O.F16] == 0.0 and e[O.F32] == 0.0
    # 1 + 2^-11 is an FP16 tie: rounds to even (1), error 2^-11 each; FP32 exact
    X = np.full((8, 8), 1.0 + 2.0 ** -11)
    A, L, m = _node_block(n, leaf, X)
    e = P.node_errors(A, L, n, leaf, scale_mode=1)[0]
    assert e[O.F16] == pytest.approx(2.0 * (8 * (1 + 2.0 ** -11)) * (8 * 2.0 ** -11) / math.sqrt(m), rel=1e-14)
    assert e[O.F32] == 0.0
    # small integers are exact in every format (scale is a power of two)
    X = np.arange(64, dtype=float).reshape(8, 8) % 9 - 4
    A, L, m = _node_block(n, leaf, X)
    assert np.all(P.node_errors(A, L, n, leaf, scale_mode=1)[0] == 0.0)


def test_errors_scale_matters():
    # values around 2^-12 lie below E4M3's normal range: with scale_mode 0
    # (never scaled up) they flush to coarse subnormals, with scale_mode 1 they
    # are scaled into range and exact
    n, leaf = 16, 4
    X = np.full((8, 8), 3.0 * 2.0 ** -12)
    A, L, m = _node_block(n, leaf, X)
    e0 = P.node_errors(A, L, n, leaf, scale_mode=0)[0]
    e1 = P.node_errors(A, L, n, leaf, scale_mode=1)[0]
    assert e1[O.E4M3] == 0.0 and e0[O.E4M3] > 0.0
    # E4M3 subnormal spacing 2^-9: 3 * 2^-12 = 0.375 * 2^-9 rounds to 0 (error 3 * 2^-12)
    assert e0[O.E4M3] == pytest.approx(2 * (8 * 3 * 2.0 ** -12) * (8 * 3 * 2.0 ** -12) / math.sqrt(m), rel=1e-14)
    # 5 * 2^-12 = 0.625 * 2^-9 rounds up to 2^-9 (error 3 * 2^-12)
    X = np.full((8, 8), 5.0 * 2.0 ** -12)
    A, L, m = _node_block(n, leaf, X)
    e0 = P.node_errors(A, L, n, leaf, scale_mode=0)[0]
    assert e0[O.E4M3] == pytest.approx(2 * (8 * 5 * 2.0 ** -12) * (8 * 3 * 2.0 ** -12) / math.sqrt(m), rel=1e-14)


def test_budgets_and_labels():
    n, leaf = 64, 8
    nd = P.nodes(n, leaf)
    b = P.budgets(n, leaf, 1, 1e-4)
    s2 = np.array([m1 * m1 for (_, _, m1, _) in nd], dtype=float)
    assert b.sum() == pytest.approx(1e-4, rel=1e-14)
    assert b[0] / b[1] == pytest.approx(s2[0] / s2[1])
    err = np.array([[1e-9, 0, 0], [1e-3, 1e-6, 0], [1, 1, 1], [1e-3, 1e-3, 1e-12]])
    bud = np.array([1e-8, 1e-5, 1e-2, 1e-12])
    np.testing.assert_array_equal(P.labels_from(err, bud), [O.E4M3, O.F16, O.F64, O.F32])
    # a floor: formats below it are never chosen, the rest of the rule unchanged
    np.testing.assert_array_equal(P.labels_from(err, bud, O.F16), [O.F16, O.F16, O.F64, O.F32])
    np.testing.assert_array_equal(P.labels_from(err, bud, O.F32), [O.F32, O.F32, O.F64, O.F32])


def test_pivot_ratio_closed_form_and_definition():
    # diagonal A: the pivots are the diagonal itself
    d = np.array([4.0, 0.25, 9.0, 1.0])
    L = np.diag(np.sqrt(d))
    assert P.pivot_ratio(L, 4) == pytest.approx(0.25 / 9.0, rel=1e-15)
    assert P.pivot_ratio(np.zeros((1, 1)), 0) == 1.0
    # pivot i = 1 / (inverse of the leading (i+1) block)[i, i], an independent route
    from paper_2601_08082_amd import spdgen
    n = 40
    A = spdgen.gen_kernel(n, 0.4, 0.05, seed=3)
    L = O.factor(A, tree=O.Tree(leaf=8, offdiag=[O.F64]))[0]
    piv = np.array([1.0 / np.linalg.inv(A[:i + 1, :i + 1])[i, i] for i in range(n)])
    assert P.pivot_ratio(L, n) == pytest.approx(piv.min() / piv.max(), rel=1e-9)


@pytest.mark.parametrize("kind", ["dominance", "kernel"])
def test_pivot_ratio_brackets_inverse_condition(kind):
    # every pivot lies in [lambda_min, lambda_max], so 1/kappa_2 <= g <= 1
    from paper_2601_08082_amd import spdgen
    n = 120
    A = (spdgen.gen_spd(n, 1.02, 0.0, seed=4) if kind == "dominance"
         else spdgen.gen_kernel(n, 0.3, 1e-3, seed=4))
    w = np.linalg.eigvalsh(A[:n, :n])
    L = O.factor(A, tree=O.Tree(leaf=16, offdiag=[O.F64]))[0]
    g = P.pivot_ratio(L, n)
    assert w[0] / w[-1] <= g * (1 + 1e-9) and g <= 1.0
    b = P.budgets(n, 16, 1, 1e-2, g)
    assert b.sum() == pytest.approx(1e-2 * g, rel=1e-14)


def test_kernel_family_labels_need_more_precision():
    # an ill-conditioned covariance matrix: with the pivot-ratio budget the
    # root and most nodes need at least F32, where a dominant matrix of the
    # same size takes E4M3 or F16 everywhere
    from paper_2601_08082_amd import spdgen
    n, leaf = 256, 32
    Ak = spdgen.gen_kernel(n, 0.3, 1e-3, seed=6)
    Lk = O.factor(Ak, tree=O.Tree(leaf=leaf, offdiag=[O.F64]))[0]
    lk = P.labels_from(P.node_errors(Ak, Lk, n, leaf, scale_mode=2),
                       P.budgets(n, leaf, 1, 1e-2, P.pivot_ratio(Lk, n)))
    Ad = spdgen.gen_spd(n, 1.5, 0.0, seed=6)
    Ld = O.factor(Ad, tree=O.Tree(leaf=leaf, offdiag=[O.F64]))[0]
    ld = P.labels_from(P.node_errors(Ad, Ld, n, leaf, scale_mode=2),
                       P.budgets(n, leaf, 1, 1e-2, P.pivot_ratio(Ld, n)))
    assert lk[0] >= O.F32 and np.sum(lk >= O.F32) > len(lk) / 2 and np.all(ld <= O.F16)


def test_labels_monotone_in_dominance():
    # a more dominant diagonal shrinks L21 relative to A: labels never get more precise
    from paper_2601_08082_amd import spdgen
    n, leaf = 256, 32
    prev = None
    for ratio in (1.05, 2.0, 10.0):
        A = spdgen.gen_spd(n, ratio, 0.0, seed=5)
        L = O.factor(A, tree=O.Tree(leaf=leaf, offdiag=[O.F64]))[0]
        lab = P.labels_from(P.node_errors(A, L, n, leaf), P.budgets(n, leaf, 1, 1e-4))
        if prev is not None:
            assert np.all(lab <= prev)
        prev = lab


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.4, P.NPARAM)
    u = P.unpack(p)
    u["mu"][:] = rng.normal(0, 1, P.NFEAT)
    u["sigma"][:] = rng.uniform(0.5, 2.0, P.NFEAT)
    return p


def test_mlp_forward_hand():
    p = np.zeros(P.NPARAM)
    u = P.unpack(p)
    u["sigma"][:] = 1.0
    prob, _ = P.forward(p, np.zeros((3, P.NFEAT)))
    np.testing.assert_allclose(prob, 0.25)
    assert P.loss(p, np.zeros((3, P.NFEAT)), np.array([0, 1, 3])) == pytest.approx(math.log(4))
    # one path: h1[0] = relu(x0), h2[0] = relu(2 h1[0]), z = [3 h2[0], 0, 0, 0]
    u["W1"][0, 0] = 1.0
    u["W2"][0, 0] = 2.0
    u["W3"][0, 0] = 3.0
    X = np.zeros((2, P.NFEAT))
    X[:, 0] = [0.5, -1.0]
    prob, _ = P.forward(p, X)
    e3 = math.exp(3.0)
    np.testing.assert_allclose(prob[0], [e3 / (e3 + 3), 1 / (e3 + 3), 1 / (e3 + 3), 1 / (e3 + 3)])
    np.testing.assert_allclose(prob[1], 0.25)


def test_mlp_gradient_finite_differences():
    p = _rand_params(1)
    rng = np.random.default_rng(2)
    X = rng.normal(0, 1.5, (40, P.NFEAT))
    y = rng.integers(0, 4, 40)
    _, g = P.loss_grad(p, X, y)
    t0 = 2 * P.NFEAT                      # mu and sigma are not trained
    assert np.all(g[:t0] == 0.0)
    idx = np.concatenate([np.arange(t0, t0 + 30),
                          rng.choice(np.arange(t0 + 30, P.NPARAM), 200, replace=False),
                          np.arange(P.NPARAM - 4, P.NPARAM)])
    h = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += h
        lp = P.loss(q, X, y)
        q[i] -= 2 * h
        lm = P.loss(q, X, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_is_signed_lr():
    p = _rand_params(3)
    g = np.random.default_rng(4).normal(0, 1, P.NPARAM)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    q, m1, v1 = P.adam_step(p, g, m, v, 1, 1e-3, eps=0.0)
    # bias-corrected first step: m_hat = g, v_hat = g^2
    t0 = 2 * P.NFEAT
    np.testing.assert_allclose(q[t0:], p[t0:] - 1e-3 * np.sign(g[t0:]), rtol=0, atol=1e-15)
    np.testing.assert_array_equal(q[:t0], p[:t0])
    np.testing.assert_allclose(m1[t0:], 0.1 * g[t0:])
    np.testing.assert_allclose(v1[t0:], 0.001 * g[t0:] ** 2)
