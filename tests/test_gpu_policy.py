"""GPU parity of the learned precision policy through the C-ABI against the
CPU oracle (oracle/policy.py): node features, quantization-error labels, the
perceptron's forward pass, gradient and Adam step; then a small training run
and what the trained policy gains over the fixed trees.

Bars: features within 1e-5 (absolute, on log2 scales; the device computes in
FP64 and stores FP32); errors e(p) within 1e-9 relative, labels equal except
where e(p) is within 1e-9 of the budget; perceptron (FP32) within 1e-5
relative of the FP64 oracle (probabilities, loss, gradient in norm, and
entrywise against the gradient's largest entry); Adam step within FP32
rounding of the oracle's update.
"""
import numpy as np
import pytest

import oracle as O
import oracle.policy as OP
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


CASES = [(300, 1.3, 64, 1), (777, 1.05, 64, 32), (1024, 4.0, 128, 1), (129, 2.0, 16, 1)]


@pytest.mark.parametrize("n,ratio,leaf,align", CASES)
def test_features_vs_oracle(M, ctx, n, ratio, leaf, align):
    print(f"[gpu] policy features n={n}", flush=True)
    A = spdgen.gen_spd(n, ratio, 0.25, seed=n + 3)
    t = M.Tree(leaf=leaf, offdiag=[M.F16], split_align=align)
    nodes = M.policy_nodes(n, t)
    assert [tuple(r) for r in nodes] == [(a, b, c, d) for (a, b, c, d) in OP.nodes(n, leaf, align)]
    F = ctx.policy_features(M.to_device_cm(A), n, t).cpu().numpy()
    Fo = OP.features(A, n, leaf, align)
    assert F.shape == Fo.shape
    np.testing.assert_allclose(F, Fo, rtol=0, atol=1e-5)


def test_features_closed_form_on_gpu(M, ctx):
    n, leaf, a, beta = 200, 16, 3.0, -0.125
    A = np.asfortranarray(a * np.eye(n) + beta * np.ones((n, n)))
    t = M.Tree(leaf=leaf)
    F = ctx.policy_features(M.to_device_cm(A), n, t).cpu().numpy()
    assert np.allclose(F[:, 0], np.log2(abs(beta) / np.sqrt(a + beta)), atol=1e-6)
    assert np.allclose(F[:, 1], 0.0, atol=1e-6)
    assert np.allclose(F[:, 2], np.log2((a + beta) / ((n - 1) * abs(beta))), atol=1e-6)


@pytest.mark.parametrize("n,ratio,leaf,align", CASES)
def test_labels_vs_oracle(M, ctx, n, ratio, leaf, align):
    print(f"[gpu] policy labels n={n}", flush=True)
    A = spdgen.gen_spd(n, ratio, 0.25, seed=n + 7)
    L = O.factor(A, tree=O.Tree(leaf=leaf, offdiag=[O.F64], split_align=align))[0]
    t = M.Tree(leaf=leaf, offdiag=[M.F16], split_align=align)
    for tau, sm in ((1e-4, 1), (1e-7, 1), (1e-4, 0)):
        lab, err = ctx.policy_labels(M.to_device_cm(A), M.to_device_cm(L), n, t, tau=tau,
                                     scale_mode=sm)
        lab, err = lab.cpu().numpy(), err.cpu().numpy()
        eo = OP.node_errors(A, L, n, leaf, align, scale_mode=sm)
        bo = OP.budgets(n, leaf, align, tau)
        np.testing.assert_allclose(err, eo, rtol=1e-9, atol=0)
        lo = OP.labels_from(eo, bo)
        close = np.any(np.abs(eo - bo[:, None]) <= 1e-9 * bo[:, None], axis=1)
        assert np.all((lab == lo) | close), (lab, lo)


def _params(seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, OP.NPARAM).astype(np.float32)
    p[:5] = rng.normal(0, 1, 5)
    p[5:10] = rng.uniform(0.5, 2.0, 5)
    return p


def test_mlp_forward_vs_oracle(M, ctx):
    import torch
    p = _params(11)
    X = np.random.default_rng(12).normal(0, 2, (1000, 5)).astype(np.float32)
    probs, cls = ctx.mlp_forward(torch.from_numpy(X).cuda(), torch.from_numpy(p).cuda())
    po, _ = OP.forward(p.astype(np.float64), X.astype(np.float64))
    np.testing.assert_allclose(probs.cpu().numpy(), po, rtol=1e-5, atol=1e-7)
    top = np.sort(po, axis=1)
    safe = top[:, -1] - top[:, -2] > 1e-4
    assert np.all(cls.cpu().numpy()[safe] == np.argmax(po, axis=1)[safe])


@pytest.mark.parametrize("rows", [1, 64, 300])
def test_mlp_gradient_and_adam_vs_oracle(M, ctx, rows):
    import torch
    p = _params(21 + rows)
    rng = np.random.default_rng(22)
    X = rng.normal(0, 2, (rows, 5)).astype(np.float32)
    y = rng.integers(0, 4, rows).astype(np.int32)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    pd = torch.from_numpy(p).cuda()
    loss, grad = ctx.mlp_train_step(Xd, yd, pd, None, None, 1, 0.0, want_grad=True)
    lo, go = OP.loss_grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.int64))
    g = grad.cpu().numpy().astype(np.float64)
    assert float(loss.item()) == pytest.approx(lo, rel=1e-5)
    assert np.linalg.norm(g - go) <= 1e-5 * np.linalg.norm(go)
    assert np.max(np.abs(g - go)) <= 1e-5 * np.max(np.abs(go))
    np.testing.assert_array_equal(pd.cpu().numpy(), p)   # lr = 0 leaves params alone
    # one Adam step from zero moments, lr 1e-3
    m = torch.zeros_like(pd)
    v = torch.zeros_like(pd)
    ctx.mlp_train_step(Xd, yd, pd, m, v, 1, 1e-3)
    q, mo, vo = OP.adam_step(p.astype(np.float64), g, np.zeros(OP.NPARAM), np.zeros(OP.NPARAM),
                             1, 1e-3)
    np.testing.assert_allclose(pd.cpu().numpy(), q, rtol=0, atol=2e-6)
    np.testing.assert_allclose(m.cpu().numpy(), mo, rtol=1e-6, atol=1e-12)
    # 1 - beta2 in FP32 is 1 - fl(0.999) = 0.00099998713 (relative 1.3e-5 from 0.001)
    np.testing.assert_allclose(v.cpu().numpy(), vo, rtol=3e-5, atol=1e-14)


@pytest.fixture(scope="module")
def trained(M, ctx):
    """A small policy trained on the device: 48 matrices n in [512, 1536]."""
    from paper_2601_08082_amd import policy as P
    tree = P.policy_tree(leaf=128)
    ns, rs, ss = P.training_recipe(48, 512, 1536, seed=31)
    X, y = P.build_dataset(ctx, ns, rs, ss, tree)
    params, hist = P.train(ctx, X, y, epochs=150, batch=256, lr=3e-3, seed=1)
    return dict(tree=tree, X=X, y=y, params=params, hist=hist, P=P)


def test_training_learns_labels(M, ctx, trained):
    print("[gpu] policy training", flush=True)
    h = trained["hist"]
    assert h[-1] < 0.5 * h[0], h[::10]
    P = trained["P"]
    assert P.accuracy(ctx, trained["X"], trained["y"], trained["params"]) >= 0.9
    # held-out matrices: predictions against the oracle's labels
    ns, rs, ss = P.training_recipe(6, 512, 1536, seed=32)
    from paper_2601_08082_amd import spdgen_gpu
    hit = tot = 0
    for n, r, sd in zip(ns, rs, ss):
        A = spdgen_gpu.gen_spd(n, r, 0.0, seed=sd)
        Ah = M.from_device_cm(A)
        Lo = O.factor(Ah, tree=O.Tree(leaf=128, offdiag=[O.F64]))[0]
        lo = OP.labels_from(OP.node_errors(Ah, Lo, n, 128), OP.budgets(n, 128, 1, 1e-4))
        ch = ctx.policy_choose(A, n, trained["tree"], trained["params"])
        hit += int(np.sum(np.array(ch) == lo))
        tot += len(lo)
    assert hit >= 0.8 * tot, (hit, tot)


def test_choose_is_argmax_of_forward(M, ctx, trained):
    from paper_2601_08082_amd import spdgen_gpu
    n = 1000
    A = spdgen_gpu.gen_spd(n, 1.5, 0.0, seed=77)
    t = trained["tree"]
    ch = ctx.policy_choose(A, n, t, trained["params"])
    _, cls = ctx.mlp_forward(ctx.policy_features(A, n, t), trained["params"])
    assert ch == cls.cpu().numpy().tolist()


def _cost(M, n, tree):
    st = M.plan_stats(n, tree)
    peak = {"E4M3": 5000.0, "F16": 2500.0, "F32": 157.3, "F64": 78.6}
    return sum(v / (peak[k] * 1e12) for k, v in st["flops"].items())


@pytest.mark.parametrize("ratio", [1.05, 8.0])
def test_policy_gain(M, ctx, trained, ratio):
    """The learned tree solves to 1e-12 like the fixed trees, at a fraction of
    the all-FP64 tree's modelled MFMA time, and is the cheapest tree whose
    error bound (the sum over nodes of the label error e_k of the node's
    chosen format) stays inside the budget tau: on a strongly dominant matrix
    it takes FP8 where the fixed tree takes FP16 (lower modelled cost); on a
    weakly dominant one it keeps FP16 where an all-FP8 tree's bound exceeds
    the budget."""
    from paper_2601_08082_amd import spdgen_gpu
    P = trained["P"]
    n, tau = 1536, 1e-4
    A = spdgen_gpu.gen_spd(n, ratio, 0.0, seed=99)
    B = spdgen_gpu.gen_rhs(n, 1, seed=199)
    X, info = P.solve_with_policy(ctx, A, B, n, trained["params"], tree=trained["tree"])
    assert info["used"] == "learned" and info["fallbacks"] == 0
    Ah, Bh = M.from_device_cm(A), M.from_device_cm(B)
    xs = np.linalg.solve(Ah[:n, :n], Bh[:n])
    x = M.from_device_cm(X)[:n]
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-12
    t = trained["tree"]
    choice = np.array(info["node_prec"])
    learned = M.Tree(leaf=t.leaf, offdiag=[M.F16], scale_mode=1, node_prec=list(choice))
    f16 = M.Tree(leaf=t.leaf, offdiag=[M.F16], scale_mode=1)
    f64 = M.Tree(leaf=t.leaf, offdiag=[M.F64])
    c_l, c_16, c_64 = _cost(M, n, learned), _cost(M, n, f16), _cost(M, n, f64)
    # error bounds from the oracle's node errors (FP64 factor of the same A)
    L64 = O.factor(Ah, tree=O.Tree(leaf=t.leaf, offdiag=[O.F64]))[0]
    e = OP.node_errors(Ah, L64, n, t.leaf, 1, scale_mode=1)
    e4 = np.concatenate([e, np.zeros((e.shape[0], 1))], axis=1)   # F64: no quantization error
    bound_l = float(np.sum(e4[np.arange(len(choice)), choice]))
    bound_e4m3 = float(np.sum(e[:, O.E4M3]))
    be_l = O.backward_error(Ah, M.from_device_cm(ctx.factor(A, n, learned)[0]))
    print(f"[gpu] policy gain ratio {ratio}: choice {choice.tolist()} cost learned/f16/f64 "
          f"{c_l:.3e}/{c_16:.3e}/{c_64:.3e} bound learned {bound_l:.2e} all-e4m3 {bound_e4m3:.2e} "
          f"backward error {be_l:.2e}", flush=True)
    assert c_l <= 0.5 * c_64 and bound_l <= tau and be_l <= tau
    if ratio > 4:
        assert c_l < c_16
    else:
        assert bound_e4m3 > tau and c_l <= c_16
