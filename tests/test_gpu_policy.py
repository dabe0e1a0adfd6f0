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
    assert np.allclose(F[:, 5], np.log2((a + beta - abs(beta)) / (a + beta)), atol=1e-6)


LABEL_CASES = CASES + [(500, -0.05, 64, 1), (260, -1e-3, 32, 8)]   # ratio < 0: kernel nugget


@pytest.mark.parametrize("n,ratio,leaf,align", LABEL_CASES)
def test_labels_vs_oracle(M, ctx, n, ratio, leaf, align):
    print(f"[gpu] policy labels n={n} ratio {ratio}", flush=True)
    A = (spdgen.gen_spd(n, ratio, 0.25, seed=n + 7) if ratio > 0
         else spdgen.gen_kernel(n, 0.3, -ratio, seed=n + 7))
    L = O.factor(A, tree=O.Tree(leaf=leaf, offdiag=[O.F64], split_align=align))[0]
    t = M.Tree(leaf=leaf, offdiag=[M.F16], split_align=align)
    g = OP.pivot_ratio(L, n)
    for tau, sm, mp in ((1e-2, 2, O.F16), (1e-2, 2, O.E4M3), (1e-4, 1, O.E4M3), (1e-7, 1, O.F32),
                        (1e-4, 0, O.E4M3)):
        lab, err = ctx.policy_labels(M.to_device_cm(A), M.to_device_cm(L), n, t, tau=tau,
                                     scale_mode=sm, min_prec=mp)
        lab, err = lab.cpu().numpy(), err.cpu().numpy()
        eo = OP.node_errors(A, L, n, leaf, align, scale_mode=sm)
        bo = OP.budgets(n, leaf, align, tau, g)
        np.testing.assert_allclose(err, eo, rtol=1e-9, atol=0)
        lo = OP.labels_from(eo, bo, mp)
        close = np.any(np.abs(eo - bo[:, None]) <= 1e-9 * bo[:, None], axis=1)
        assert np.all((lab == lo) | close), (lab, lo)


def _params(seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, OP.NPARAM).astype(np.float32)
    p[:OP.NFEAT] = rng.normal(0, 1, OP.NFEAT)
    p[OP.NFEAT:2 * OP.NFEAT] = rng.uniform(0.5, 2.0, OP.NFEAT)
    return p


def test_mlp_forward_vs_oracle(M, ctx):
    import torch
    p = _params(11)
    X = np.random.default_rng(12).normal(0, 2, (1000, OP.NFEAT)).astype(np.float32)
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
    X = rng.normal(0, 2, (rows, OP.NFEAT)).astype(np.float32)
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
    """A small policy trained on the device: 64 matrices n in [512, 2048] of
    both input families (dominance ratio and covariance kernel)."""
    from paper_2601_08082_amd import policy as P
    tree = P.policy_tree(leaf=128)
    specs = P.training_recipe(64, 512, 2048, seed=31)
    X, y = P.build_dataset(ctx, specs, tree)
    params, hist = P.train(ctx, X, y, epochs=150, batch=256, lr=3e-3, seed=1)
    return dict(tree=tree, X=X, y=y, params=params, hist=hist, P=P)


def test_training_learns_labels(M, ctx, trained):
    print("[gpu] policy training", flush=True)
    h = trained["hist"]
    assert h[-1] < 0.5 * h[0], h[::10]
    P = trained["P"]
    y = trained["y"].cpu().numpy()
    print(f"[gpu]   label counts {np.bincount(y, minlength=4).tolist()}", flush=True)
    assert np.bincount(y, minlength=4)[O.F32] > 0
    # the covariance family's F16 / F32 boundary is not learned reliably
    # (see the held-out check): a lower bar than a separable set would get
    assert P.accuracy(ctx, trained["X"], trained["y"], trained["params"]) >= 0.85
    # held-out matrices: predictions against the oracle's labels.  The
    # dominance family's labels follow from the features; the covariance
    # family's are reported (its F16 / F32 boundary is not learned reliably)
    hit = {"dominance": 0, "kernel": 0}
    tot = {"dominance": 0, "kernel": 0}
    for sp in P.training_recipe(8, 512, 1536, seed=32):
        n = sp.n
        A = sp.generate()
        Ah = M.from_device_cm(A)
        Lo = O.factor(Ah, tree=O.Tree(leaf=128, offdiag=[O.F64]))[0]
        lo = OP.labels_from(OP.node_errors(Ah, Lo, n, 128, scale_mode=P.SCALE_MODE),
                            OP.budgets(n, 128, 1, P.TAU, OP.pivot_ratio(Lo, n)), P.MIN_PREC)
        ch = ctx.policy_choose(A, n, trained["tree"], trained["params"])
        hit[sp.kind] += int(np.sum(np.array(ch) == lo))
        tot[sp.kind] += len(lo)
    print(f"[gpu]   held-out agreement {hit} of {tot}", flush=True)
    assert tot["dominance"] > 0 and hit["dominance"] >= 0.9 * tot["dominance"], (hit, tot)


def test_choose_is_argmax_of_forward(M, ctx, trained):
    from paper_2601_08082_amd import spdgen_gpu
    n = 1000
    A = spdgen_gpu.gen_spd(n, 1.5, 0.0, seed=77)
    t = trained["tree"]
    ch = ctx.policy_choose(A, n, t, trained["params"])
    _, cls = ctx.mlp_forward(ctx.policy_features(A, n, t), trained["params"])
    assert ch == cls.cpu().numpy().tolist()


GAIN_SYSTEMS = [("dominance", 32768, 1.1, 0.0), ("kernel", 16384, 0.1, 0.1)]


@pytest.mark.parametrize("kind,n,a,b", GAIN_SYSTEMS, ids=[g[0] for g in GAIN_SYSTEMS])
def test_policy_gain(M, ctx, kind, n, a, b):
    """Measured time to a refined solution (correction below 1e-12) with the
    shipped weights (policy_mi355x.npy): the learned tree (its choice of
    precisions included), the fixed all-FP16 tree and the paper's three-level
    tree [F16, F32, F64] (each falling back to FP64 when it does not
    converge), and the all-FP64 tree.  The learned tree must converge without
    a fallback and give the FP64 solution; on the dominant system it must
    beat the FP64 tree and the three-level tree, and stay within 15% of the
    all-FP16 tree it then equals (plus the feature pass).  The covariance system's
    times are reported: the network does not learn that family's FP16 / FP32
    boundary reliably, and the fixed FP16 tree converges there too (more
    refinement steps), so no gain over it is claimed."""
    import torch
    from paper_2601_08082_amd import policy as P
    params = P.load_params()
    tree = P.policy_tree()
    sp = P.MatrixSpec(kind, n, a, b, 99)
    A = sp.generate()
    B = P.spdgen_rhs(n, 199)
    res = P.measure(ctx, A, B, n, params, tree, tol=1e-12, reps=3)
    print(f"[gpu] policy gain {kind} n={n}: " + ", ".join(
        f"{k} {res[k]['tts_ms']:.2f} ms ({res[k]['used']}, {res[k]['ir_iters']} it)"
        for k in ("learned", "fixed", "three_level", "fp64")) +
        f", choice {res['learned']['choice_counts']}, gain vs fixed {res['gain_vs_fixed']:.2f} "
        f"vs three-level {res['gain_vs_three_level']:.2f} vs fp64 {res['gain_vs_fp64']:.2f}",
        flush=True)
    assert res["learned"]["used"] == "learned" and res["learned"]["fallbacks"] == 0
    X, info = P.solve_with_policy(ctx, A, B, n, params, tree=tree)
    assert info["used"] == "learned"
    # backward error of the refined solution, on the device in FP64
    Ad = A[:n, :n]           # row-major view of the column-major matrix: A^T = A
    x = X[0, :n]
    r = B[0, :n] - Ad @ x
    nA = torch.linalg.matrix_norm(Ad, 2) if n <= 4096 else torch.linalg.matrix_norm(Ad, "fro")
    assert float(r.norm() / (nA * x.norm())) <= 1e-14
    if kind == "dominance":
        # the labels admit FP16 at every node, where the paper's three-level
        # tree spends FP32 and FP64 on the inner levels
        assert res["gain_vs_fp64"] > 1.0
        assert res["gain_vs_three_level"] > 1.0
        assert res["gain_vs_fixed"] > 0.85
