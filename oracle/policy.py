"""CPU oracle of the learned precision policy (TEST INFRASTRUCTURE ONLY).

The paper fixes one precision per recursion level (Section 3.3).  A learned
per-node choice is this project's addition on top of that fixed layering (the
paper's future work, Section 5, names dynamic quantization instead).  The
policy built here picks the precision of every internal Tree-POTRF node (the
node's Tree-TRSM and Tree-SYRK updates, Algorithm 1) from five features of
the input matrix, with a 6-64-64-4 perceptron.  This module is the plain
FP64 reference of every step of it:

  nodes      internal Tree-POTRF nodes in preorder (the numbering of the
             per-node precision override), with their split and depth;
  features   per node, from the lower triangle of A before factorization
             (node = rows/cols [i0, i0+m), split m1, A21 = A[i0+m1:i0+m, i0:i0+m1]):
               f1 = log2( rms(A21) / sqrt(mean diag of the node) )   (-64 if A21 = 0)
               f2 = log2( maxabs(A21) / rms(A21) )                   (0 if A21 = 0)
               f3 = log2( min over the node's rows i of a_ii / sum_{j != i} |a_ij| ),
                    full rows of the symmetric A, clamped to [-30, 30]
               f4 = depth,  f5 = log2(m1)
               f6 = log2( min over the node's rows i of (a_ii - max_{j != i} |a_ij|)
                          / mean diag of the node ), full rows, clamped to [-30, 30]
                    (values <= 2^-30, including <= 0, give -30).  For equal diagonal
                    entries a_ii - |a_ij| is the smaller eigenvalue of the 2 x 2
                    principal submatrix (i, j), an upper bound on lambda_min(A) by
                    interlacing: the one feature that sees a small lambda_min in a
                    matrix that is not diagonally dominant.
  errors     per node and p in (E4M3, F16, F32), with X = L21 of an FP64
             factor (the operand block the node's updates multiply):
               e(p) = 2 ||X||_F ||X - s Q_p(X / s)||_F / ||A_node||_F,
             s the power-of-two block scale of Section 3.4 (scale_mode given),
             ||A_node||_F over the symmetric node block;
  budgets    tau * g * m1^2 / sum over nodes of m1^2, with g the pivot ratio
             min_i l_ii^2 / max_i l_ii^2 of the FP64 factor.  Every pivot
             l_ii^2 is the reciprocal of a diagonal entry of the inverse of a
             leading block of A, so it lies between A's extreme eigenvalues
             and g >= 1 / kappa_2(A).  Refinement (Section 2.2) contracts by
             about kappa times the factor's relative error, so the budget
             shrinks with the conditioning that g indicates;
  labels     the cheapest p (E4M3 < F16 < F32 < F64), not below a floor
             min_prec, with e(p) <= budget;
  mlp        x_hat = (x - mu) / sigma, h1 = relu(W1 x_hat + b1),
             h2 = relu(W2 h1 + b2), z = W3 h2 + b3, p = softmax(z); mean
             cross-entropy loss; its exact gradient; one Adam step.

Only tests import this module; it shares no code with the GPU library.
"""
from __future__ import annotations

import math

import numpy as np

from . import E4M3, F16, F32, F64, round_array, scale, split

H = 64
NCLS = 4
NFEAT = 6
# flat parameter layout: mu(6) sigma(6) W1(64x6) b1(64) W2(64x64) b2(64) W3(4x64) b3(4), row-major
SIZES = [("mu", (NFEAT,)), ("sigma", (NFEAT,)), ("W1", (H, NFEAT)), ("b1", (H,)),
         ("W2", (H, H)), ("b2", (H,)), ("W3", (NCLS, H)), ("b3", (NCLS,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
NTRAIN = NPARAM - 2 * NFEAT   # mu and sigma are fixed by the data, not trained


def unpack(params: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = params[o:o + k].reshape(shp)
        o += k
    return out


# ---------------------------------------------------------------- tree nodes
def nodes(n: int, leaf: int, align: int = 1):
    """Internal Tree-POTRF nodes (m > leaf) in preorder: (i0, m, m1, depth)."""
    out = []

    def rec(i0, m, d):
        if m <= leaf or m <= 0:
            return
        m1 = split(m, align)
        out.append((i0, m, m1, d))
        rec(i0, m1, d + 1)
        rec(i0 + m1, m - m1, d + 1)

    rec(0, n, 0)
    return out


def _sym(A: np.ndarray, n: int) -> np.ndarray:
    """Symmetric matrix from the lower triangle of A[:n, :n]."""
    Lo = np.tril(A[:n, :n])
    return Lo + np.tril(Lo, -1).T


# ---------------------------------------------------------------- features
def features(A: np.ndarray, n: int, leaf: int, align: int = 1) -> np.ndarray:
    S = _sym(A, n)
    d = np.diag(S).copy()
    off = np.abs(S).sum(axis=1) - np.abs(d)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(off > 0, d / off, np.inf)
    Soff = np.abs(S)
    np.fill_diagonal(Soff, 0.0)
    gap = d - Soff.max(axis=1) if n > 1 else d.copy()
    out = []
    for (i0, m, m1, dep) in nodes(n, leaf, align):
        X = S[i0 + m1:i0 + m, i0:i0 + m1]
        rms = math.sqrt(float(np.mean(X * X)))
        mx = float(np.max(np.abs(X)))
        mdiag = float(np.mean(d[i0:i0 + m]))
        if rms > 0.0 and mdiag > 0.0:
            f1 = math.log2(rms / math.sqrt(mdiag))
        elif rms > 0.0:
            f1 = 64.0
        else:
            f1 = -64.0
        f2 = math.log2(mx / rms) if rms > 0.0 else 0.0
        r = float(np.min(ratio[i0:i0 + m]))
        f3 = 30.0 if r >= 2.0 ** 30 else (-30.0 if r <= 2.0 ** -30 else math.log2(r))
        v = float(np.min(gap[i0:i0 + m])) / mdiag
        f6 = 30.0 if v >= 2.0 ** 30 else (-30.0 if v <= 2.0 ** -30 else math.log2(v))
        out.append([f1, f2, f3, float(dep), math.log2(m1), f6])
    return np.array(out, dtype=np.float64).reshape(-1, NFEAT)


# ---------------------------------------------------------------- labels
def quant_dequant(X: np.ndarray, prec: int, scale_mode: int) -> np.ndarray:
    """s * Q_p(X / s) with the block's power-of-two scale (Section 3.4)."""
    mx = float(np.max(np.abs(X))) if X.size else 0.0
    s = scale(mx, prec, scale_mode)
    return round_array(X / s, prec) * s


def node_errors(A: np.ndarray, L: np.ndarray, n: int, leaf: int, align: int = 1,
                scale_mode: int = 1) -> np.ndarray:
    """(nodes x 3) e(p) for p = E4M3, F16, F32."""
    S = _sym(A, n)
    out = []
    for (i0, m, m1, _) in nodes(n, leaf, align):
        X = np.asarray(L[i0 + m1:i0 + m, i0:i0 + m1], dtype=np.float64)
        an = float(np.linalg.norm(S[i0:i0 + m, i0:i0 + m]))
        xn = float(np.linalg.norm(X))
        row = []
        for p in (E4M3, F16, F32):
            dn = float(np.linalg.norm(X - quant_dequant(X, p, scale_mode)))
            row.append(2.0 * xn * dn / an if an > 0 else math.inf)
        out.append(row)
    return np.array(out, dtype=np.float64).reshape(-1, 3)


def pivot_ratio(L: np.ndarray, n: int) -> float:
    """min_i l_ii^2 / max_i l_ii^2 over the diagonal of the factor L[:n, :n]."""
    if n == 0:
        return 1.0
    d = np.diag(np.asarray(L[:n, :n], dtype=np.float64)) ** 2
    return float(d.min() / d.max())


def budgets(n: int, leaf: int, align: int, tau: float, g: float = 1.0) -> np.ndarray:
    s2 = np.array([float(m1) ** 2 for (_, _, m1, _) in nodes(n, leaf, align)])
    return tau * g * s2 / s2.sum() if s2.size else s2


def labels_from(err: np.ndarray, bud: np.ndarray, min_prec: int = E4M3) -> np.ndarray:
    """Cheapest format from min_prec up whose error fits the node's budget."""
    lab = np.full(err.shape[0], F64, dtype=np.int64)
    for i in range(err.shape[0]):
        for p in (E4M3, F16, F32):
            if p >= min_prec and err[i, p] <= bud[i]:
                lab[i] = p
                break
    return lab


# ---------------------------------------------------------------- MLP
def forward(params: np.ndarray, X: np.ndarray):
    """Class probabilities (rows x 4) and the intermediate values."""
    P = unpack(np.asarray(params, dtype=np.float64))
    xh = (X - P["mu"]) / P["sigma"]
    a1 = xh @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["W3"].T + P["b3"]
    zm = z - z.max(axis=1, keepdims=True)
    e = np.exp(zm)
    p = e / e.sum(axis=1, keepdims=True)
    return p, dict(xh=xh, a1=a1, h1=h1, a2=a2, h2=h2, z=z)


def loss(params: np.ndarray, X: np.ndarray, y: np.ndarray) -> float:
    p, _ = forward(params, X)
    return float(-np.mean(np.log(p[np.arange(len(y)), y])))


def loss_grad(params: np.ndarray, X: np.ndarray, y: np.ndarray):
    """Mean cross-entropy and its gradient (mu, sigma entries zero)."""
    P = unpack(np.asarray(params, dtype=np.float64))
    p, c = forward(params, X)
    B = X.shape[0]
    l = float(-np.mean(np.log(p[np.arange(B), y])))
    dz = p.copy()
    dz[np.arange(B), y] -= 1.0
    dz /= B
    g = {"mu": np.zeros(NFEAT), "sigma": np.zeros(NFEAT)}
    g["W3"] = dz.T @ c["h2"]
    g["b3"] = dz.sum(axis=0)
    dh2 = dz @ P["W3"]
    da2 = dh2 * (c["a2"] > 0)
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ P["W2"]
    da1 = dh1 * (c["a1"] > 0)
    g["W1"] = da1.T @ c["xh"]
    g["b1"] = da1.sum(axis=0)
    return l, np.concatenate([g[name].ravel() for name, _ in SIZES])


def adam_step(params, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba) of the trained entries; returns new (params, m, v)."""
    params, m, v = params.copy(), m.copy(), v.copy()
    sl = slice(2 * NFEAT, NPARAM)
    m[sl] = b1 * m[sl] + (1 - b1) * grad[sl]
    v[sl] = b2 * v[sl] + (1 - b2) * grad[sl] ** 2
    mh = m[sl] / (1 - b1 ** t)
    vh = v[sl] / (1 - b2 ** t)
    params[sl] -= lr * mh / (np.sqrt(vh) + eps)
    return params, m, v
