"""Reference for the learned warm start of the eigensolve (TEST INFRASTRUCTURE ONLY).

The learned form replaces the full eigensolve of a density matrix L by a few steps
of subspace iteration started from columns of L chosen by a small MLP (an addition of
this implementation; the paper always computes leading eigenvectors exactly). This module gives
the plain numpy definition of every piece, independent of the GPU code:

* row features of a density matrix (bond-local: diagonal weight, row weight,
  position of the row's bond index and leaf index, matrix size);
* the training target: the leverage of each row in the kept leading subspace,
  sum_{j<k} U_ij^2;
* the MLP 8 -> 32 -> 32 -> 1 (tanh, tanh, logistic) with its loss
  (mean squared error) and the gradients by backpropagation;
* the warm-started subspace iteration with Rayleigh-Ritz and the residual check;
* the acceptance rule of the learned solve (when its subspace may stand in for the
  full eigensolve) and the rank it keeps.
"""
from __future__ import annotations

import numpy as np

F_IN, H1, H2 = 8, 32, 32
N_PARAMS = F_IN * H1 + H1 + H1 * H2 + H2 + H2 + 1


def features(L: np.ndarray, rest: int, bonded: bool) -> np.ndarray:
    """Row features of a symmetric PSD matrix whose rows are (bond index, leaf index).

    rest: the leaf dimension (rows are bond-major); bonded: whether the leading row
    mode is an MPS bond (False for the first tree vertex, whose rows are two leaves).
    """
    n = L.shape[0]
    d = np.diag(L).copy()
    dmax = d.max() if n else 0.0
    tr = d.sum()
    rn2 = (L * L).sum(axis=1)
    fro2 = rn2.sum()
    f = np.zeros((n, F_IN))
    safe = lambda a, b: np.where(b > 0, a / np.where(b > 0, b, 1.0), 0.0)
    rel = safe(d, dmax) if dmax > 0 else np.zeros(n)
    f[:, 0] = rel
    f[:, 1] = np.log10(np.maximum(rel, 1e-30)) / 15.0
    f[:, 2] = safe(d, tr) if tr > 0 else 0.0
    f[:, 3] = np.sqrt(safe(rn2, fro2)) if fro2 > 0 else 0.0
    f[:, 4] = np.where((d > 0) & (tr > 0), rn2 / np.where(d * tr > 0, d * tr, 1.0), 0.0)
    i = np.arange(n)
    if bonded:
        nb = n // rest
        f[:, 5] = (i // rest) / max(1, nb - 1)
        f[:, 6] = (i % rest) / max(1, rest - 1)
    else:
        f[:, 5] = i / max(1, n - 1)
        f[:, 6] = 0.0
    f[:, 7] = n / 128.0
    return f


def leverage(U: np.ndarray) -> np.ndarray:
    """Target: squared row norms of the kept orthonormal basis (sum = kept rank)."""
    return (U * U).sum(axis=1)


# ------------------------------------------------------------------ the MLP

def unpack(w: np.ndarray):
    o = 0
    W1 = w[o:o + F_IN * H1].reshape(F_IN, H1); o += F_IN * H1
    b1 = w[o:o + H1]; o += H1
    W2 = w[o:o + H1 * H2].reshape(H1, H2); o += H1 * H2
    b2 = w[o:o + H2]; o += H2
    W3 = w[o:o + H2]; o += H2
    b3 = w[o]; o += 1
    assert o == N_PARAMS
    return W1, b1, W2, b2, W3, b3


def init_weights(seed: int) -> np.ndarray:
    """Glorot-uniform layers, zero biases (for tests that pass weights explicitly)."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in ((F_IN, H1), (H1, H2)):
        lim = np.sqrt(6.0 / (a + b))
        parts += [rng.uniform(-lim, lim, a * b), np.zeros(b)]
    lim = np.sqrt(6.0 / (H2 + 1))
    parts += [rng.uniform(-lim, lim, H2), np.zeros(1)]
    return np.concatenate(parts)


def forward(w, X):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    z1 = X @ W1 + b1
    h1 = np.tanh(z1)
    z2 = h1 @ W2 + b2
    h2 = np.tanh(z2)
    z3 = h2 @ W3 + b3
    out = 1.0 / (1.0 + np.exp(-z3))
    return out, (X, h1, h2, out)


def loss_and_grad(w, X, y):
    """Mean squared error over the batch and its gradient by backpropagation."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    out, (X_, h1, h2, _) = forward(w, X)
    B = X.shape[0]
    r = out - y
    loss = float(np.mean(r * r))
    g_out = 2.0 * r / B
    g_z3 = g_out * out * (1.0 - out)
    gW3 = h2.T @ g_z3
    gb3 = g_z3.sum()
    g_h2 = np.outer(g_z3, W3)
    g_z2 = g_h2 * (1.0 - h2 * h2)
    gW2 = h1.T @ g_z2
    gb2 = g_z2.sum(axis=0)
    g_h1 = g_z2 @ W2.T
    g_z1 = g_h1 * (1.0 - h1 * h1)
    gW1 = X_.T @ g_z1
    gb1 = g_z1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return loss, grad


# ------------------------------------------------------------------ warm-started subspace iteration

def warm_subspace(L, scores, p, iters):
    """Columns of L at the p highest scores, then `iters` steps of V <- orth(L V),
    Rayleigh-Ritz on V^T L V. Returns (Ritz values desc, Ritz vectors, residuals)."""
    idx = np.argsort(-scores, kind="stable")[:p]
    V, _ = np.linalg.qr(L[:, idx])
    for _ in range(iters):
        V, _ = np.linalg.qr(L @ V)
    H = V.T @ L @ V
    th, Y = np.linalg.eigh(0.5 * (H + H.T))
    th, Y = th[::-1], Y[:, ::-1]
    X = V @ Y
    res = np.linalg.norm(L @ X - X * th, axis=0)
    return th, X, res


# ------------------------------------------------------------------ the learned solve and its acceptance rule

DROP_REL = 1e-26      # a start column whose new part has squared norm <= DROP_REL * its own is dropped
TAIL_REL = 1e-13      # weight allowed outside the subspace when the cutoff (not chi) decides the rank:
                      # the rank rule's floor at the default cutoff (0.1 x 1e-12)
FRO_SLACK = 1e-13     # relative rounding allowance of the Frobenius-norm bound
REASONS = ("size", "dependent", "cut", "residual")


def orth_drop(V: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the columns of V taken in order (Gram-Schmidt, applied
    twice), leaving out every column whose part outside the span of the earlier ones
    has squared norm <= DROP_REL times its own (all-zero columns included)."""
    n, p = V.shape
    Q = np.zeros((n, 0))
    for j in range(p):
        v = V[:, j]
        nv2 = float(v @ v)
        u = v - Q @ (Q.T @ v)
        u = u - Q @ (Q.T @ u)
        nu2 = float(u @ u)
        if nv2 > 0.0 and nu2 > DROP_REL * nv2:
            Q = np.column_stack([Q, u / np.sqrt(nu2)])
    return Q


def rank_rule(theta: np.ndarray, navail: int, n: int, chi: int, tau_rel: float, tau_deg: float,
              floor: float) -> int:
    """The keep rule of the density-matrix step applied to descending values theta
    (navail of them) of a matrix of order n: at most chi, drop values <= tau_rel*theta_1,
    never cut where the values do not separate (theta_k - theta_{k+1} <= tau_deg*theta_k
    with theta_{k+1} above floor*theta_1)."""
    w1 = theta[0]
    k = min(chi, n, navail)
    while k >= 1 and theta[k - 1] <= tau_rel * w1:
        k -= 1
    while 1 <= k < navail and theta[k] > floor * w1 and theta[k - 1] - theta[k] <= tau_deg * theta[k - 1]:
        k -= 1
    return k


def subspace_size(n: int, chi: int, rest: int) -> int:
    """Columns of the warm start: 4 more than the rank the step can keep, where the
    bond (n // rest rows' worth) bounds it, and at most n - 1."""
    kprev = n // rest if rest > 0 else n
    return min((kprev if (rest > 0 and kprev < chi) else chi) + 4, n - 1)


def learned_solve(L, w, chi, rest, residual_tol=1e-6, tau_rel=1e-12, tau_deg=0.1, floor=1e-13, iters=3,
                  scores=None):
    """The learned solve of one density matrix, step by step.

    1. Score every row of L with the MLP on its features; take the columns of L at the
       p best scores (ties to the lower row), p = subspace_size.
    2. Orthonormalise them (orth_drop); then up to `iters` times: W = L V, H = V^T W,
       Ritz pairs (theta, y) of H in descending order, kept rank k by the keep rule on
       theta padded with zeros to p values.
    3. Bound the largest eigenvalue of L on the complement of span(V) by
       b = min(t, f) with t = tr(L) - tr(H) and f = sqrt(max(0, ||L||^2 - 2||W||^2 +
       ||H||^2) + FRO_SLACK * ||L||^2) (Frobenius norms). Accept when the weight outside
       is below the rank rule's floor, t <= floor * theta_1, or when b cannot move a cut that chi
       decides (k = min(chi, n), b <= theta_k / 2 and b < (1 - tau_deg) theta_k),
       and every kept Ritz pair has ||W y - theta V y|| <= residual_tol * theta (relative
       to its own Ritz value: the smallest kept directions must be resolved too).
       Else V <- orth_drop(W) and repeat.

    scores, when given, replaces the MLP's row scores (tests of the rule itself).
    Returns (accepted, U (n x k) or None, k, reason) with reason None or one of REASONS.
    Identities behind the bound: with P = VV^T, V orthonormal and C = (I-P) L (I-P),
    tr(C) = tr(L) - tr(H) and, for PSD L, C is PSD so its largest eigenvalue is at most
    tr(C); also ||L||^2 = ||H||^2 + 2||(I-P)LV||^2 + ||C||^2 and ||W||^2 = ||H||^2 +
    ||(I-P)LV||^2, so ||C||^2 = ||L||^2 - 2||W||^2 + ||H||^2 (FRO_SLACK covers its
    rounding).
    """
    L = 0.5 * (L + L.T)
    n = L.shape[0]
    p = subspace_size(n, chi, rest)
    if n < 16 or p < 2 or 4 * p > 3 * n:
        return False, None, 0, "size"
    if scores is None:
        scores = forward(w, features(L, rest if rest > 0 else n, rest > 0))[0]
    idx = np.argsort(-scores, kind="stable")[:p]
    V = orth_drop(L[:, idx])
    if V.shape[1] == 0:
        return False, None, 0, "dependent"
    trL = float(np.trace(L))
    fro2L = float((L * L).sum())
    kmax = min(chi, n)
    reason = "cut"
    for _ in range(iters):
        W = L @ V
        H = V.T @ W
        H = 0.5 * (H + H.T)
        th, Y = np.linalg.eigh(H)
        th, Y = th[::-1], Y[:, ::-1]
        thp = np.concatenate([th, np.zeros(p - len(th))])
        k = rank_rule(thp, p, n, chi, tau_rel, tau_deg, floor)
        t = max(trL - float(np.trace(H)), 0.0)
        f = np.sqrt(max(fro2L - 2.0 * float((W * W).sum()) + float((H * H).sum()), 0.0) + FRO_SLACK * fro2L)
        b = min(t, f)
        th1 = thp[0]
        ok = k >= 1 and th1 > 0
        if ok:
            thk = thp[k - 1]
            ok = t <= floor * th1 or (k == kmax and b <= 0.5 * thk and b < thk - tau_deg * thk)
        if ok:
            Xr = V @ Y[:, :k]
            R = W @ Y[:, :k] - Xr * th[:k]
            if (np.linalg.norm(R, axis=0) / th[:k]).max() <= residual_tol:
                return True, Xr, k, None
            reason = "residual"
        else:
            reason = "cut"
        V = orth_drop(W)
        if V.shape[1] == 0:
            return False, None, 0, "dependent"
    return False, None, 0, reason
