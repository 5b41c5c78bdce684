"""Pins of the learned-warm-start reference (oracle/mlp.py): gradients against
central finite differences, feature invariances, targets, and the warm-started
subspace iteration against the exact eigendecomposition."""
import numpy as np
import pytest

from paper_2406_09769_amd import inputs
from oracle import dm, mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    w = mlp.init_weights(1) + 0.1 * rng.standard_normal(mlp.N_PARAMS)
    X = rng.standard_normal((17, mlp.F_IN))
    y = rng.uniform(0, 1, 17)
    _, g = mlp.loss_and_grad(w, X, y)
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    for i in idx:
        e = np.zeros_like(w)
        e[i] = h
        fd = (mlp.loss_and_grad(w + e, X, y)[0] - mlp.loss_and_grad(w - e, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd))


def test_output_is_a_probability_and_loss_is_mse():
    rng = np.random.default_rng(1)
    w = mlp.init_weights(2)
    X = rng.standard_normal((9, mlp.F_IN))
    out, _ = mlp.forward(w, X)
    assert np.all((out > 0) & (out < 1))
    y = rng.uniform(0, 1, 9)
    assert abs(mlp.loss_and_grad(w, X, y)[0] - np.mean((out - y) ** 2)) < 1e-15


def _harvest(net, chi, env):
    st = dm.Stats()
    dm.contract_approx(net, chi, env, stats=st, harvest=True)
    return [(L, k) for L, k, *_ in st.harvest]


def test_features_are_scale_invariant_and_bounded():
    L, k = _harvest(inputs.ising_2d(8, 8, 0.44), 8, 1)[10]
    f = mlp.features(L, 2, True)
    g = mlp.features(3.7e5 * L, 2, True)
    assert np.allclose(f, g, atol=1e-13)
    assert np.all(f[:, [0, 2, 3, 4, 5, 6]] >= -1e-15) and np.all(f[:, [0, 2, 3, 4, 5, 6]] <= 1 + 1e-12)


def test_leverage_sums_to_kept_rank():
    for L, k in _harvest(inputs.ising_2d(7, 7, 0.5), 6, 1)[:8]:
        U, _, kk, _ = dm.keep(L, 6)
        t = mlp.leverage(U)
        assert abs(t.sum() - kk) < 1e-12 and np.all(t <= 1 + 1e-12)


def test_warm_subspace_converges_to_exact_subspace():
    for L, k in _harvest(inputs.ising_2d(8, 8, 0.44), 8, 1)[5:15]:
        U, w, kk, _ = dm.keep(L, 8)
        p = min(kk + 2, L.shape[0])
        th, X, res = mlp.warm_subspace(L, np.diag(L), p, 6)
        assert np.allclose(th[:kk], w[:kk], rtol=1e-9, atol=1e-14 * w[0])
        P = X[:, :kk] @ X[:, :kk].T
        assert np.max(np.abs(P - U @ U.T)) < 1e-6
        assert np.max(res[:kk]) <= 1e-6 * th[0]


def test_training_lowers_the_loss_on_harvested_matrices():
    rows, ys = [], []
    for L, k in _harvest(inputs.ising_2d(10, 10, 0.44), 8, 1):
        U, _, kk, _ = dm.keep(L, 8)
        rows.append(mlp.features(L, 2, L.shape[0] > 4))
        ys.append(mlp.leverage(U))
    X, y = np.concatenate(rows), np.concatenate(ys)
    w = mlp.init_weights(3)
    l0 = mlp.loss_and_grad(w, X, y)[0]
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for t in range(1, 301):               # Adam
        _, g = mlp.loss_and_grad(w, X, y)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        w -= 1e-2 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
    assert mlp.loss_and_grad(w, X, y)[0] < 0.5 * l0


# ---------------------------------------------------------------- the learned solve's acceptance rule

def _psd(rng, w):
    n = len(w)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * w) @ Q.T, Q


def _proj(U):
    return U @ U.T


def test_orth_drop_keeps_independent_and_drops_dependent_columns():
    rng = np.random.default_rng(5)
    a, b, u = rng.standard_normal((3, 20))
    u /= np.linalg.norm(u)
    na = np.linalg.norm(a)
    # a + b and 0 are dependent; a new part of 1e-9 (squared 1e-18 > DROP_REL) survives
    Q = mlp.orth_drop(np.column_stack([a, b, a + b, np.zeros(20), a + 1e-9 * na * u]))
    assert Q.shape[1] == 3
    assert np.allclose(Q.T @ Q, np.eye(3), atol=1e-12)
    for v in (a, b, u):
        assert np.linalg.norm(v - Q @ (Q.T @ v)) <= 1e-5 * np.linalg.norm(v)
    # a new part of 1e-14 (squared 1e-28 < DROP_REL) is dropped
    Q2 = mlp.orth_drop(np.column_stack([a, b, a + 1e-14 * na * u]))
    assert Q2.shape[1] == 2


def test_learned_solve_exact_when_the_rank_fits_the_subspace():
    # rank 6 PSD matrix, n = 24 with rows (bond 12, leaf 2); the subspace (6+... p=10)
    # holds the whole range: accepted at the first iteration, same projector and rank
    rng = np.random.default_rng(6)
    w = np.concatenate([np.geomspace(1.0, 1e-9, 6), np.zeros(18)])
    L, _ = _psd(rng, w)
    ok, U, k, why = mlp.learned_solve(L, mlp.init_weights(3), 16, 2)
    Ue, _, ke, _ = dm.keep(L, 16)
    assert ok and why is None and k == ke == 6
    # the weakest kept direction (eigenvalue 1e-9) is only fixed to ~eps/1e-9 by any
    # FP64 solver: compare what the projector captures of L
    P, Pe = _proj(U), _proj(Ue)
    assert np.abs(P @ L @ P - Pe @ L @ Pe).max() <= 1e-13


def test_learned_solve_rejects_an_invariant_subspace_that_misses_weight():
    # block-diagonal L; the start columns all lie in the first block, so V stays an exact
    # invariant subspace (zero residual) while the second block's leading eigenvalue
    # exceeds the kept ones: the trace certificate must refuse it at every iteration
    rng = np.random.default_rng(7)
    A, _ = _psd(rng, np.geomspace(1.0, 1e-3, 16))
    B, _ = _psd(rng, np.array([0.5, 0.2] + [0.0] * 14))
    L = np.zeros((32, 32))
    L[:16, :16], L[16:, 16:] = A, B
    scores = np.concatenate([np.ones(16), np.zeros(16)])
    ok, U, k, why = mlp.learned_solve(L, None, 8, 0, scores=scores)
    assert not ok and why == "cut"
    # the same matrix with scores that reach both blocks is accepted
    scores2 = np.zeros(32)
    scores2[[0, 1, 2, 3, 16, 17, 4, 5, 6, 7, 8, 9]] = 1.0
    ok2, U2, k2, why2 = mlp.learned_solve(L, None, 8, 0, scores=scores2)
    Ue, _, ke, _ = dm.keep(L, 8)
    if ok2:
        assert k2 == ke and np.abs(_proj(U2) - _proj(Ue)).max() <= 1e-4


def test_learned_solve_capped_rank_matches_exact_projector():
    # geometric spectrum, the rank is capped by chi: accepted projectors agree with the
    # exact top-chi subspace to the bound the residual check gives (Davis-Kahan:
    # sin(angle) <= ||R|| / gap)
    rng = np.random.default_rng(8)
    w = 0.2 ** np.arange(40)
    L, _ = _psd(rng, w)
    chi = 8
    ok, U, k, why = mlp.learned_solve(L, None, chi, 0, scores=np.diag(L).copy(), residual_tol=1e-9)
    Ue, _, ke, _ = dm.keep(L, chi)
    assert ok and k == ke == chi
    gap = w[chi - 1] - w[chi]
    assert np.abs(_proj(U) - _proj(Ue)).max() <= 2 * np.sqrt(chi) * 1e-9 / gap


def test_learned_solve_too_small_a_saving_goes_to_the_exact_solve():
    L, _ = _psd(np.random.default_rng(9), np.geomspace(1, 1e-3, 8))
    assert mlp.learned_solve(L, None, 8, 0, scores=np.ones(8))[3] == "size"


def test_learned_solve_on_method_density_matrices_matches_keep():
    # on density matrices the method produces (a 12x12 lattice at chi 16) every accepted
    # solve keeps the exact rank and spans the exact subspace to the residual bound
    net = inputs.ising_2d(12, 12, 0.44)
    acc = 0
    for L, _ in _harvest(net, 16, 1):
        n = L.shape[0]
        rest = 2 if n > 4 else 0
        ok, U, k, why = mlp.learned_solve(L, None, 16, rest, scores=np.diag(L).copy())
        if not ok:
            continue
        acc += 1
        Ue, we, ke, _ = dm.keep(L, 16)
        assert k <= ke
        if k == ke:
            gap = we[k - 1] - (we[k] if k < n else 0.0)
            assert np.abs(_proj(U) - _proj(Ue)).max() <= max(1e-8, 4e-6 * we[0] * np.sqrt(k) / gap)
        else:   # the cutoff form may drop eigen-directions whose weight is below TAIL_REL
            assert we[k:ke].sum() <= 2 * mlp.TAIL_REL * we[0] * n
    assert acc > 0
