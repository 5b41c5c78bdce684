"""Device kernels through the C-ABI diagnostics, against plain numpy FP64.

GEMM: the contraction GEMM (FP64 matrix cores, index-table gathers) on ragged,
strided and transposed operands and two-level index maps.
Eigensolve: kept subspace (projector) and rank versus numpy's eigh and the
oracle's keep rule. Rescale: exact powers of two."""
import numpy as np
import pytest

from oracle import dm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2406_09769_amd import tnapprox
    return tnapprox


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (64, 64, 16), (65, 63, 17), (200, 130, 70),
                                   (3, 257, 129), (128, 128, 256)])
def test_gemm_matches_numpy(T, M, N, K):
    rng = np.random.default_rng(M * 1000 + N + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    C = T.tn_debug_gemm(A, B)
    ref = A @ B
    assert np.max(np.abs(C - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))) * max(1, K) ** 0.5


@pytest.mark.parametrize("lo", [1, 7, 64])
def test_gemm_strided_and_two_level_maps(T, lo):
    rng = np.random.default_rng(lo)
    A = rng.standard_normal((90, 37)).T          # A is a transposed view (m stride 1)
    B = rng.standard_normal((51, 90)).T[:, ::1]  # B(k, n) with n stride 90
    C = T.tn_debug_gemm(A, B, lo_split=lo)
    assert np.allclose(C, A @ B, rtol=0, atol=1e-12)


def _psd(n, spectrum, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return q @ np.diag(spectrum) @ q.T


@pytest.mark.parametrize("n", [2, 3, 4, 7, 15, 16, 17, 31, 33, 48, 63, 64, 65, 97, 98, 99, 127, 128,
                               129, 135, 136, 193, 256, 257, 384, 511, 512])   # above 135: global scratch
def test_eig_subspace_and_rank_match_oracle(T, n):
    rng = np.random.default_rng(n)
    w = np.sort(np.exp(-rng.uniform(0, 30, n)))[::-1]
    L = _psd(n, w, n + 1)
    ucols = max(1, n // 2)
    U, fb = T.tn_debug_eig(L, ucols)
    Uo, wo, k, _ = dm.keep(L, ucols)
    kept = int(np.sum(np.any(U != 0.0, axis=0)))
    assert kept == k and fb == 0
    assert np.all(U[:, k:] == 0.0)
    Uk = U[:, :k]
    assert np.allclose(Uk.T @ Uk, np.eye(k), atol=1e-12)
    # both solvers are backward stable (error ~eps*||L||), so their kept subspaces
    # agree to first order within eps*||L|| / gap at the cut; what the subspace
    # captures of L agrees within a few n*eps*||L|| whatever the gap
    eps = np.finfo(float).eps
    gap = wo[k - 1] - (wo[k] if k < n else 0.0)
    P, Po = Uk @ Uk.T, Uo @ Uo.T
    assert np.max(np.abs(P - Po)) < max(1e-9, 4 * eps * wo[0] / gap)
    assert np.max(np.abs(P @ L @ P - Po @ L @ Po)) < 10 * n * eps * wo[0]


def _hard_spectra(n, rng):
    """Spectra that stress a tridiagonal solver's deflation: geometric decay over 35
    orders, exact triples, a rank-deficient matrix (zeros), one eigenvalue repeated n
    times, and n eigenvalues within 1e-9 of each other."""
    yield "geometric", np.sort(np.exp(-rng.uniform(0, 35, n)))[::-1]
    yield "triples", np.repeat(np.exp(-2.0 * np.arange((n + 2) // 3)), 3)[:n]
    w = np.zeros(n)
    r = max(1, n // 4)
    w[:r] = np.sort(np.exp(-rng.uniform(0, 5, r)))[::-1]
    yield "rank_deficient", w
    yield "flat", np.ones(n)
    yield "near_flat", np.sort(1.0 + 1e-9 * rng.standard_normal(n))[::-1]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 16, 24, 32, 40, 47, 56, 63, 64, 65, 80, 91, 100, 127, 128])
def test_eig_divide_and_conquer_matches_ql_and_oracle(T, n):
    """The divide-and-conquer tridiagonal solve (orders up to 64 in LDS, 65 to 128 with its
    second eigenvector buffer and merge matrices in global scratch) against the QL solve and
    the oracle: same kept rank, orthonormal vectors, and kept subspaces that agree within
    eps ||L|| / gap at the cut (both solvers are backward stable)."""
    rng = np.random.default_rng(100 + n)
    eps = np.finfo(float).eps
    for name, w in _hard_spectra(n, rng):
        L = _psd(n, w, n + 7)
        ucols = max(1, n // 2)
        Ud, fbd = T.tn_debug_eig(L, ucols, tridiag=T.TN_TRIDIAG_AUTO)
        Uq, fbq = T.tn_debug_eig(L, ucols, tridiag=T.TN_TRIDIAG_QL)
        Uo, wo, k, fbo = dm.keep(L, ucols)
        kd = int(np.sum(np.any(Ud != 0.0, axis=0)))
        kq = int(np.sum(np.any(Uq != 0.0, axis=0)))
        assert (kd, fbd) == (kq, fbq) == (k, int(fbo)), (name, kd, kq, k)
        Uk = Ud[:, :k]
        assert np.allclose(Uk.T @ Uk, np.eye(k), atol=1e-12), name
        if fbo:                      # nothing separates: any orthonormal choice is valid
            continue
        gap = wo[k - 1] - (wo[k] if k < n else 0.0)
        P, Pq, Po = Uk @ Uk.T, Uq[:, :k] @ Uq[:, :k].T, Uo @ Uo.T
        bound = max(1e-9, 8 * n * eps * wo[0] / gap)
        assert np.max(np.abs(P - Po)) < bound, (name, np.max(np.abs(P - Po)), bound)
        assert np.max(np.abs(P - Pq)) < bound, (name, np.max(np.abs(P - Pq)), bound)
        assert np.max(np.abs(P @ L @ P - Po @ L @ Po)) < 10 * n * eps * wo[0], name


def test_eig_does_not_split_degenerate_cluster(T):
    w = np.array([1.0, 0.5, 0.25, 0.25, 0.1, 0.0])
    L = _psd(6, w, 3)
    U, _ = T.tn_debug_eig(L, 3)
    assert int(np.sum(np.any(U != 0.0, axis=0))) == 2


def test_eig_zero_padding_is_invisible(T):
    rng = np.random.default_rng(9)
    a = rng.standard_normal((20, 20))
    L = a @ a.T
    Lp = np.zeros((40, 40))
    Lp[:20, :20] = L
    U, _ = T.tn_debug_eig(Lp, 16)
    k = int(np.sum(np.any(U != 0.0, axis=0)))
    assert k == dm.keep(L, 16)[2]
    assert np.all(U[20:, :] == 0.0)


def test_eig_zero_matrix_falls_back(T):
    U, fb = T.tn_debug_eig(np.zeros((8, 8)), 4)
    assert fb == 1


@pytest.mark.parametrize("scale", [1.0, 3e-200, 7e250, -2.5])
def test_rescale_is_exact_power_of_two(T, scale):
    x = np.random.default_rng(1).standard_normal(1000) * scale
    y, e = T.tn_debug_rescale(x)
    _, want = np.frexp(np.max(np.abs(x)))
    assert e == want
    assert np.array_equal(y, np.ldexp(x, -e))


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("M,N,K", [(5, 300, 37), (30, 130, 70), (90, 77, 51), (16, 512, 4), (64, 64, 16)])
def test_gemm_split_precision_within_its_bound(T, precision, M, N, K):
    """Split BF16 / FP16 products against the FP64 product. Bound, element by element:
    |C - AB| <= 2^-20 (|A||B|): each value is carried to ~2^-24 relative by its three
    parts, the dropped part products are below 2^-24 |a||b|, and the FP32 sums of the
    six products over K add a few 2^-24 of the running sum; operands are scaled to a
    common power of two first, so the bound holds at any magnitude."""
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.standard_normal((M, K)) * np.exp(rng.uniform(-3, 0, (M, K)))
    B = rng.standard_normal((K, N)) * np.exp(rng.uniform(-3, 0, (K, N)))
    for scale in (1.0, 2.0 ** 40, 2.0 ** -37):
        C = T.tn_debug_gemm(A * scale, B, precision=precision)
        ref = (A * scale) @ B
        bound = 2.0 ** -20 * (np.abs(A * scale) @ np.abs(B))
        assert np.all(np.abs(C - ref) <= bound + 1e-300), (precision, scale, np.max(np.abs(C - ref) / bound))
        # and it is not exact FP64 arithmetic in disguise: the error is at the split level
        if precision == 1 and scale == 1.0 and K >= 16:
            assert np.max(np.abs(C - ref)) > 0


def _operands(M, N, K, layout, rng):
    """A (M x K) and B (K x N) as views whose fast mode is k (A) / n (B) for "kn", or
    m (A) / k (B) for "mk"."""
    if layout == "kn":
        return rng.standard_normal((M, K)), rng.standard_normal((K, N))
    return rng.standard_normal((K, M)).T, rng.standard_normal((N, K)).T


CHIP_SHAPES = [(1, 1, 1), (3, 257, 5), (16, 513, 17), (20, 300, 40), (32, 129, 33), (64, 64, 16), (130, 200, 37),
               (300, 70, 1100), (700, 65, 600), (70, 90, 2100), (40, 33, 10300)]
# at least 2^16 columns, at most 32 rows and 32-deep K: the streaming kernel (one shape per K
# class, ragged column counts); the last two take the split-K path (few tiles, long K)
STREAM_SHAPES = [(4, 65536, 3), (8, 70001, 8), (32, 65539, 16), (17, 66000, 32), (33, 65536, 8), (32, 32, 8192),
                 (32, 2048, 2048)]


@pytest.mark.parametrize("layout", ["kn", "mk"])
@pytest.mark.parametrize("M,N,K", CHIP_SHAPES + STREAM_SHAPES)
def test_gemm_chip_wide_fp64(T, M, N, K, layout):
    """The launch of a contraction too large for one workgroup (row + k offsets within
    the LDS cache: pipelined tiles; few rows and shallow K over many columns: the streaming
    kernel; else the plain tiled kernel, with K split into parts when few tiles would
    leave the chip idle), against numpy."""
    rng = np.random.default_rng(M * 31 + N * 7 + K)
    A, B = _operands(M, N, K, layout, rng)
    C = T.tn_debug_gemm(A, B, chip_wide=True)
    ref = A @ B
    assert np.max(np.abs(C - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))) * max(1, K) ** 0.5


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("layout", ["kn", "mk"])
@pytest.mark.parametrize("M,N,K", CHIP_SHAPES)
def test_gemm_chip_wide_split_within_its_bound(T, precision, M, N, K, layout):
    """Chip-wide split BF16 / FP16 products within |C - AB| <= 2^-20 (|A||B|), element by
    element. Rows of A and columns of B are scaled by powers of two up to 2^±40 apart:
    every row of an A chunk and every column of a B chunk carries its own scale, so the
    bound holds however far apart their magnitudes lie (FP16 parts alone span 2^-24..2^16)."""
    rng = np.random.default_rng(M * 13 + N * 5 + K + precision)
    A, B = _operands(M, N, K, layout, rng)
    A = A * np.exp(rng.uniform(-3, 0, A.shape)) * 2.0 ** rng.integers(-40, 41, (M, 1))
    B = B * np.exp(rng.uniform(-3, 0, B.shape)) * 2.0 ** rng.integers(-40, 41, (1, N))
    C = T.tn_debug_gemm(A, B, precision=precision, chip_wide=True)
    ref = A @ B
    bound = 2.0 ** -20 * (np.abs(A) @ np.abs(B))
    assert np.all(np.abs(C - ref) <= bound + 1e-300), (precision, np.max(np.abs(C - ref) / bound))
    if K >= 16:   # the split level, not FP64 arithmetic
        assert np.max(np.abs(C - ref)) > 0
