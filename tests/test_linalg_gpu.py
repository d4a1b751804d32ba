"""GPU checks of the batched dense primitives of the construction against
LAPACK (numpy) through the test hooks of include/h2_testing.h."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
h2 = pytest.importorskip("paper_2003_10173_amd")
L = h2.lib


def F(a):
    return np.asfortranarray(a, dtype=np.float64)


def gemm(ta, tb, A, B, Cm, alpha=1.0, beta=0.0):
    A, B, Cm = F(A), F(B), F(Cm.copy())
    M, N = Cm.shape
    K = A.shape[0] if ta else A.shape[1]
    h2.check(L().h2_test_gemm(ta, tb, M, N, K, alpha, A.ctypes.data, A.shape[0], B.ctypes.data,
                              B.shape[0], beta, Cm.ctypes.data, M), "gemm")
    return Cm


@pytest.mark.parametrize("M,N,K", [(5, 7, 3), (64, 64, 64), (130, 33, 70), (20, 30, 5000),
                                   (100, 1, 4099), (1, 1, 1)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_matches_numpy(M, N, K, ta, tb):
    g = np.random.default_rng(M * 7 + N + K)
    A = g.standard_normal((K, M) if ta else (M, K))
    B = g.standard_normal((N, K) if tb else (K, N))
    C0 = g.standard_normal((M, N))
    got = gemm(ta, tb, A, B, C0, alpha=0.5, beta=-2.0)
    want = 0.5 * (A.T if ta else A) @ (B.T if tb else B) - 2.0 * C0
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max()) * np.sqrt(K)


def qr(A):
    A = F(A)
    m, n = A.shape
    k = min(m, n)
    Q = np.zeros((m, k), order="F")
    R = np.zeros((k, n), order="F")
    h2.check(L().h2_test_qr(m, n, A.ctypes.data, Q.ctypes.data, R.ctypes.data), "qr")
    return Q, R


@pytest.mark.parametrize("m,n,rank", [(50, 20, 20), (64, 102, 64), (300, 40, 7), (3000, 60, 60),
                                      (9000, 30, 30), (10, 10, 0), (33, 1, 1)])
def test_qr_backward_stable_and_matches_lapack(m, n, rank):
    g = np.random.default_rng(m + n)
    A = g.standard_normal((m, rank)) @ g.standard_normal((rank, n)) if rank else np.zeros((m, n))
    Q, R = qr(A)
    k = min(m, n)
    assert np.abs(Q.T @ Q - np.eye(k)).max() <= 1e-13 * max(1, m / 100)
    assert np.abs(Q @ R - A).max() <= 1e-13 * max(1.0, np.abs(A).max()) * np.sqrt(m)
    assert np.allclose(np.triu(R), R)
    Rl = np.linalg.qr(A, mode="r")
    # same Householder sign convention as LAPACK: R agrees up to rounding
    if rank == min(m, n):
        assert np.abs(np.abs(R) - np.abs(Rl)).max() <= 1e-11 * max(1.0, np.abs(Rl).max())


def svd(A):
    A = F(A)
    m, n = A.shape
    s = np.zeros(n)
    U = np.zeros((m, n), order="F")
    V = np.zeros((n, n), order="F")
    h2.check(L().h2_test_svd(m, n, A.ctypes.data, s.ctypes.data, U.ctypes.data, V.ctypes.data), "svd")
    return s, U, V


@pytest.mark.parametrize("m,n,decay", [(40, 40, 0.0), (102, 64, 0.3), (200, 64, 0.6),
                                       (256, 256, 0.1), (70, 70, 1.0), (665, 104, 0.2),
                                       (600, 600, 0.02), (1100, 100, 0.1), (97, 97, 0.0),
                                       (1024, 1024, 0.01), (1024, 1000, 0.05)])
def test_jacobi_svd_matches_lapack(m, n, decay):
    """Square, tall and ragged shapes on both Jacobi kernels, up to the
    multi-workgroup kernel's largest matrix (1024 x 1024)."""
    g = np.random.default_rng(m * n)
    U0 = np.linalg.qr(g.standard_normal((m, n)))[0]
    V0 = np.linalg.qr(g.standard_normal((n, n)))[0]
    sv = np.exp(-decay * np.arange(n))
    A = U0 @ np.diag(sv) @ V0.T
    s, U, V = svd(A)
    sl = np.linalg.svd(A, compute_uv=False)
    assert np.abs(s - sl).max() <= 1e-14 * sl[0] * n
    assert np.all(np.diff(s) <= 0)
    keep = s > 1e-10 * s[0]
    assert np.abs(U[:, keep].T @ U[:, keep] - np.eye(keep.sum())).max() <= 1e-12
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-12
    assert np.abs(U[:, keep] * s[keep] @ V[:, keep].T - A).max() <= 1e-12 * sl[0] * n



def test_svd_rejects_shapes_beyond_its_limits():
    """More than 1024 columns, or fewer rows than columns, is H2_EINVAL
    (checked on the host before anything is launched)."""
    for shape in ((1100, 1025), (10, 20)):
        with pytest.raises(h2.H2Error) as e:
            svd(np.ones(shape))
        assert e.value.status == -1

def test_svd_ordering_with_nan_column_is_a_permutation():
    """Singular values are ordered by a ranking that treats NaN as below every
    number, so the ordering is a permutation even for non-finite input: the
    finite values come first, descending, the NaN last, and the factors of the
    finite columns are untouched (one-workgroup Jacobi path: a pair with a
    NaN column is never rotated)."""
    g = np.random.default_rng(5)
    A = g.standard_normal((40, 6)) * np.array([1.0, 3.0, 0.5, 2.0, 5.0, 0.25])
    A[:, 2] = np.nan
    s, U, V = svd(A)
    assert np.isnan(s[-1]) and np.all(np.isfinite(s[:-1]))
    assert np.all(np.diff(s[:-1]) <= 0)
    B = np.delete(A, 2, axis=1)
    assert np.abs(s[:-1] - np.linalg.svd(B, compute_uv=False)).max() <= 1e-13 * s[0]


def test_jacobi_wait_limit_reports_nan():
    """The multi-workgroup Jacobi orders its rounds by bounded waits on
    per-block round counters.  With the poll limit forced to zero from the
    host every wait gives up at once: the kernel still ends normally and the
    call's singular values are NaN.  The default limit restores exact results."""
    g = np.random.default_rng(11)
    A = g.standard_normal((200, 160))
    L().h2_test_svd_spin_limit(0)
    try:
        s, _, _ = svd(A)
    finally:
        L().h2_test_svd_spin_limit(1 << 22)
    assert np.all(np.isnan(s))
    s2, _, _ = svd(A)
    sl = np.linalg.svd(A, compute_uv=False)
    assert np.abs(s2 - sl).max() <= 1e-14 * sl[0] * 160


def test_jacobi_svd_batch_uneven():
    """Several matrices of uneven sizes in one call (small and multi-workgroup
    ones mixed, odd block counts, a ragged last block)."""
    g = np.random.default_rng(7)
    shapes = [(665, 111), (96, 96), (300, 250), (50, 30), (130, 97), (400, 399), (64, 64)]
    mats, svs = [], []
    for (m, n) in shapes:
        U0 = np.linalg.qr(g.standard_normal((m, n)))[0]
        V0 = np.linalg.qr(g.standard_normal((n, n)))[0]
        sv = np.exp(-0.05 * np.arange(n)) * g.uniform(0.5, 2.0)
        mats.append(U0 @ np.diag(sv) @ V0.T)
        svs.append(sv)
    ms = np.array([m for m, _ in shapes], dtype=np.int32)
    ns = np.array([n for _, n in shapes], dtype=np.int32)
    A = np.concatenate([F(a).ravel(order="F") for a in mats])
    S = np.zeros(int(ns.sum()))
    U = np.zeros(A.size)
    V = np.zeros(int((ns.astype(np.int64) ** 2).sum()))
    h2.check(L().h2_test_svd_batch(len(shapes), ms.ctypes.data, ns.ctypes.data, A.ctypes.data,
                                   S.ctypes.data, U.ctypes.data, V.ctypes.data), "svd batch")
    oa = os_ = ov = 0
    for (m, n), a in zip(shapes, mats):
        s = S[os_:os_ + n]
        u = U[oa:oa + m * n].reshape((m, n), order="F")
        v = V[ov:ov + n * n].reshape((n, n), order="F")
        sl = np.linalg.svd(a, compute_uv=False)
        assert np.abs(s - sl).max() <= 1e-14 * sl[0] * n, (m, n)
        assert np.abs(u.T @ u - np.eye(n)).max() <= 1e-12, (m, n)
        assert np.abs(v.T @ v - np.eye(n)).max() <= 1e-12, (m, n)
        assert np.abs(u * s @ v.T - a).max() <= 1e-12 * sl[0] * n, (m, n)
        oa += m * n
        os_ += n
        ov += n * n


def cholqr(A, mode):
    A = F(A)
    m, n = A.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    h2.check(L().h2_test_cholqr(m, n, A.ctypes.data, Q.ctypes.data, R.ctypes.data, mode),
             "cholqr")
    return Q, R



def test_tall_qr_rejects_shapes_beyond_its_limits():
    """TSQR takes at most 96 columns; both tall QRs need m >= n; the hook's
    mode is 0..3.  Each is H2_EINVAL from a host check."""
    for shape, mode in (((500, 97), 0), ((50, 60), 0), ((50, 60), 1), ((50, 20), 4)):
        with pytest.raises(h2.H2Error) as e:
            cholqr(np.ones(shape), mode)
        assert e.value.status == -1, (shape, mode)

@pytest.mark.parametrize("m,n,rank,blocked", [(2048, 74, 74, 0), (900, 42, 10, 0), (500, 96, 96, 0),
                                              (300, 20, 20, 0), (97, 96, 50, 0), (3000, 40, 40, 0),
                                              (1281, 64, 30, 0), (320, 96, 96, 0),
                                              (2048, 600, 600, 1), (1500, 300, 120, 1),
                                              (700, 130, 130, 1)])
def test_tall_qr_orthonormal_and_backward_stable(m, n, rank, blocked):
    g = np.random.default_rng(m + 3 * n)
    U = np.linalg.qr(g.standard_normal((m, rank)))[0]
    sv = np.logspace(0, -12, rank)
    A = (U * sv) @ g.standard_normal((rank, n))
    Q, R = cholqr(A, blocked)
    # Householder nodes: Q orthonormal to rounding for full-rank input; when
    # later panels are numerically dependent on earlier ones, orthogonality
    # of the noise directions is ~1e-10 while the factorisation stays backward
    # stable (the construction only uses the significant directions)
    tol = 1e-12 if (rank == n or not blocked) else 1e-9
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= tol
    assert np.linalg.norm(Q @ R - A) <= 1e-13 * np.linalg.norm(A)
    assert np.allclose(np.triu(R), R)
    # same singular values as the input (backward stability)
    s1 = np.linalg.svd(A, compute_uv=False)
    s2 = np.linalg.svd(R, compute_uv=False)
    assert np.abs(s1 - s2).max() <= 1e-13 * s1[0]


@pytest.mark.parametrize("m,n,rank", [(191, 96, 96), (192, 96, 60), (1700, 88, 88), (3000, 150, 150),
                                      (900, 130, 40), (150, 140, 140), (400, 7, 7)])
def test_qr_by_shape_r_only_matches_gram(m, n, rank):
    """The shape-dispatched QR: R alone satisfies R^T R = A^T A (Gram factor
    use) and matches the full factorisation's R up to row signs."""
    g = np.random.default_rng(11 * m + n)
    U = np.linalg.qr(g.standard_normal((m, rank)))[0]
    sv = np.logspace(0, -10, rank)
    A = (U * sv) @ g.standard_normal((rank, n))
    Q, R = cholqr(A, 2)
    _, R3 = cholqr(A, 3)
    nA = np.linalg.norm(A, 2)
    assert np.linalg.norm(Q @ R - A) <= 1e-13 * np.linalg.norm(A)
    assert np.allclose(np.triu(R), R) and np.allclose(np.triu(R3), R3)
    assert np.abs(R3.T @ R3 - A.T @ A).max() <= 1e-13 * nA * nA
    assert np.abs(np.abs(R3) - np.abs(R)).max() <= 1e-12 * nA
