"""GPU parity of HGEMV (Sec. 3.2 four-stage product) against the oracle.

Oracle-built H2 matrices are imported into the device layout through the C ABI
and applied to seeded vectors; FP64 must match the oracle's product within
1e-12 relative (a handful of reordered sums per entry).
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.h2 import H2Matrix as OH2
from oracle.hessians import KernelHessian, tree_order
from oracle.ns import build as obuild, power_norm
from oracle.tree import Tree as OTree
from tests.h2_helpers import oracle_to_packed, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
h2 = pytest.importorskip("paper_2003_10173_amd")


def _random_h2(T, kmax, seed, kmin=0):
    g = np.random.Generator(np.random.PCG64(seed))
    H = OH2(T)
    L = T.L
    for l in range(2, L + 1):
        H.rank[l][:] = g.integers(kmin, kmax + 1, size=1 << l)
    for i in range(1 << L):
        H.U[i] = g.standard_normal((T.size(L, i), H.rank[L][i]))
    for l in range(1, L + 1):
        for i in range(1 << l):
            H.E[l][i] = g.standard_normal((H.rank[l][i], H.rank[l - 1][i // 2]))
        for (t, s) in T.far[l]:
            H.S[l][(t, s)] = g.standard_normal((H.rank[l][t], H.rank[l][s]))
    for (t, s) in T.near:
        H.D[(t, s)] = g.standard_normal((T.size(L, t), T.size(L, s)))
    return H


@pytest.fixture(scope="module")
def kernel1d():
    cfg = si.config_kernel1d()
    T = OTree(cfg["points"], cfg["leaf"], cfg["eta"])
    K = KernelHessian(cfg["points"], cfg["ell"], cfg["shift"])
    A = tree_order(K.apply, T.perm)
    nu, _ = power_norm(A, T.n, cfg["seed"])
    H, _ = obuild(A, T, cfg["tol"], nu, cfg["cap"], cfg["p"], adaptive=False, seed=cfg["seed"])
    return cfg, T, H


def _run(H, T, nv, seed, alpha=1.0, beta=0.0):
    gt = h2.Tree(T.points, T.leaf_size, T.eta)
    G = h2.H2Matrix.from_host(gt, *oracle_to_packed(H))
    x = si.gaussian_vectors(T.n, nv, seed)
    y0 = si.gaussian_vectors(T.n, nv, seed + 1)
    xd = torch.tensor(x.T.copy(), device="cuda")
    yd = torch.tensor(y0.T.copy(), device="cuda")
    G.gemv(xd, yd, alpha=alpha, beta=beta)
    torch.cuda.synchronize()
    want = alpha * H.matvec(x) + beta * y0
    return yd.cpu().numpy().T, want, G


@pytest.mark.parametrize("nv", [1, 16, 33])
def test_hgemv_kernel1d_matches_oracle(kernel1d, nv):
    cfg, T, H = kernel1d
    got, want, _ = _run(H, T, nv, 101)
    assert rel_err(got, want) <= 1e-12


@pytest.mark.parametrize("shape,leaf,kmax,nv", [
    ((2100, 2), 64, 12, 7),       # ragged leaves, random ranks incl. zero
    ((777, 1), 20, 6, 64),        # 1D, leaf 20, many vectors
    ((1500, 3), 32, 9, 40),       # 3D, two column chunks with a ragged tail
])
def test_hgemv_random_h2_matches_oracle(shape, leaf, kmax, nv):
    pts = np.random.Generator(np.random.PCG64(shape[0])).uniform(size=shape)
    T = OTree(pts, leaf, 0.7)
    H = _random_h2(T, kmax, 3)
    got, want, G = _run(H, T, nv, 5, alpha=0.75, beta=-1.5)
    assert rel_err(got, want) <= 1e-12
    r, U, E, S, D = G.export()
    r0, U0, E0, S0, D0 = oracle_to_packed(H)
    assert np.array_equal(r, r0) and np.array_equal(D, D0) and np.array_equal(S, S0)


def test_hgemv_single_leaf_and_identity():
    T = OTree(np.linspace(0, 1, 40), 64, 0.7)     # L = 0: one dense leaf
    H = _random_h2(T, 0, 1)
    got, want, _ = _run(H, T, 3, 2)
    assert rel_err(got, want) <= 1e-13
    gt = h2.Tree(np.linspace(0, 1, 300), 32, 0.7)
    I = h2.H2Matrix.identity(gt, 2.5)
    x = torch.randn(4, 300, dtype=torch.float64, device="cuda")
    assert torch.allclose(I.gemv(x), 2.5 * x, rtol=0, atol=0)


def test_hgemv_reduced_precision_storage(kernel1d):
    cfg, T, H = kernel1d
    gt = h2.Tree(T.points, T.leaf_size, T.eta)
    G = h2.H2Matrix.from_host(gt, *oracle_to_packed(H))
    x = si.gaussian_vectors(T.n, 16, 7)
    want = H.matvec(x)
    xf = torch.tensor(x.T.copy(), device="cuda", dtype=torch.float32)
    for prec, tol in ((h2.H2_FP64, 1e-6), (h2.H2_FP32, 1e-6), (h2.H2_BF16, 1e-2)):
        Gp = G if prec == h2.H2_FP64 else G.convert(prec)
        y = Gp.gemv(xf)
        torch.cuda.synchronize()
        assert rel_err(y.cpu().numpy().T, want) <= tol, prec


@pytest.mark.parametrize("nv", [5, 33, 70])
def test_hgemv_reduced_precision_ragged_random(nv):
    """FP32 (FP32 matrix cores) and BF16 (BF16 operands, FP32 accumulation)
    on a random 2D H2 with ragged leaves of up to 64 and several vector
    tiles.  Bounds from the arithmetic: FP32 storage and products carry
    2^-24 relative rounding per term (sums of ~1.7k terms: 1e-5 relative);
    BF16 rounds both operands to 2^-9 relative, so each product is off by at
    most 2^-8 relative, 2e-2 on the result after cancellation in a
    random-sign sum."""
    pts = np.random.Generator(np.random.PCG64(99)).uniform(size=(2500, 2))
    T = OTree(pts, 64, 0.7)
    H = _random_h2(T, 10, 4)
    gt = h2.Tree(pts, 64, 0.7)
    G = h2.H2Matrix.from_host(gt, *oracle_to_packed(H))
    x = si.gaussian_vectors(T.n, nv, 8)
    want = H.matvec(x)
    xf = torch.tensor(x.T.copy(), device="cuda", dtype=torch.float32)
    for prec, tol in ((h2.H2_FP32, 1e-5), (h2.H2_BF16, 2e-2)):
        y = G.convert(prec).gemv(xf)
        torch.cuda.synchronize()
        err = rel_err(y.cpu().numpy().T, want)
        assert err <= tol, (prec, err)
        if prec == h2.H2_BF16:
            assert err >= 1e-5   # the BF16 path really rounds its operands


@pytest.mark.parametrize("nv", [7, 20, 64, 70])
def test_hgemv_tile_widths_agree_and_tuner_picks_one(nv):
    """Every matrix-core tile width gives the same product (the same sums in
    the same order); the autotuner records one of them for the tree."""
    from paper_2003_10173_amd._lib import lib
    pts = np.random.Generator(np.random.PCG64(31)).uniform(size=(1800, 2))
    T = OTree(pts, 64, 0.7)
    H = _random_h2(T, 12, 6)
    gt = h2.Tree(pts, 64, 0.7)
    G = h2.H2Matrix.from_host(gt, *oracle_to_packed(H))
    x = torch.tensor(si.gaussian_vectors(T.n, nv, 4).T.copy(), device="cuda")
    outs = []
    for nt in (1, 2, 4):
        y = torch.empty_like(x)
        h2.check(lib().h2_test_gemv_tile(G.handle, nv, x.data_ptr(), y.data_ptr(), nt), "tile")
        outs.append(y.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    y = G.gemv(x)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), outs[0])
    assert lib().h2_test_tuned_tile(G.handle, nv) in (1, 2, 4)


@pytest.mark.parametrize("nv", [20, 64])
def test_hgemv_split_far_lists(nv):
    """Couplings of large rank on few tiles: the far lists are split over
    workgroups (partial sums added in group order by the last to arrive).
    Every tile width gives the same sums, the product matches the oracle's,
    and the unsplit product (the entry point that allocates nothing) agrees
    to rounding."""
    from paper_2003_10173_amd._lib import lib
    pts = np.random.Generator(np.random.PCG64(37)).uniform(size=(1500, 2))
    T = OTree(pts, 64, 0.7)
    H = _random_h2(T, 64, 8, kmin=40)
    gt = h2.Tree(pts, 64, 0.7)
    G = h2.H2Matrix.from_host(gt, *oracle_to_packed(H))
    assert lib().h2_test_gemv_split_groups(G.handle, nv) > 1
    x = torch.tensor(si.gaussian_vectors(T.n, nv, 6).T.copy(), device="cuda")
    outs = []
    for nt in (1, 2, 4):
        y = torch.empty_like(x)
        h2.check(lib().h2_test_gemv_tile(G.handle, nv, x.data_ptr(), y.data_ptr(), nt), "tile")
        outs.append(y.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    y = G.gemv(x)
    y_na = torch.empty_like(x)
    G.gemv_noalloc(x, y_na)
    torch.cuda.synchronize()
    want = H.matvec(si.gaussian_vectors(T.n, nv, 6))
    got = y.cpu().numpy().T
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    assert float((y - y_na).abs().max() / y_na.abs().max()) <= 1e-13


def test_hgemv_empty_and_invalid_calls():
    """No vectors is a valid call that leaves y untouched, through all three
    entry points; a negative count or a leading dimension below n is
    H2_EINVAL (host checks, nothing is launched)."""
    n = 300
    gt = h2.Tree(np.linspace(0, 1, n), 32, 0.7)
    I = h2.H2Matrix.identity(gt, 2.0)
    for dt in (torch.float64, torch.float32):
        x = torch.empty(0, n, dtype=dt, device="cuda")
        assert I.gemv(x).shape == (0, n)
    x0 = torch.empty(0, n, dtype=torch.float64, device="cuda")
    assert I.gemv_noalloc(x0, torch.empty_like(x0)).shape == (0, n)
    x = torch.randn(2, n, dtype=torch.float64, device="cuda")
    y = torch.full_like(x, 7.0)
    lib = h2._lib.lib()
    p = h2._ptr
    for f in (lib.h2_gemv, lib.h2_gemv_noalloc):
        assert f(I.handle, 0, 1.0, None, n, 0.0, None, n, None) == 0
        assert f(I.handle, -1, 1.0, p(x), n, 0.0, p(y), n, None) == -1
        assert f(I.handle, 2, 1.0, p(x), n - 1, 0.0, p(y), n, None) == -1
        assert f(I.handle, 2, 1.0, p(x), n, 0.0, p(y), n - 1, None) == -1
        assert f(I.handle, 2, 1.0, None, n, 0.0, p(y), n, None) == -1
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
    assert torch.equal(I.gemv(x), 2.0 * x)
