"""Pins of the oracle's higher-order inversion forms (Appendix A.2 hyperpower
iteration, Appendix A.3 unrolled iterations from a warm start), of the
minimal-surface Hessian of the Appendix A example and of the global low-rank
pre-pass of Sec. 3.3, against what the mathematics fixes: closed forms through
eigvalsh, equality with plain Newton-Schulz steps, finite differences of the
objective, the flat-surface stencil, exactness for rank-r operators and the
Halko-Martinsson-Tropp error bound."""
import math

import numpy as np
import pytest

import seeded_inputs as si
from oracle import ns as ns_mod
from oracle.h2 import H2Matrix
from oracle.hessians import KernelHessian, MinimalSurface, dense_from_apply, tree_order
from oracle.ns import build, hyperpower_eval, newton_schulz, ns_eval, power_norm
from oracle.tree import Tree


@pytest.fixture(scope="module")
def kernel256():
    cfg = si.config_kernel1d(256)
    T = Tree(cfg["points"], 32, 0.7)
    K = KernelHessian(cfg["points"], 0.1, 1e-2)
    A = tree_order(K.apply, T.perm)
    nu, _ = power_norm(A, T.n, 1, rel=1e-12, max_it=500)
    H, _ = build(A, T, 1e-12, nu, 16, 10, adaptive=True, seed=1)
    lam = np.linalg.eigvalsh(K.dense())
    return T, H, lam


# ----------------------------------------------------------------- hyperpower
def test_hyperpower_order2_sampler_is_newton_schulz(kernel256):
    """Setting l = 2 gives the Newton-Schulz iteration (Appendix A.2): the
    Horner-style sampler of Alg. 4 at l = 2 equals Alg. 3's samples to rounding."""
    T, H, lam = kernel256
    X = H2Matrix.scaled_identity(T, 0.8 / lam[-1])
    Om = si.gaussian_vectors(T.n, 7, 3)
    a = hyperpower_eval(X, H, Om, 2)
    b = ns_eval(X, H, Om)
    assert np.linalg.norm(a - b) <= 1e-14 * np.linalg.norm(b)


@pytest.mark.parametrize("order", [3, 4, 8])
def test_hyperpower_residual_closed_form(kernel256, order):
    """From X0 = I / nu every iterate is a polynomial in A, and
    R_{k+1} = I - A X_k sum_{i<l} R_k^i = R_k^l, so E_k = max_i |1 - lam_i / nu|^(l^k)."""
    T, H, lam = kernel256
    X, info = newton_schulz(H, 1e-6, 20, 32, 10, x0="identity", adaptive=True, seed=3,
                            eps_build=1e-10, nu_rel=1e-12, resid_rel=1e-7, order=order)
    nu = info["nu"]
    rmax = float(np.max(np.abs(1.0 - lam / nu)))
    checked = 0
    for k, E in enumerate(info["E"]):
        want = rmax ** (order ** k)
        if want < 1e-4:
            break
        assert abs(E - want) <= 1e-3 * want, (k, E, want)
        checked += 1
    assert checked >= 2
    assert info["status"] == "converged"
    # l-th order convergence: iterations ~ log_l of those of Newton-Schulz
    kappa = lam[-1] / lam[0]
    bound = math.log(kappa * math.log(1e6), order) + 2
    assert info["iterations"] <= bound + 1


def test_hyperpower_sign_slip_breaks_closed_form(kernel256, monkeypatch):
    """A planted sign slip in Alg. 4 (R <- R + A X R) must break the pin."""
    T, H, lam = kernel256

    def slipped(Xk, A, Om, order):
        Y = Om.copy()
        R = Om.copy()
        for _ in range(order - 1):
            R = R + A.matvec_tree(Xk.matvec_tree(R))
            Y = Y + R
        return Xk.matvec_tree(Y)
    monkeypatch.setattr(ns_mod, "hyperpower_eval", slipped)
    X, info = newton_schulz(H, 0.0, 1, 32, 10, x0="identity", adaptive=True, seed=3,
                            eps_build=1e-10, nu_rel=1e-12, resid_rel=1e-7, order=3)
    rmax = float(np.max(np.abs(1.0 - lam / info["nu"])))
    assert abs(info["E"][1] - rmax ** 3) > 1e-2 * rmax ** 3


# ----------------------------------------------------------------- unrolled, warm start
def test_unrolled_construction_equals_newton_schulz_steps(kernel256):
    """u unrolled steps from a warm start X0 in one construction
    (X_u = X0 sum_{i<2^u} (I - A X0)^i) equal u Newton-Schulz steps from X0
    in exact arithmetic; with tight construction thresholds both agree to the
    construction error, and E = max_i |1 - lam_i x0(lam_i)|^(2^u)."""
    T, H, lam = kernel256
    X0 = H2Matrix.scaled_identity(T, 1.6 / lam[-1])
    u = 3
    Xu, iu = newton_schulz(H, 0.0, 1, 32, 10, x0=X0, adaptive=True, seed=4,
                           eps_build=1e-11, nu_rel=1e-12, resid_rel=1e-7, unroll=u)
    Xn, inn = newton_schulz(H, 0.0, u, 32, 10, x0=X0, adaptive=True, seed=4,
                            eps_build=1e-11, nu_rel=1e-12, resid_rel=1e-7)
    assert iu["iterations"] == 1 and inn["iterations"] == u
    Du, Dn = Xu.dense_tree(), Xn.dense_tree()
    assert np.linalg.norm(Du - Dn, 2) <= 1e-8 * np.linalg.norm(Dn, 2)
    r = 1.0 - 1.6 * lam / lam[-1]
    want = float(np.max(np.abs(r))) ** (2 ** u)
    assert abs(iu["E"][1] - want) <= 1e-3 * want
    assert abs(iu["E"][0] - float(np.max(np.abs(r)))) <= 1e-3


def test_warm_start_converges_in_fewer_iterations(kernel256):
    """The inverse of a nearby matrix as X0 (Appendix A.1: the previous
    optimisation step's inverse) needs fewer iterations than I / nu."""
    T, H, lam = kernel256
    cfg = si.config_kernel1d(256)
    K2 = KernelHessian(cfg["points"], 0.11, 1.2e-2)      # the next step's Hessian
    A2 = tree_order(K2.apply, T.perm)
    nu2, _ = power_norm(A2, T.n, 1)
    H2_, _ = build(A2, T, 1e-10, nu2, 16, 10, adaptive=True, seed=1)
    Xprev, info1 = newton_schulz(H, 1e-6, 60, 32, 10, x0="identity", adaptive=True, seed=5,
                                 eps_build=1e-8)
    assert info1["status"] == "converged"
    Xc, ic = newton_schulz(H2_, 1e-6, 60, 32, 10, x0="identity", adaptive=True, seed=5,
                           eps_build=1e-8)
    Xw, iw = newton_schulz(H2_, 1e-6, 60, 32, 10, x0=Xprev, adaptive=True, seed=5,
                           eps_build=1e-8)
    assert iw["status"] == "converged" and ic["status"] == "converged"
    assert iw["E"][0] < 1.0
    assert iw["iterations"] < ic["iterations"]


# ----------------------------------------------------------------- minimal surface
def test_minsurf_derivatives_by_finite_differences():
    """Gradient and Hessian of the discrete area against central differences
    of the objective and of the gradient: the error falls by 100 per decade of
    the step (second order), so the analytic forms are exact derivatives."""
    H = MinimalSurface(si.config_minsurf2d(16))
    m0 = H.M[1:-1, 1:-1].ravel()
    g = np.random.default_rng(1)
    d = g.standard_normal(H.n)
    d /= np.linalg.norm(d)
    errs_g, errs_h = [], []
    hv = H.apply(d)
    gd = float(H.gradient() @ d)
    for eps in (1e-3, 1e-4):
        fd = (H.objective(m0 + eps * d) - H.objective(m0 - eps * d)) / (2 * eps)
        errs_g.append(abs(fd - gd) / abs(fd))
        fdh = (H.gradient(m0 + eps * d) - H.gradient(m0 - eps * d)) / (2 * eps)
        errs_h.append(np.linalg.norm(fdh - hv) / np.linalg.norm(hv))
    assert errs_g[1] <= 2e-6 and errs_h[1] <= 1e-7
    assert 50 <= errs_g[0] / errs_g[1] <= 200
    assert 50 <= errs_h[0] / errs_h[1] <= 200


def test_minsurf_flat_surface_is_five_point_laplacian():
    cfg = si.config_minsurf2d(12)
    cfg["heights"] = np.zeros_like(cfg["heights"])
    H = MinimalSurface(cfg)
    g = 12
    V = np.random.default_rng(2).standard_normal((H.n, 3))
    P = np.zeros((g + 2, g + 2, 3))
    P[1:-1, 1:-1] = V.reshape(g, g, 3)
    want = 4 * P[1:-1, 1:-1] - P[:-2, 1:-1] - P[2:, 1:-1] - P[1:-1, :-2] - P[1:-1, 2:]
    assert np.abs(H.apply(V) - want.reshape(H.n, 3)).max() <= 1e-13


def test_minsurf_hessian_symmetric_positive_definite():
    H = MinimalSurface(si.config_minsurf2d(16, step=1))
    D = dense_from_apply(H.apply, H.n)
    assert np.abs(D - D.T).max() <= 1e-14 * np.abs(D).max()
    lam = np.linalg.eigvalsh(D)
    assert lam[0] > 0
    # the flat-surface Laplacian bounds: lambda_max < 8 times the largest
    # coefficient 1 / s (s >= 1), so below 8
    assert lam[-1] < 8.0


# ----------------------------------------------------------------- global low rank
def _psd_with_decay(n, seed, rate):
    g = np.random.default_rng(seed)
    Q = np.linalg.qr(g.standard_normal((n, n)))[0]
    lam = np.exp(-rate * np.arange(n))
    return (Q * lam) @ Q.T, lam


def test_global_lowrank_exact_for_rank_r():
    """For H of rank r the range finder with r + p columns is exact:
    B B^T = H to rounding and B has r columns."""
    from oracle.lowrank import global_lowrank
    g = np.random.default_rng(3)
    C = g.standard_normal((300, 12))
    H = C @ C.T
    B, applies = global_lowrank(lambda V: H @ V, 300, 20, 10, seed=5)
    assert applies == 2 * 30
    assert B.shape[1] == 12
    assert np.linalg.norm(B @ B.T - H, 2) <= 1e-12 * np.linalg.norm(H, 2)


def test_global_lowrank_within_hmt_bound():
    """||H - B B^T|| <= 2 (1 + 11 sqrt(r + p) sqrt(n)) lam_{r+1} + lam_{r+1}:
    Halko-Martinsson-Tropp's bound for ||(I - Q Q^T) H||, taken twice for the
    two-sided projection, plus the dropped eigenvalues of T (at most lam_{r+1}
    by interlacing)."""
    from oracle.lowrank import global_lowrank
    n, r, p = 200, 15, 10
    H, lam = _psd_with_decay(n, 4, 0.3)
    B, _ = global_lowrank(lambda V: H @ V, n, r, p, seed=6)
    err = np.linalg.norm(H - B @ B.T, 2)
    assert err <= (2 * (1 + 11 * np.sqrt(r + p) * np.sqrt(n)) + 1) * lam[r]
    # and, as typical for a decaying spectrum, within a small factor of the best
    assert err <= 10 * lam[r]


def test_build_lowrank_recovers_misfit_plus_sparse():
    """Misfit-like global low rank plus a sparse regularisation (diffusion
    Gauss-Newton Hessian on a 16 x 16 grid): the construction of H - B B^T
    with B B^T added back meets the tolerance against the dense Hessian, and
    its Hessian products are the global ones plus the residual construction's."""
    from oracle.hessians import DiffusionGN
    from oracle.lowrank import build_lowrank
    cfg = si.config_diffusion2d(16)
    G = DiffusionGN(cfg)
    T = Tree(cfg["points"], 32, 0.7)
    A = tree_order(G.apply, T.perm)
    H, info = build_lowrank(A, T, 1e-6, 40, 24, 10, seed=2)
    Hd = dense_from_apply(G.apply, cfg["n"])
    err = np.linalg.norm(H.dense_user() - Hd, 2) / np.linalg.norm(Hd, 2)
    assert err <= 1e-6
    assert info["global_rank"] == 40 and info["global_applies"] == 100
    assert info["applies"] == info["global_applies"] + info["residual_applies"]
    # the residual has lost the dominant misfit directions
    Rd = info["residual"].dense_user()
    assert np.linalg.norm(Rd - (Hd - info_B_dense(info, T)), 2) <= 1e-6 * np.linalg.norm(Hd, 2)


def info_B_dense(info, T):
    B = np.empty_like(info["B"])
    B[T.perm] = info["B"]
    return B @ B.T


def test_build_lowrank_exactly_low_rank_operator():
    """An exactly rank-r operator: the residual is zero, so its construction
    finds no rank anywhere and the result is B B^T."""
    from oracle.lowrank import build_lowrank
    T = Tree(si.points_1d_cell_centres(256), 32, 0.7)
    C = np.random.default_rng(9).standard_normal((256, 8))
    H = C @ C.T
    Hs, info = build_lowrank(lambda V: H @ V, T, 1e-8, 16, 16, 10, seed=3)
    pr = info["residual_peel"]
    assert all(int(pr.kw[l].max()) == 0 for l in range(1, T.L + 1))
    assert info["global_rank"] == 8
    Ht = H[np.ix_(T.perm, T.perm)]
    assert np.linalg.norm(Hs.dense_tree() - Ht, 2) <= 1e-10 * np.linalg.norm(H, 2)
