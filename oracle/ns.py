"""Norm estimates and hierarchical Newton-Schulz inversion (oracle side).

Paper: 2-norms by the power method, stopped once the value has converged to 2
significant digits (Sec. 3.2, matrix norms).  Newton-Schulz X <- (2I - XA)X
(Appendix A, Alg. 1) with each iterate rebuilt by the construction of
Sec. 3.3 from a sampler that evaluates (2I - X_k A) X_k Omega (Alg. 2 and
Alg. 3), at a construction threshold eps_k chosen per iteration (dynamic
threshold, Alg. 2).

Readings taken here:
  * power method: v <- A v / ||A v|| from one seeded Gaussian vector, stop at a
    relative change <= rel (1e-2 = two digits), at least 3 iterations
  * residual E = ||I - A X||_2 by the power method on R^T R (R = I - A X), so
    four HGEMVs per iteration, with X and A symmetric
  * starting iterate X0 = I / nu (nu = ||A||_2 estimate) or X0 = A^T / nu^2
  * iterate threshold: eps_k = eps_build (static) or
    clamp(0.1 E_k^2, eps_build, 1e-2) (dynamic); an iterate is built to absolute
    accuracy eps_k / ||A||_2 -- the scale at which its error enters I - A X
  * stop when E <= eps or after max_iter iterations; divergence when E grows
    above 1 from one iteration to the next

Higher-order forms (Appendix A.2 and A.3):
  * hyperpower iteration of order l: X_{k+1} = X_k (I + R_k + ... + R_k^(l-1)),
    R_k = I - A X_k; its sampler applies the sum Horner-style (Alg. 4):
    Y = R = Omega, then l - 1 times R <- R - A (X_k R), Y <- Y + R, and
    finally Y <- X_k Y.  l = 2 is Newton-Schulz, sampled by Alg. 3.
  * unrolled iterations from a warm start: u Newton-Schulz steps written in
    terms of X_0 give X_u = X_0 sum_{i < 2^u} (I - A X_0)^i (the printed
    binomial form is garbled: its sum is the residual (I - A X_0)^(2^u), and
    its sign is flipped), i.e. one hyperpower step of order 2^u, built in a
    single construction.
  * warm start: X0 is a given H2 matrix (the previous inverse).
"""
import numpy as np

from . import rng
from .h2 import H2Matrix
from .peel import peel, recompress


def power_norm(apply_tree, n, seed, iteration=0, rel=1e-2, min_it=3, max_it=30):
    """2-norm estimate of a symmetric operator by the power method.

    Returns (nu, iterations).
    """
    key = rng.stream_key(seed, rng.PHASE_NORM, 0, 0, iteration)
    v = rng.gaussian(key, np.arange(n), np.arange(1))
    v = v / np.linalg.norm(v)
    prev = None
    nu = 0.0
    it = 0
    for it in range(1, max_it + 1):
        w = apply_tree(v)
        nu = float(np.linalg.norm(w))
        if nu == 0.0:
            return 0.0, it
        v = w / nu
        if prev is not None and it >= min_it and abs(nu - prev) <= rel * nu:
            break
        prev = nu
    return nu, it


def residual_norm(A, X, seed, iteration, rel=1e-2, min_it=3, max_it=30):
    """E = ||I - A X||_2 via the power method on R^T R (four HGEMVs per step)."""
    def RtR(v):
        r = v - A.matvec_tree(X.matvec_tree(v))
        return r - X.matvec_tree(A.matvec_tree(r))
    key = rng.stream_key(seed, rng.PHASE_RESID, 0, 0, iteration)
    v = rng.gaussian(key, np.arange(A.tree.n), np.arange(1))
    v = v / np.linalg.norm(v)
    prev = None
    lam = 0.0
    for it in range(1, max_it + 1):
        w = RtR(v)
        lam = float(np.linalg.norm(w))
        if lam == 0.0:
            return 0.0
        v = w / lam
        E = np.sqrt(lam)
        if prev is not None and it >= min_it and abs(E - prev) <= rel * E:
            break
        prev = E
    return float(np.sqrt(lam))


def build(apply_tree, tree, tol, nu, rank_cap, oversample, adaptive=True,
          max_rounds=16, seed=1, iteration=0, first_cols=None):
    """Peeling followed by recompression: the oracle's buildH(S, eps)."""
    pr = peel(apply_tree, tree, tol, nu, rank_cap, oversample, adaptive,
              max_rounds, seed, iteration, first_cols)
    H = recompress(tree, pr, tol, nu, rank_cap)
    return H, pr


def ns_eval(Xk, A, Om):
    """Samples of the Newton-Schulz iterate (Alg. 3): (2I - X_k A) X_k Omega."""
    W = Xk.matvec_tree(Om)
    return 2.0 * W - Xk.matvec_tree(A.matvec_tree(W))


def hyperpower_eval(Xk, A, Om, order):
    """Samples of the order-l hyperpower iterate (Alg. 4):
    X_k (I + R + ... + R^(l-1)) Omega with R = I - A X_k."""
    Y = Om.copy()
    R = Om.copy()
    for _ in range(order - 1):
        R = R - A.matvec_tree(Xk.matvec_tree(R))
        Y = Y + R
    return Xk.matvec_tree(Y)


def newton_schulz(A, eps, max_iter, rank_cap, oversample, x0="identity",
                  dynamic=False, eps_build=None, adaptive=True, max_rounds=16,
                  seed=1, nu_rel=1e-2, resid_rel=1e-2, order=2, unroll=0):
    """Hierarchical Newton-Schulz for a symmetric positive definite H2 A.

    x0: "identity" (I / nu), "scaled" (A^T / nu^2) or an H2Matrix on A's tree
    (warm start).  order: hyperpower order l >= 2 of every step (2 is
    Newton-Schulz); unroll = u >= 1 builds u unrolled Newton-Schulz steps per
    construction (order 2^u).
    Returns (X, info) with info holding the residual history, per-iteration
    sample counts and the status string.
    """
    if unroll:
        order = 2 ** unroll
    if order < 2:
        raise ValueError(order)
    tree = A.tree
    n = tree.n
    if eps_build is None:
        eps_build = eps / 10.0
    nuA, _ = power_norm(A.matvec_tree, n, seed, 0, rel=nu_rel,
                        max_it=30 if nu_rel >= 1e-2 else 500)
    if isinstance(x0, H2Matrix):
        if x0.tree is not tree:
            raise ValueError("warm start must share A's tree")
        X = x0
    elif x0 == "identity":
        X = H2Matrix.scaled_identity(tree, 1.0 / nuA)
    elif x0 == "scaled":
        X = A.copy_scaled(1.0 / (nuA * nuA))
    else:
        raise ValueError(x0)
    info = {"nu": nuA, "E": [], "applies": [], "status": "max_iter", "eps_k": []}
    k = 0
    while True:
        E = residual_norm(A, X, seed, k, rel=resid_rel,
                          max_it=30 if resid_rel >= 1e-2 else 3000)
        info["E"].append(E)
        if eps > 0 and E <= eps:
            info["status"] = "converged"
            break
        if k >= 1 and E > info["E"][-2] and E > 1.0:
            info["status"] = "diverged"
            break
        if k >= max_iter:
            break
        eps_k = min(max(0.1 * E * E, eps_build), 1e-2) if dynamic else eps_build
        info["eps_k"].append(eps_k)
        Xk = X

        if order == 2:
            def sampler(Om, Xk=Xk):
                return ns_eval(Xk, A, Om)
        else:
            def sampler(Om, Xk=Xk):
                return hyperpower_eval(Xk, A, Om, order)
        X, pr = build(sampler, tree, eps_k, 1.0 / nuA, rank_cap, oversample,
                      adaptive, max_rounds, seed, k + 1)
        info["applies"].append(pr.applies)
        k += 1
    info["iterations"] = k
    return X, info
