"""Global low-rank pre-pass combined with the hierarchical construction
(oracle side).

Paper, Sec. 3.3, the paragraph on combining the construction with global
low-rank approximations: when the data-misfit Hessian has a small global rank,
an initial approximation B B^T is taken by the usual dense randomized sampling;
the hierarchical construction then runs on the residual H - B B^T, and B B^T
is added back to the result as a low-rank update.

Readings taken here (the paper gives no formulas):
  * the range finder is the two-pass randomized one of Halko, Martinsson and
    Tropp: Y = H Omega with r + p Gaussian columns (stream phase GLOBAL, tree
    order), Q from the Householder QR of Y, Z = H Q, T = Q^T Z symmetrised;
    T = V diag(lam) V^T, and the eigenvalues above 1e-13 lam_max (at most r of
    them) give B = Q V_r diag(sqrt(lam_r)), so B B^T = Q T_r Q^T; the
    Hessians are symmetric positive semi-definite.  2 (r + p) products.
  * nu = ||H||_2 by the power method on H (as for a plain build) sets the
    threshold eps nu / (4 L) of both constructions below
  * the construction of the residual uses the sampler H Omega - B (B^T Omega);
    its recompression caps basis ranks at rank_cap + r' (r' the columns of
    B): a global rank-r' term adds up to r' to the rank of every block, so
    the residual's blocks need that much room even where H's do not
  * the low-rank update A_res + B B^T is recompressed by the same construction
    applied to the sampler A_res Omega + B (B^T Omega): products with the H2
    and with B only, no Hessian products
"""
import numpy as np

from . import rng
from .ns import build, power_norm
from .peel import peel, recompress

PHASE_GLOBAL = 7
EIG_CUT = 1e-13


def global_lowrank(apply_tree, n, rank, oversample, seed, iteration=0):
    """B (n x r') with B B^T ~ H from 2 (rank + oversample) products.

    Returns (B, applies)."""
    b = min(rank + oversample, n)
    key = rng.stream_key(seed, PHASE_GLOBAL, 0, 0, iteration)
    Om = rng.gaussian(key, np.arange(n), np.arange(b))
    Y = apply_tree(Om)
    Q, _ = np.linalg.qr(Y, mode="reduced")
    Z = apply_tree(Q)
    T = Q.T @ Z
    T = 0.5 * (T + T.T)
    lam, V = np.linalg.eigh(T)
    lam, V = lam[::-1], V[:, ::-1]
    if lam[0] <= 0:
        return np.zeros((n, 0)), 2 * b
    k = min(rank, int(np.sum(lam > EIG_CUT * lam[0])))
    B = Q @ (V[:, :k] * np.sqrt(lam[:k]))
    return B, 2 * b


def build_lowrank(apply_tree, tree, tol, rank, rank_cap, oversample, adaptive=True,
                  max_rounds=16, seed=1):
    """H2 of H from a global low-rank pre-pass and the construction of the
    residual H - B B^T, with B B^T added back.

    Returns (H2, info) with the products taken by each part."""
    n = tree.n
    nu, it = power_norm(apply_tree, n, seed)
    B, a_global = global_lowrank(apply_tree, n, rank, oversample, seed)

    def residual(Om):
        return apply_tree(Om) - B @ (B.T @ Om)
    pr = peel(residual, tree, tol, nu, rank_cap, oversample, adaptive, max_rounds, seed)
    Hres = recompress(tree, pr, tol, nu, rank_cap + B.shape[1])

    def total(Om):
        return Hres.matvec_tree(Om) + B @ (B.T @ Om)
    H, pr2 = build(total, tree, tol, nu, rank_cap, oversample, adaptive, max_rounds, seed,
                   iteration=1)
    info = {"nu": nu, "norm_applies": it, "global_rank": B.shape[1],
            "global_applies": a_global, "residual_applies": pr.applies,
            "applies": a_global + pr.applies, "residual": Hres, "residual_peel": pr,
            "update_peel": pr2, "B": B}
    return H, info
