"""Randomized peeling and recompression into a strong-admissibility H2 (oracle).

Paper, Sec. 3.3 (construction from Hessian-vector products): levels are
processed coarse to fine; at each level the matrix is sampled with patterned
Gaussian columns that are nonzero on one side of every block being sampled,
the coarser blocks already constructed are removed from the samples, a QR of
the sampled block rows gives the column basis U, and the product V = A^T [0 U]
gives the row basis; sampling repeats until the block meets the threshold.
The sampling partition is the weak (sibling) one while the destination H2
uses strong admissibility, so the sampled low-rank blocks are added to the
destination as local low-rank updates and the matrix is recompressed
(Sec. 3.2: QR downsweep of block rows, SVD truncation upsweep, projection).

Readings taken here (the paper gives no formulas for them):
  * sibling pairs (t1, t2) = (2p, 2p+1) of level l are sampled together;
    Omega is Gaussian on the rows of every t1 and zero elsewhere
  * samples have the peeled coarser levels subtracted using their factors
  * adaptive stopping by the Halko-Martinsson-Tropp estimator: after each
    round r >= 1, e = 10 sqrt(2/pi) max_j ||(I - Q Q^T) y_j|| with Q from the
    earlier rounds; a pair whose e <= tau freezes; at least 2 rounds
  * range basis Q0: Householder QR of the samples, SVD of R, keep the
    singular values above 1e-13 sigma_1; each column gets a canonical sign
    (its largest-magnitude entry positive, first index on ties).  One
    projection matrix carries the bases of every pair of a level, and after
    the coarser levels are removed a residual of size tau still couples
    neighbouring pairs, so without a canonical sign the result would depend
    on the sign convention of the QR/SVD routine used
  * projection Y' = A [0; Q0] (minus peeled levels), B0 = Y'[t1];
    SVD(B0) = W S V^T truncated at tau gives A[t2,t1] ~ (Q0 V) (W S)^T
  * leaf diagonal blocks from stacked identities, symmetrised
  * tau = eps * nu / (4 L), nu the 2-norm estimate of the sampled operator
  * recompression once after all levels, at the same threshold, with the
    destination rank cap
  * the round budget is clamped so that at most 1024 sample columns are kept
    per pair (the first round may be wider than the others: a per-level
    first-round width, e.g. from a learned rank prediction, is an input)
"""
import math

import numpy as np

from . import rng
from .h2 import H2Matrix
from .tree import sibling_level

RANK_CUT = 1e-13


def range_basis(Z):
    """Orthonormal basis of the numerical range of Z (Householder QR + SVD of R)."""
    if Z.shape[1] == 0 or Z.shape[0] == 0:
        return np.zeros((Z.shape[0], 0))
    Q, R = np.linalg.qr(Z, mode="reduced")
    Ur, s, _ = np.linalg.svd(R)
    if s[0] == 0.0:
        return np.zeros((Z.shape[0], 0))
    k = int(np.sum(s > RANK_CUT * s[0]))
    return canonical_signs(Q @ Ur[:, :k])


def canonical_signs(Q):
    """Flip columns so that each column's largest-magnitude entry is positive."""
    if Q.shape[1] == 0:
        return Q
    idx = np.argmax(np.abs(Q), axis=0)
    sgn = np.where(Q[idx, np.arange(Q.shape[1])] < 0, -1.0, 1.0)
    return Q * sgn


class PeelResult:
    def __init__(self):
        self.F = {}          # level -> (N, K_l) side factors (B on t1 rows, Q on t2 rows)
        self.kw = {}         # level -> int array of pair ranks
        self.Ddiag = []      # leaf diagonal blocks
        self.applies = 0
        self.rounds = {}     # level -> rounds taken
        self.k0 = {}         # level -> range-basis sizes
        self.sig = {}        # level -> per pair singular values of B0 (descending)
        self.first_cols = {} # level -> width of the first sampling round
        self.needed = {}     # level -> per pair sample columns held when the estimator accepted
        self.converged = True


def weak_apply(tree, l, F, Om):
    """Product of the level-l weak low-rank blocks with Om (tree order).

    Rows t2 receive Q (B^T Om[t1]); rows t1 receive B (Q^T Om[t2]).
    """
    Y = np.zeros_like(Om)
    for p in range(1 << (l - 1)):
        a1, b1 = tree.rng(l, 2 * p)
        a2, b2 = tree.rng(l, 2 * p + 1)
        Y[a2:b2] += F[a2:b2] @ (F[a1:b1].T @ Om[a1:b1])
        Y[a1:b1] += F[a1:b1] @ (F[a2:b2].T @ Om[a2:b2])
    return Y


def peel(apply_tree, tree, tol, nu, rank_cap, oversample, adaptive=True,
         max_rounds=16, seed=1, iteration=0, first_cols=None):
    """Weak-partition peeling of the operator `apply_tree` (tree-order columns).

    first_cols: optional {level: width} of the first sampling round (the
    other rounds take rank_cap + oversample columns).
    Returns a PeelResult with the factors of every level and the leaf diagonal.
    """
    N, L = tree.n, tree.L
    res = PeelResult()

    def A(Om):
        res.applies += Om.shape[1]
        return apply_tree(Om)

    def subtract(l, Om, Y):
        for lp in range(1, l):
            Y -= weak_apply(tree, lp, res.F[lp], Om)
        return Y

    b = rank_cap + oversample
    tau = tol * nu / (4 * max(L, 1))
    for l in range(1, L + 1):
        npairs = 1 << (l - 1)
        Z = [np.zeros((tree.size(l, 2 * p + 1), 0)) for p in range(npairs)]
        frozen = [False] * npairs
        needed = [-1] * npairs
        b0 = max(b, int(first_cols.get(l, b))) if first_cols else b
        res.first_cols[l] = b0
        rounds_max = max(2, min(max_rounds, 1 + (1024 - b0) // b))
        r = 0
        while True:
            key = rng.stream_key(seed, rng.PHASE_RANGE, l, r, iteration)
            width = b0 if r == 0 else b
            Om = np.zeros((N, width))
            for p in range(npairs):
                a1, b1 = tree.rng(l, 2 * p)
                Om[a1:b1] = rng.gaussian(key, np.arange(a1, b1), np.arange(width))
            Y = subtract(l, Om, A(Om))
            for p in range(npairs):
                if frozen[p]:
                    continue
                a2, b2 = tree.rng(l, 2 * p + 1)
                Yp = Y[a2:b2]
                if adaptive and r >= 1:
                    Q = range_basis(Z[p])
                    resid = Yp - Q @ (Q.T @ Yp)
                    e = 10.0 * math.sqrt(2.0 / math.pi) * float(np.max(np.linalg.norm(resid, axis=0)))
                    if e <= tau:
                        frozen[p] = True
                        needed[p] = Z[p].shape[1]
                    Z[p] = np.hstack([Z[p], Yp])
                else:
                    Z[p] = np.hstack([Z[p], Yp])
            r += 1
            if not adaptive:
                break
            if r >= 2 and all(frozen):
                break
            if r >= rounds_max:
                res.converged = False
                break
        res.rounds[l] = r
        res.needed[l] = np.array([needed[p] if needed[p] >= 0 else Z[p].shape[1]
                                  for p in range(npairs)], dtype=np.int64)
        Q0 = [range_basis(Z[p]) for p in range(npairs)]
        k0 = np.array([q.shape[1] for q in Q0], dtype=np.int64)
        res.k0[l] = k0
        K0 = int(k0.max())
        kw = np.zeros(npairs, dtype=np.int64)
        res.sig[l] = [np.zeros(0) for _ in range(npairs)]
        Qs, Bs = [None] * npairs, [None] * npairs
        if K0 > 0:
            Om2 = np.zeros((N, K0))
            for p in range(npairs):
                a2, b2 = tree.rng(l, 2 * p + 1)
                Om2[a2:b2, :k0[p]] = Q0[p]
            Y2 = subtract(l, Om2, A(Om2))
            for p in range(npairs):
                a1, b1 = tree.rng(l, 2 * p)
                B0 = Y2[a1:b1, :k0[p]]
                if k0[p] == 0:
                    Qs[p] = Q0[p]
                    Bs[p] = np.zeros((b1 - a1, 0))
                    continue
                W, s, Vt = np.linalg.svd(B0, full_matrices=False)
                res.sig[l][p] = s
                k = int(np.sum(s > tau))
                kw[p] = k
                Qs[p] = Q0[p] @ Vt[:k].T
                Bs[p] = W[:, :k] * s[:k]
        Kl = int(kw.max()) if npairs else 0
        F = np.zeros((N, Kl))
        for p in range(npairs):
            if kw[p] == 0:
                continue
            a1, b1 = tree.rng(l, 2 * p)
            a2, b2 = tree.rng(l, 2 * p + 1)
            F[a1:b1, :kw[p]] = Bs[p]
            F[a2:b2, :kw[p]] = Qs[p]
        res.F[l] = F
        res.kw[l] = kw
    # leaf diagonal blocks from stacked identities
    mmax = max(tree.size(L, i) for i in range(1 << L))
    OmD = np.zeros((N, mmax))
    for i in range(1 << L):
        a, b_ = tree.rng(L, i)
        OmD[a:b_, :b_ - a] = np.eye(b_ - a)
    YD = subtract(L + 1, OmD, A(OmD))
    for i in range(1 << L):
        a, b_ = tree.rng(L, i)
        M = YD[a:b_, :b_ - a]
        res.Ddiag.append(0.5 * (M + M.T))
    return res


def recompress(tree, pr, tol, nu, rank_cap):
    """Fold the weak factors into a strong-admissibility H2 (nested bases)."""
    L = tree.L
    H = H2Matrix(tree)
    if L == 0:
        H.D[(0, 0)] = pr.Ddiag[0]
        return H
    tau_c = tol * nu / (4 * L)
    F, kw = pr.F, pr.kw

    def Frows(l, lev, i):
        anc = i >> (lev - l)
        k = int(kw[l][anc >> 1])
        a, b = tree.rng(lev, i)
        return F[l][a:b, :k]

    def ksib(l, lev, i):
        return int(kw[l][(i >> (lev - l)) >> 1])

    partners = [dict() for _ in range(L + 1)]
    for lev in range(1, L + 1):
        for (t, s) in tree.far[lev]:
            partners[lev].setdefault(t, []).append(s)

    # (R1) downsweep: R^l_t with R^T R = sum of F^l_s^T F^l_s over the far
    # block row of t and of its ancestors, grouped by sibling level l
    R = {}
    for lev in range(1, L + 1):
        for i in range(1 << lev):
            by_level = {}
            for j in partners[lev].get(i, []):
                by_level.setdefault(sibling_level(lev, i, j), []).append(j)
            for l in range(1, lev + 1):
                if ksib(l, lev, i) == 0:
                    continue
                blocks = []
                if l <= lev - 1 and (lev - 1, i >> 1, l) in R:
                    blocks.append(R[(lev - 1, i >> 1, l)])
                for j in by_level.get(l, []):
                    blocks.append(Frows(l, lev, j))
                if blocks:
                    R[(lev, i, l)] = np.linalg.qr(np.vstack(blocks), mode="r")

    # (R2) upsweep: truncated SVD of the weighted block row gives bases
    P = {}

    def truncate(G):
        if G.shape[0] == 0 or G.shape[1] == 0:
            return np.zeros((G.shape[0], 0))
        Uf, s, _ = np.linalg.svd(G, full_matrices=False)
        k = min(rank_cap, int(np.sum(s > tau_c)))
        return Uf[:, :k]

    for i in range(1 << L):
        cols = [Frows(l, L, i) @ R[(L, i, l)].T for l in range(1, L + 1) if (L, i, l) in R]
        G = np.hstack(cols) if cols else np.zeros((tree.size(L, i), 0))
        U = truncate(G)
        H.U[i] = U
        H.rank[L][i] = U.shape[1]
        for l in range(1, L + 1):
            P[(L, i, l)] = U.T @ Frows(l, L, i)
    for lev in range(L - 1, 0, -1):
        for i in range(1 << lev):
            c1, c2 = 2 * i, 2 * i + 1
            k1, k2 = int(H.rank[lev + 1][c1]), int(H.rank[lev + 1][c2])
            cols = [np.vstack([P[(lev + 1, c1, l)], P[(lev + 1, c2, l)]]) @ R[(lev, i, l)].T
                    for l in range(1, lev + 1) if (lev, i, l) in R]
            G = np.hstack(cols) if cols else np.zeros((k1 + k2, 0))
            Ut = truncate(G)
            k = Ut.shape[1]
            H.rank[lev][i] = k
            H.E[lev + 1][c1] = Ut[:k1]
            H.E[lev + 1][c2] = Ut[k1:]
            for l in range(1, lev + 1):
                P[(lev, i, l)] = Ut[:k1].T @ P[(lev + 1, c1, l)] + Ut[k1:].T @ P[(lev + 1, c2, l)]
    for c in (0, 1):
        H.E[1][c] = np.zeros((int(H.rank[1][c]), 0))

    # (R3) couplings, (R4) dense near field
    for lev in range(1, L + 1):
        for (t, s) in tree.far[lev]:
            l = sibling_level(lev, t, s)
            H.S[lev][(t, s)] = P[(lev, t, l)] @ P[(lev, s, l)].T
    for (t, s) in tree.near:
        if t == s:
            H.D[(t, s)] = pr.Ddiag[t]
        else:
            l = sibling_level(L, t, s)
            H.D[(t, s)] = Frows(l, L, t) @ Frows(l, L, s).T
    return H


def weak_dense(tree, pr):
    """Dense (tree order) matrix represented by the peeled weak factors + diagonal."""
    N, L = tree.n, tree.L
    A = np.zeros((N, N))
    for l in range(1, L + 1):
        A += weak_apply(tree, l, pr.F[l], np.eye(N))
    for i in range(1 << L):
        a, b = tree.rng(L, i)
        A[a:b, a:b] += pr.Ddiag[i]
    return A
