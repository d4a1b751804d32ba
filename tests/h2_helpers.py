"""Shared test helpers: oracle <-> packed-layout conversion and GPU guards."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # noqa: BLE001
        return False


def oracle_to_packed(H):
    """Pack an oracle H2Matrix into the (ranks, U, E, S, D) layout of include/h2.h."""
    T = H.tree
    L = T.L
    ranks = np.concatenate([H.rank[l] for l in range(L + 1)]).astype(np.int32)
    U = np.concatenate([H.U[i].ravel() for i in range(1 << L)] + [np.zeros(0)])
    E = [np.zeros(0)]
    for l in range(1, L + 1):
        for i in range(1 << l):
            E.append(np.asarray(H.E[l][i]).reshape(H.rank[l][i], H.rank[l - 1][i // 2]).ravel())
    E = np.concatenate(E)
    S = [np.zeros(0)]
    for l in range(1, L + 1):
        for (t, s) in T.far[l]:
            S.append(np.asarray(H.S[l][(t, s)]).reshape(H.rank[l][t], H.rank[l][s]).ravel())
    S = np.concatenate(S)
    D = np.concatenate([H.D[(t, s)].ravel() for (t, s) in T.near])
    return ranks, U, E, S, D


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def packed_to_oracle(T, ranks, U, E, S, D):
    """Unpack the (ranks, U, E, S, D) layout of include/h2.h into an oracle
    H2Matrix on the oracle tree T (the inverse of oracle_to_packed)."""
    from oracle.h2 import H2Matrix
    L = T.L
    H = H2Matrix(T)
    ranks = np.asarray(ranks, dtype=np.int64)
    H.rank = [ranks[(1 << l) - 1:(2 << l) - 1].copy() for l in range(L + 1)]
    o = 0
    for i in range(1 << L):
        a, b = T.rng(L, i)
        k = int(H.rank[L][i])
        H.U[i] = np.asarray(U[o:o + (b - a) * k]).reshape(b - a, k)
        o += (b - a) * k
    o = 0
    for l in range(1, L + 1):
        for i in range(1 << l):
            kc, kp = int(H.rank[l][i]), int(H.rank[l - 1][i // 2])
            H.E[l][i] = np.asarray(E[o:o + kc * kp]).reshape(kc, kp)
            o += kc * kp
    o = 0
    for l in range(1, L + 1):
        for (t, s) in T.far[l]:
            kt, ks = int(H.rank[l][t]), int(H.rank[l][s])
            H.S[l][(t, s)] = np.asarray(S[o:o + kt * ks]).reshape(kt, ks)
            o += kt * ks
    o = 0
    for (t, s) in T.near:
        a, b = T.rng(L, t)
        c, d = T.rng(L, s)
        H.D[(t, s)] = np.asarray(D[o:o + (b - a) * (d - c)]).reshape(b - a, d - c)
        o += (b - a) * (d - c)
    return H
