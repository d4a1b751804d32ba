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
