"""Training and use of the first-round rank predictor (h2_mlp).

Records come from the library's own adaptive builds (h2_records_*): for every
sibling pair of every level, the 16 features and log(1 + columns the estimator
accepted).  Training
runs on the GPU through h2_mlp_train_step (BF16-weight products, FP32 Adam).
"""
import os
import time

import numpy as np

from . import MLP, KernelSampler, Tree, build, opts, records_enable, records_read

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "rank_mlp.npz")


def generate_records(problems, progress=None):
    """Run one plain adaptive build per problem dict (points, ell, shift,
    leaf, eta, cap, p, tol, seed) and return the recorded (features, targets)."""
    records_enable(True)
    try:
        for i, cfg in enumerate(problems):
            tree = Tree(cfg["points"], cfg["leaf"], cfg["eta"])
            S = KernelSampler(cfg["points"], cfg["ell"], cfg["shift"])
            build(tree, S, opts(rank_cap=cfg["cap"], oversample=cfg["p"], tol=cfg["tol"],
                                adaptive=1, max_rounds=16, seed=cfg["seed"]))
            if progress:
                progress(i)
        return records_read()
    finally:
        records_enable(False)


def train(F, T, epochs=40, batch=256, lr=2e-3, seed=7, progress=None):
    """Train a fresh network on (F, T); returns (MLP, per-epoch mean loss)."""
    import torch
    net = MLP(MLP.he_init(seed))
    Fd = torch.tensor(F, dtype=torch.float32, device="cuda")
    Td = torch.tensor(T, dtype=torch.float32, device="cuda")
    g = np.random.Generator(np.random.PCG64(seed))
    hist = []
    n = len(T)
    for ep in range(epochs):
        order = torch.tensor(g.permutation(n), device="cuda")
        for s in range(0, n - batch + 1, batch):
            idx = order[s:s + batch]
            net.train_step(Fd[idx], Td[idx], lr)
        y = net.forward(Fd)
        hist.append(float(torch.mean((y - Td) ** 2)))
        if progress:
            progress(ep, hist[-1])
    return net, hist


def save(net, path=WEIGHTS, meta=None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=net.params(), **(meta or {}))


def load(path=WEIGHTS):
    """The trained network, or None when no weights file exists."""
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return MLP(z["params"])
