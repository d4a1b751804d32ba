"""Write the stored expected values of the full-size parity tests.

Calls only the oracle (and the seeded input generators).  The oracle's runs at
these sizes take minutes to an hour of CPU time, too long for a test, so the
GPU tests compare against what this script stored:

  diffusion64_build_ns.json   diffusion Gauss-Newton Hessian on the 64 x 64
                              grid (N = 4096): build at 1e-4 (adaptive) and
                              Newton-Schulz from I / nu to 1e-4 (dynamic
                              threshold), plus sampled entries of both
                              operators applied to seeded probes
  batch8_build.json           8 of the 256 uneven 2D kernel Hessians (the
                              smallest, the largest and 6 drawn by a seeded
                              generator): builds at 1e-4 and sampled products

Sampled entries: probes are seeded N(0,1) vectors (user order); rows are drawn
by a seeded generator; each stored value is (A p)[row] for the oracle's H2.

Rounding spread: the construction amplifies rounding (its truncations cut
through dense singular spectra), so each record also stores the largest
difference between the oracle's sampled values and those of a second oracle
run whose samples carry a seeded relative perturbation of 1e-14 (the
rounding level of FP64 sums over a few thousand terms, as in the samplers'
time stepping and the subtraction of peeled levels): the spread two correct
FP64 implementations may show.  For the Newton-Schulz record the second run
inverts the perturbed build with perturbed samples in every iterate, and its
history of E_k and products per iteration is stored beside the first run's.

Usage: python tests/golden/make_golden.py [diffusion64] [batch8]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import seeded_inputs as si  # noqa: E402
from oracle.hessians import DiffusionGN, KernelHessian, tree_order  # noqa: E402
from oracle.ns import build as obuild, newton_schulz as ons, power_norm  # noqa: E402
from oracle.tree import Tree  # noqa: E402

PROBE_SEED = 77
ROW_SEED = 78
NPROBE = 4
NROWS = 128


def sample_rows(n, seed=ROW_SEED, count=NROWS):
    g = np.random.Generator(np.random.PCG64(seed))
    return np.sort(g.choice(n, size=min(count, n), replace=False))


def sampled_products(M, n):
    P = si.gaussian_vectors(n, NPROBE, PROBE_SEED)
    rows = sample_rows(n)
    Y = M.matvec(P)
    return {"probe_seed": PROBE_SEED, "rows": rows.tolist(),
            "values": Y[rows].T.tolist(),           # NPROBE x NROWS
            "max_abs": [float(np.max(np.abs(Y[:, j]))) for j in range(NPROBE)]}


PERTURB = 1e-14


def perturbed(apply_tree, seed=12345):
    """apply_tree with its output multiplied by 1 + PERTURB N(0,1) entrywise."""
    g = np.random.Generator(np.random.PCG64(seed))

    def f(Om):
        Y = apply_tree(Om)
        return Y * (1.0 + PERTURB * g.standard_normal(Y.shape))
    return f


def spread(M, M2, n):
    """Largest |difference| of the sampled products of two runs, per probe."""
    a = sampled_products(M, n)
    b = sampled_products(M2, n)
    return [float(np.max(np.abs(np.asarray(x) - np.asarray(y))))
            for x, y in zip(a["values"], b["values"])]


def build_record(T, H, pr, nu):
    L = T.L
    return {"n": T.n, "levels": L, "nu": nu, "applies": int(pr.applies),
            "rounds": [int(pr.rounds[l]) for l in range(1, L + 1)],
            "range_cols": [int(pr.k0[l].max()) for l in range(1, L + 1)],
            "weak_rank": [int(pr.kw[l].max()) for l in range(1, L + 1)],
            "ranks": np.concatenate([H.rank[l] for l in range(L + 1)]).astype(int).tolist()}


def diffusion64():
    cfg = si.config_diffusion2d(64)
    T = Tree(cfg["points"], cfg["leaf"], cfg["eta"])
    G = DiffusionGN(cfg)
    A = tree_order(G.apply, T.perm)
    t0 = time.time()
    nu, _ = power_norm(A, T.n, cfg["seed"])
    H, pr = obuild(A, T, cfg["tol"], nu, cfg["cap"], cfg["p"], adaptive=True, max_rounds=16,
                   seed=cfg["seed"])
    print("diffusion64 build %.1f s, %d applies" % (time.time() - t0, pr.applies), flush=True)
    Hp, _ = obuild(perturbed(A), T, cfg["tol"], nu, cfg["cap"], cfg["p"], adaptive=True,
                   max_rounds=16, seed=cfg["seed"])
    t0 = time.time()
    X, info = ons(H, 1e-4, 60, T.leaf_size, cfg["p"], x0="identity", dynamic=True,
                  adaptive=True, max_rounds=16, seed=cfg["seed"])
    print("diffusion64 Newton-Schulz %.1f s, %d iterations" % (time.time() - t0,
                                                              info["iterations"]), flush=True)
    # the whole pipeline perturbed: Newton-Schulz of the perturbed build Hp
    # with every iterate's samples perturbed too (the spread of the inverse
    # includes what the build's spread does to it)
    import oracle.ns as ns_mod
    plain_build = ns_mod.build
    ns_mod.build = lambda f, *a, **k: plain_build(perturbed(f), *a, **k)
    try:
        Xp, infop = ons(Hp, 1e-4, 60, T.leaf_size, cfg["p"], x0="identity", dynamic=True,
                        adaptive=True, max_rounds=16, seed=cfg["seed"])
    finally:
        ns_mod.build = plain_build
    out = {"_about": "oracle build + Newton-Schulz of the 64 x 64 diffusion Gauss-Newton "
                     "Hessian; written by tests/golden/make_golden.py",
           "build": build_record(T, H, pr, nu),
           "build_products": dict(sampled_products(H, T.n), spread=spread(H, Hp, T.n)),
           "ns": {"eps": 1e-4, "max_iter": 60, "rank_cap": T.leaf_size, "oversample": cfg["p"],
                  "x0": "identity", "dynamic": True, "seed": cfg["seed"], "nu": info["nu"],
                  "iterations": info["iterations"], "E": info["E"],
                  "applies": [int(a) for a in info["applies"]], "status": info["status"],
                  "eps_k": [float(e) for e in info["eps_k"]],
                  "E_perturbed": infop["E"],
                  "applies_perturbed": [int(a) for a in infop["applies"]]},
           "ns_products": dict(sampled_products(X, T.n), spread=spread(X, Xp, T.n))}
    with open(os.path.join(HERE, "diffusion64_build_ns.json"), "w") as f:
        json.dump(out, f)


def batch8_indices(count=256, seed=4242):
    ns = np.array([si.batch_problem(b)["n"] for b in range(count)])
    lo, hi = int(np.argmin(ns)), int(np.argmax(ns))
    rest = [b for b in range(count) if b not in (lo, hi)]
    g = np.random.Generator(np.random.PCG64(seed))
    pick = sorted(int(b) for b in g.choice(rest, size=6, replace=False))
    return [lo, hi] + pick


def batch8():
    out = {"_about": "oracle builds of 8 of the 256 uneven 2D kernel Hessians (smallest, "
                     "largest, 6 seeded picks); written by tests/golden/make_golden.py",
           "problems": []}
    for b in batch8_indices():
        p = si.batch_problem(b)
        T = Tree(p["points"], p["leaf"], p["eta"])
        K = KernelHessian(p["points"], p["ell"], p["shift"])
        Hd = K.dense()                   # explicit matvecs by the assembled kernel matrix
        A = tree_order(lambda V: Hd @ V, T.perm)
        t0 = time.time()
        nu, _ = power_norm(A, T.n, p["seed"])
        H, pr = obuild(A, T, p["tol"], nu, p["cap"], p["p"], adaptive=True, max_rounds=16,
                       seed=p["seed"])
        print("batch problem %d (N=%d) build %.1f s, %d applies" % (
            b, T.n, time.time() - t0, pr.applies), flush=True)
        Hp, _ = obuild(perturbed(A), T, p["tol"], nu, p["cap"], p["p"], adaptive=True,
                       max_rounds=16, seed=p["seed"])
        rec = build_record(T, H, pr, nu)
        rec["index"] = b
        rec["products"] = dict(sampled_products(H, T.n), spread=spread(H, Hp, T.n))
        out["problems"].append(rec)
        del Hd
        with open(os.path.join(HERE, "batch8_build.json"), "w") as f:
            json.dump(out, f)


if __name__ == "__main__":
    which = sys.argv[1:] or ["diffusion64", "batch8"]
    if "diffusion64" in which:
        diffusion64()
    if "batch8" in which:
        batch8()
