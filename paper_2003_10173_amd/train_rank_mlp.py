"""Train the first-round rank predictor and write data/rank_mlp.npz.

Usage (on a GPU):  python -m paper_2003_10173_amd.train_rank_mlp [--runs N] [--epochs E]
Problems come from seeded_inputs.learned_training_problem (1D and 2D kernel
families, eps in 1e-3..1e-6); every run is a plain adaptive build whose
per-pair features and ranks are recorded, then the network is trained with
the library's GPU kernels.
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    import numpy as np
    import seeded_inputs as si
    from paper_2003_10173_amd import learned as LN
    t0 = time.perf_counter()
    probs = [si.learned_training_problem(i) for i in range(a.runs)]
    F, T = LN.generate_records(
        probs, progress=lambda i: (i % 25 == 0) and print("run %d, %.0f s" % (
            i, time.perf_counter() - t0), flush=True))
    print("records %d, %.0f s" % (len(T), time.perf_counter() - t0), flush=True)
    net, hist = LN.train(F, T, epochs=a.epochs,
                         progress=lambda e, l: (e % 10 == 0) and print(
                             "epoch %d loss %.4f" % (e, l), flush=True))
    LN.save(net, a.out or LN.WEIGHTS,
            meta=dict(runs=np.int64(a.runs), records=np.int64(len(T)),
                      loss=np.array(hist, dtype=np.float64)))
    print("saved; final loss %.4f, %.0f s" % (hist[-1], time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    main()
