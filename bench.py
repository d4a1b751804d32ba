"""Benchmark: H2 Hessian build + Newton-Schulz inverse at 1e-4, and HGEMV GB/s.

One step = the whole hot path on one batch of synthetic input: randomized
peeling of the Hessian from Hessian-vector products (norm estimate, sampling
rounds, range bases, projections, leaf diagonal), recompression into the
strong H2, then hierarchical Newton-Schulz from X0 = I/||A|| until
||I - A X||_2 <= 1e-4 (every iterate rebuilt by peeling from HGEMV samples).

Default workload: the 2D time-dependent diffusion Gauss-Newton Hessian on a
64 x 64 interior grid (N = 4096, leaf 64, rank cap 24, adaptive sampling,
eps = 1e-4), plain FP64 GPU path.  Prints ONE JSON line (rank 0).
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6         # MI355X FP64 vector / dense FP64 MFMA
FP32_PEAK_TFLOPS = 157.3        # MI355X FP32 MFMA (dense)
BF16_PEAK_TFLOPS = 2500.0       # MI355X BF16 MFMA (dense)
DOMINANT = "k_svd_block"        # largest share of the step's kernel time (rocprofv3)
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_svd_block_diffusion64_pmc.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2003_10173_amd", "csrc", "linalg.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hgemv-nv", type=int, default=34)
    ap.add_argument("--hgemv-reps", type=int, default=50)
    ap.add_argument("--appendix-grid", type=int, default=64,
                    help="grid side of the minimal-surface inversion form (the paper's is 128)")
    ap.add_argument("--forms-only", action="store_true",
                    help="measure only the named forms (comma list in --only) and print them")
    ap.add_argument("--only", default="appendix_a,global_lowrank")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision form and the 256x256 precision ladder")
    return ap.parse_args()


def hip_events_time(fn, reps, stream):
    """Average duration (ms) of fn() over reps launches, HIP events on `stream`."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def source_digest(path, kernel=DOMINANT):
    """Digest of the kernel's own source text (from its signature to the
    closing brace at column 0), so unrelated edits elsewhere in the file keep
    the recorded counters valid."""
    import hashlib
    with open(path) as f:
        text = f.read()
    start = text.find("void " + kernel + "(")
    if start < 0:
        return None
    end = text.find("\n}\n", start)
    return hashlib.sha256(text[start:end + 3].encode()).hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE runs, each scaled by the same
    counter's reading for a plain copy of known size), or None when the summary
    is missing or the kernel source changed since the counters were taken."""
    try:
        with open(PMC_SUMMARY) as f:
            line = next(l for l in f if l.startswith("traffic: "))
        t = json.loads(line[len("traffic: "):])
    except (OSError, StopIteration, ValueError):
        return None
    if t.get("kernel") != DOMINANT or t.get("source_digest") != source_digest(KERNEL_SOURCE):
        return None
    kib = t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]
    return int(kib * 1024)


def precision_ladder(h2, torch, si, stream, reps=20):
    """HGEMV of the 2D kernel Hessian on a 256 x 256 grid (N = 65536, leaf 64,
    rank cap 32, built by peeling at 1e-4) on 64 vectors in FP64, FP32 and
    BF16 storage (FP32 accumulation); errors against the FP64 product."""
    cfg = si.config_kernel2d(256)
    tree = h2.Tree(cfg["points"], cfg["leaf"], cfg["eta"])
    S = h2.KernelSampler(cfg["points"], cfg["ell"], cfg["shift"])
    o = h2.opts(rank_cap=cfg["cap"], oversample=cfg["p"], tol=cfg["tol"], adaptive=1,
                max_rounds=16, seed=cfg["seed"])
    t0 = time.perf_counter()
    A, st = h2.build(tree, S, o)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    n, nv = tree.n, cfg["nv"]
    x = torch.tensor(si.gaussian_vectors(n, nv, cfg["vec_seed"]).T.copy(), device="cuda")
    y64 = A.gemv(x)
    out = {"workload": "kernel2d 256x256 (N=65536), leaf 64, cap 32, eps 1e-4, nv=64",
           "build_s": round(t_build, 3), "applies": st["applies"]}
    # vector element bytes: x read once, y written once (w_x + w_y per entry)
    forms = [("fp64", A, x, y64, 8)]
    xf = x.float()
    for prec, name in ((h2.H2_FP32, "fp32"), (h2.H2_BF16, "bf16")):
        B = A.convert(prec)
        forms.append((name, B, xf, B.gemv(xf), 4))
    # cache flush between cold calls: a plain copy of 2 x 512 MiB, larger than
    # the 256 MB Infinity Cache and every L2
    fsrc = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
    fdst = torch.empty_like(fsrc)
    for name, M, xv, yv, vb in forms:
        words, mbytes = M.words()
        M.gemv(xv, yv)
        ms = hip_events_time(lambda: M.gemv(xv, yv), reps, stream)
        cold = []
        for _ in range(5):
            h2.stream_copy(fsrc, fdst)
            cold.append(hip_events_time(lambda: M.gemv(xv, yv), 1, stream))
        ms_cold = sorted(cold)[len(cold) // 2]
        alg = mbytes + 2 * vb * n * nv
        flops = 2.0 * nv * words
        gbs = alg / (ms * 1e-3) / 1e9
        gbs_cold = alg / (ms_cold * 1e-3) / 1e9
        err = float(torch.linalg.norm(yv.double() - y64) / torch.linalg.norm(y64))
        peak_fl = {"fp64": FP64_PEAK_TFLOPS, "fp32": FP32_PEAK_TFLOPS, "bf16": BF16_PEAK_TFLOPS}[name]
        out[name] = {"ms": round(ms, 4), "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "ms_cold": round(ms_cold, 4), "GB/s_cold": round(gbs_cold, 1),
                     "frac_cold": round(gbs_cold / HBM_PEAK_GBS, 4),
                     "TFLOP/s": round(flops / (ms * 1e-3) / 1e12, 3),
                     "mfma_frac": round(flops / (ms * 1e-3) / 1e12 / peak_fl, 4),
                     "alg_bytes": int(alg), "flops": flops, "rel_err_vs_fp64": err}
        print("precision %s: %.3f ms (cold %.3f), %.0f GB/s, %.2f TFLOP/s, err %.2e"
              % (name, ms, ms_cold, gbs, out[name]["TFLOP/s"], err), file=sys.stderr, flush=True)
    del fsrc, fdst
    return out


def learned_form(h2, torch, si):
    """Build of the advection-diffusion Gauss-Newton Hessian on a 128 x 128 grid
    (N = 16384, cap 32, eps 1e-4) with plain adaptive sampling and with the
    trained first-round predictor: wall time, Hessian applies, sampling rounds,
    and each build's relative error on 8 Gaussian probes against the Hessian
    itself (valid: the estimator converged and the error is at most 10 eps)."""
    from paper_2003_10173_amd import learned as LN
    net = LN.load()
    if net is None:
        return None
    cfg = si.config_advdiff2d(128)
    S = h2.AdvDiffSampler(cfg)
    tree = h2.Tree(cfg["points"], cfg["leaf"], cfg["eta"])
    out = {"workload": "advdiff2d 128x128 (N=16384), leaf 64, cap 32, eps 1e-4, build only"}
    for name, extra in (("plain", {}), ("learned", {"learned": net})):
        o = h2.opts(rank_cap=cfg["cap"], oversample=cfg["p"], tol=1e-4, adaptive=1,
                    max_rounds=16, seed=6, **extra)
        h2.build(tree, S, o)                      # warm-up (allocations)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ab, st = h2.build(tree, S, o)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        x = torch.tensor(si.gaussian_vectors(tree.n, 8, 77).T.copy(), device="cuda")
        y_ref = S(x)
        err = float(torch.linalg.norm(Ab.gemv(x) - y_ref) / torch.linalg.norm(y_ref))
        out[name] = {"s": round(t_b, 4), "applies": st["applies"],
                     "rounds": sum(st["rounds"]), "first_cols": st["first_cols"],
                     "probe_rel_err": err, "valid": bool(st["converged"]) and err <= 1e-3}
        print("learned form %s: %.3f s, %d applies, %d rounds, probe error %.1e" % (
            name, out[name]["s"], st["applies"], out[name]["rounds"], err), file=sys.stderr,
            flush=True)
    return out


def c3_inverse_form(h2, torch, si):
    """Build and 20 Newton-Schulz iterations (from I / nu, dynamic threshold)
    of the 2D kernel Hessian on a 256 x 256 grid (N = 65536, leaf 64, cap 32,
    build at 1e-4), with FP32 samplers while the residual is large (FP64
    residuals and refinement) and all in FP64.  With rank cap 32 the iterates
    cannot represent the inverse to 1e-4 (at 128 x 128 the residual levels
    off near 2e-2), so the form runs the fixed count of the 1D configuration
    and reports the residual it reaches.  Not part of the default run
    (about a minute per form): `--forms-only --only c3_inverse`."""
    cfg = si.config_kernel2d(256)
    tree = h2.Tree(cfg["points"], cfg["leaf"], cfg["eta"])
    S = h2.KernelSampler(cfg["points"], cfg["ell"], cfg["shift"])
    o = h2.opts(rank_cap=cfg["cap"], oversample=cfg["p"], tol=cfg["tol"], adaptive=1,
                max_rounds=16, seed=cfg["seed"])
    out = {"workload": "kernel2d 256x256 (N=65536), leaf 64, cap 32, build at 1e-4 + 20 Newton-Schulz "
                       "iterations (dynamic threshold, X0 = I/nu)"}
    for name, prec in (("fp32_samplers", h2.H2_FP32), ("fp64", h2.H2_FP64)):
        nopts = h2.ns_opts(eps=1e-4, max_iter=20, x0=0, dynamic=1, rank_cap=cfg["cap"],
                           oversample=cfg["p"], adaptive=1, max_rounds=16, seed=cfg["seed"],
                           prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A, bst = h2.build(tree, S, o)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        X, nst = h2.newton_schulz(A, nopts)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t0
        # a fixed count: valid when the 20 iterations ran without divergence
        ok = bool(bst["converged"]) and nst["status"] in (0, 1) and nst["iterations"] == 20
        out[name] = {"s": round(t_all, 3), "build_s": round(t_build, 3),
                     "iterations": nst["iterations"], "low_iterations": nst.get("low_iterations"),
                     "residual": nst["resid"][-1], "valid": ok}
        print("c3 inverse %s: %.1f s (build %.1f s), %d iterations, residual %.2e" % (
            name, t_all, t_build, nst["iterations"], nst["resid"][-1]), file=sys.stderr, flush=True)
        del A, X
    return out


def batched_form(h2, torch, si, count=256):
    """Construction of `count` uneven 2D kernel Hessians (N log-uniform in
    [1024, 16384] on random-aspect grids, ell ~ U[0.02, 0.2], cap 32, eps 1e-4)
    in one level-synchronous batch against one build after the other."""
    ps = si.config_batch(count)
    trees = [h2.Tree(p["points"], p["leaf"], p["eta"]) for p in ps]
    samp = [h2.KernelSampler(p["points"], p["ell"], p["shift"]) for p in ps]
    opts = [h2.opts(rank_cap=p["cap"], oversample=p["p"], tol=p["tol"], adaptive=1, max_rounds=16,
                    seed=p["seed"]) for p in ps]
    h2.build(trees[0], samp[0], opts[0])       # warm-up (allocations, tile tuning)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h2.build_batched(trees, samp, opts)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    for i in range(count):
        h2.build(trees[i], samp[i], opts[i])
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    print("batched form: %d problems, batched %.2f s, sequential %.2f s" % (count, tb, ts),
          file=sys.stderr, flush=True)
    return {"workload": "%d uneven kernel2d Hessians (N %d..%d, total %d), cap 32, eps 1e-4, build"
                        % (count, min(p["n"] for p in ps), max(p["n"] for p in ps),
                           sum(p["n"] for p in ps)),
            "batched_s": round(tb, 3), "sequential_s": round(ts, 3), "speedup": round(ts / tb, 3)}


def host_cpu():
    """Host cores usable by this process and the CPU model name."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return cores, model


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [i["num_threads"] for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return max(n)
    except Exception:  # noqa: BLE001
        pass
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


# the paper's inversion times for its minimal-surface example (n = 16,384,
# one P100; Appendix A): context for the appendix form, not a target
PAPER_APPENDIX_A_S = {"static": 178.0, "dynamic": 51.0, "hyperpower8": 20.0,
                      "hyperpower16": 20.0, "warm_static": 32.0, "warm_dynamic": 14.0,
                      "warm_unrolled": 4.0}


def appendix_a_form(h2, torch, si, grid):
    """Newton-Schulz inversion of the minimal-surface Hessian (Appendix A
    example) on a grid x grid mesh, leaf 64, construction threshold 1e-6,
    stop at ||I - A X||_2 <= 1e-4.  First optimisation step from X0 = I/nu:
    static threshold, dynamic threshold (from 1e-2), hyperpower orders 8 and
    16 (dynamic).  Second step (the next surface): from I/nu, warm-started
    from the first step's inverse, and warm-started with the warm run's
    Newton-Schulz steps unrolled into one construction."""
    out = {"workload": "minsurf2d %dx%d (N=%d), leaf 64, eps_k 1e-6, stop 1e-4, X0 = I/nu"
                       % (grid, grid, grid * grid),
           "paper_p100_s_at_128x128": PAPER_APPENDIX_A_S}
    cfgs = [si.config_minsurf2d(grid, 0), si.config_minsurf2d(grid, 1)]
    tree = h2.Tree(cfgs[0]["points"], cfgs[0]["leaf"], cfgs[0]["eta"])
    mats = []
    for c in cfgs:
        A, st = h2.build(tree, h2.MinSurfSampler(c),
                         h2.opts(rank_cap=c["cap"], oversample=c["p"], tol=c["tol"], adaptive=1,
                                 max_rounds=16, seed=c["seed"]))
        mats.append(A)
    c = cfgs[0]

    def run(name, A, **kw):
        o = h2.ns_opts(eps=c["eps"], max_iter=60, eps_build=c["eps_build"], rank_cap=0,
                       oversample=c["p"], adaptive=1, max_rounds=16, seed=c["seed"], **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info = h2.newton_schulz(A, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"s": round(dt, 3), "iterations": info["iterations"],
                     "applies": int(sum(info["applies"])), "residual": info["resid"][-1],
                     "ok": info["status"] == 0}
        print("appendix A %s: %.2f s, %d iterations, %d samples, E %.2e" % (
            name, dt, info["iterations"], out[name]["applies"], info["resid"][-1]),
            file=sys.stderr, flush=True)
        return X, info
    run("static", mats[0], x0=0, dynamic=0)
    Xprev, info = run("dynamic", mats[0], x0=0, dynamic=1)
    run("hyperpower8", mats[0], x0=0, dynamic=1, order=8)
    run("hyperpower16", mats[0], x0=0, dynamic=1, order=16)
    run("step2_identity_dynamic", mats[1], x0=0, dynamic=1)
    run("warm_static", mats[1], x0=2, x0_matrix=Xprev, dynamic=0)
    _, iw = run("warm_dynamic", mats[1], x0=2, x0_matrix=Xprev, dynamic=1)
    # every Newton-Schulz step the warm run took, unrolled into one
    # construction (at most 6: 2^6 - 1 powers of the residual per sample)
    u = min(max(iw["iterations"], 1), 6)
    run("warm_unrolled", mats[1], x0=2, x0_matrix=Xprev, dynamic=1, unroll=u)
    out["unroll"] = u
    return out


def lowrank_form(h2, torch, si, rank=220):
    """Hessian products of the plain construction against the global
    low-rank pre-pass + construction of H - B B^T (Sec. 3.3) on a misfit-only
    advection-diffusion Gauss-Newton Hessian with limited data (128 x 128
    grid, 20 observation points at 10 times: a misfit of global rank at most
    200), both at 1e-4."""
    cfg = si.config_advdiff2d(128, nobs=20)
    S = h2.AdvDiffSampler(cfg)
    tree = h2.Tree(cfg["points"], cfg["leaf"], cfg["eta"])
    o = h2.opts(rank_cap=cfg["cap"], oversample=cfg["p"], tol=1e-4, adaptive=1, max_rounds=16,
                seed=6)
    out = {"workload": "advdiff2d 128x128 (N=16384) misfit-only, 20 points x 10 times, cap 32, "
                       "eps 1e-4, global rank %d" % rank}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = h2.build(tree, S, o)
    torch.cuda.synchronize()
    out["plain"] = {"s": round(time.perf_counter() - t0, 3), "applies": st["applies"],
                    "converged": st["converged"]}
    t0 = time.perf_counter()
    _, sl = h2.build_lowrank(tree, S, rank, o)
    torch.cuda.synchronize()
    out["lowrank"] = {"s": round(time.perf_counter() - t0, 3), "applies": sl["applies"],
                      "global_applies": sl["global_applies"], "global_rank": sl["global_rank"],
                      "residual_applies": sl["applies"] - sl["global_applies"],
                      "converged": sl["converged"]}
    print("global low rank: plain %d products, low rank + residual %d (%d global)" % (
        st["applies"], sl["applies"], sl["global_applies"]), file=sys.stderr, flush=True)
    return out


def cpu_baseline(cfg):
    """The oracle, as it stands, timed on the same workload: the full FP64
    build of the diffusion Hessian and the full Newton-Schulz run from I / nu
    to ||I - A X||_2 <= 1e-4 with the dynamic threshold (nothing extrapolated)."""
    from oracle.hessians import DiffusionGN, tree_order
    from oracle.ns import build as obuild, newton_schulz as ons, power_norm
    from oracle.tree import Tree as OTree

    T = OTree(cfg["points"], cfg["leaf"], cfg["eta"])
    G = DiffusionGN(cfg)
    A = tree_order(G.apply, T.perm)
    t0 = time.perf_counter()
    nu, _ = power_norm(A, T.n, cfg["seed"])
    H, pr = obuild(A, T, cfg["tol"], nu, cfg["cap"], cfg["p"], adaptive=True, max_rounds=16,
                   seed=cfg["seed"])
    t_build = time.perf_counter() - t0
    print("cpu baseline: oracle build %.1f s" % t_build, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    _, info = ons(H, 1e-4, 60, T.leaf_size, cfg["p"], x0="identity", dynamic=True,
                  adaptive=True, max_rounds=16, seed=cfg["seed"])
    t_ns = time.perf_counter() - t0
    cores, model = host_cpu()
    return {"value": round(t_build + t_ns, 3), "unit": "s", "cores": blas_threads(),
            "kind": "oracle", "host_cores": cores, "cpu_model": model,
            "build_s": round(t_build, 3), "ns_s": round(t_ns, 3),
            "ns_iterations": info["iterations"], "ns_residual": info["E"][-1],
            "sample": "the whole step, timed: oracle (numpy/LAPACK FP64) build of the "
                      "diffusion2d Hessian at 1e-4 + Newton-Schulz from I/nu to 1e-4 "
                      "(%d iterations), same seeds as the GPU step" % info["iterations"]}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(problems would shard by independent Hessians or subtrees); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2003_10173_amd as h2
    import seeded_inputs as si

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.forms_only:
        # reference copy of known size (512 MiB each way) for scaling byte counters
        src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            h2.stream_copy(src, dst)
        torch.cuda.synchronize()
        del src, dst
        fns = {"appendix_a": lambda: appendix_a_form(h2, torch, si, args.appendix_grid),
               "global_lowrank": lambda: lowrank_form(h2, torch, si),
               "precision_ladder": lambda: precision_ladder(h2, torch, si, stream),
               "learned": lambda: learned_form(h2, torch, si),
               "batched": lambda: batched_form(h2, torch, si),
               "c3_inverse": lambda: c3_inverse_form(h2, torch, si)}
        print(json.dumps({k: fns[k]() for k in args.only.split(",")}), flush=True)
        return
    cfg = si.config_diffusion2d(args.grid)
    tree = h2.Tree(cfg["points"], cfg["leaf"], cfg["eta"])
    sampler = h2.DiffusionSampler(cfg)
    bopts = h2.opts(rank_cap=cfg["cap"], oversample=cfg["p"], tol=cfg["tol"], adaptive=1,
                    max_rounds=16, seed=cfg["seed"])
    nopts = h2.ns_opts(eps=1e-4, max_iter=60, x0=0, dynamic=1, rank_cap=0,
                       oversample=cfg["p"], adaptive=1, max_rounds=16, seed=cfg["seed"])

    checks = {"build_converged": True, "ns_status_ok": True, "ns_residual_le_1e-4": True}

    def check_step(bst, nst):
        # the step counts only if the build met its estimator and Newton-Schulz
        # reached ||I - A X||_2 <= 1e-4
        checks["build_converged"] &= bool(bst["converged"])
        checks["ns_status_ok"] &= nst["status"] == 0
        checks["ns_residual_le_1e-4"] &= nst["resid"][-1] <= 1e-4

    def step():
        A, bst = h2.build(tree, sampler, bopts)
        X, nst = h2.newton_schulz(A, nopts)
        check_step(bst, nst)
        return A, bst, X, nst

    for i in range(args.warmup):
        _, b0, _, n0 = step()
        torch.cuda.synchronize()
        print("warmup step %d: build %.1f ms, NS %d iterations %.1f ms" % (
            i, b0["time_ms"][7], n0["iterations"], n0["time_ms"][3]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    h2.timing_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        A, bst, X, nst = step()
        print("step %d: build %.1f ms, NS %d iterations %.1f ms, residual %.2e" % (
            i, bst["time_ms"][7], nst["iterations"], nst["time_ms"][3], nst["resid"][-1]),
            file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    # dominant kernel, timed live by HIP events on the stream it ran on
    launches, k_ms, k_flops = h2.timing_read(DOMINANT)
    h2.timing_enable(False)
    k_avg = k_ms / max(launches, 1)
    k_tflops = k_flops / max(k_ms, 1e-9) / 1e9
    roofline = {"bound": "alu", "achieved": round(k_tflops, 4), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(k_tflops / FP64_PEAK_TFLOPS, 6),
                "traffic": traffic_per_launch(), "kernel": DOMINANT,
                "launches": launches, "avg_launch_ms": round(k_avg, 4),
                "flops_per_launch": k_flops / max(launches, 1),
                "share_of_step": round(k_ms / elapsed / 1e3, 4)}

    # ---- HGEMV of the built Hessian (the NS sampler is all HGEMVs), all stages
    nv = args.hgemv_nv
    n = tree.n
    x = torch.randn(nv, n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    words, mbytes = A.words()
    ms = hip_events_time(lambda: A.gemv(x, y), args.hgemv_reps, stream)
    alg_bytes = mbytes + 2 * 8 * n * nv
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    hgemv = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gbs / HBM_PEAK_GBS, 5), "nv": nv,
             "alg_bytes_per_call": int(alg_bytes), "ms_per_call": round(ms, 5)}
    # reference copy of known size (512 MiB each way) for scaling byte counters
    src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        h2.stream_copy(src, dst)
    torch.cuda.synchronize()
    del src, dst

    forms = None
    if not args.no_forms:
        # mixed precision on the same workload: FP32 sampling, FP64 residual + refinement
        mopts = h2.ns_opts(eps=1e-4, max_iter=60, x0=0, dynamic=1, rank_cap=0,
                           oversample=cfg["p"], adaptive=1, max_rounds=16, seed=cfg["seed"],
                           prec=h2.H2_FP32)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Am, bm = h2.build(tree, sampler, bopts)
        Xm, nm = h2.newton_schulz(Am, mopts)
        torch.cuda.synchronize()
        t_mixed = time.perf_counter() - t1
        mixed_ok = bool(bm["converged"]) and nm["status"] == 0 and nm["resid"][-1] <= 1e-4
        print("mixed step: %.1f ms, %d iterations (%d FP32), residual %.2e" % (
            1e3 * t_mixed, nm["iterations"], nm["low_iterations"], nm["resid"][-1]),
            file=sys.stderr, flush=True)
        # the same step with hyperpower iterations of order 4 and 8 (Appendix A.2):
        # fewer, wider constructions -- the work moves from compression to sampling
        hyper = {}
        for order in (4, 8):
            hopts = h2.ns_opts(eps=1e-4, max_iter=60, x0=0, dynamic=1, rank_cap=0,
                               oversample=cfg["p"], adaptive=1, max_rounds=16, seed=cfg["seed"],
                               order=order)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            Ah, bh = h2.build(tree, sampler, bopts)
            Xh, nh = h2.newton_schulz(Ah, hopts)
            torch.cuda.synchronize()
            th = time.perf_counter() - t1
            hyper["order%d" % order] = {
                "s": round(th, 4), "iterations": nh["iterations"], "residual": nh["resid"][-1],
                "samples": int(sum(nh["applies"])),
                "valid": bool(bh["converged"]) and nh["status"] == 0 and nh["resid"][-1] <= 1e-4}
            print("hyperpower order %d step: %.1f ms, %d iterations, residual %.2e" % (
                order, 1e3 * th, nh["iterations"], nh["resid"][-1]), file=sys.stderr, flush=True)
        forms = {"plain_fp64_s": round(ms_per_step / 1e3, 4),
                 "hyperpower": hyper,
                 "mixed_fp32_s": round(t_mixed, 4),
                 "mixed_iterations": nm["iterations"], "mixed_fp32_iterations": nm["low_iterations"],
                 "mixed_residual": nm["resid"][-1], "mixed_valid": mixed_ok,
                 "precision_ladder": precision_ladder(h2, torch, si, stream),
                 "learned": learned_form(h2, torch, si),
                 "batched": batched_form(h2, torch, si),
                 "appendix_a": appendix_a_form(h2, torch, si, args.appendix_grid),
                 "global_lowrank": lowrank_form(h2, torch, si)}

    cpu = None
    if not args.no_cpu_baseline:
        print("cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg)

    out = {
        "metric": "build+inverse s at 1e-4 rel err (mixed/batched/learned vs plain FP64); HGEMV GB/s",
        "value": round(ms_per_step / 1e3, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "diffusion2d Gauss-Newton Hessian, %dx%d grid, N=%d, leaf %d, "
                               "rank cap %d, eps 1e-4, build + Newton-Schulz (FP64)"
                               % (args.grid, args.grid, n, cfg["leaf"], cfg["cap"]),
                   "form": "plain FP64 GPU"},
        "ns_iterations": nst["iterations"],
        "ns_residual": nst["resid"][-1],
        "build_applies": bst["applies"],
        "build_ms": round(bst["time_ms"][7], 2),
        "ns_ms": round(nst["time_ms"][3], 2),
        "ns_phase_ms": {"residual": round(nst["time_ms"][0], 2), "build": round(nst["time_ms"][1], 2),
                        "refine": round(nst["time_ms"][2], 2)},
        "hgemv_gbs": round(gbs, 2),
        "checks": checks,
        "unmeasured": "build + inverse of the 256x256 kernel Hessian (N=65536, FP32 Newton-"
                      "Schulz) and of the 256-problem batch are not timed per step; their "
                      "HGEMV and build-only forms are under forms",
        "roofline": roofline,
        "hgemv": hgemv,
        "forms": forms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if not all(checks.values()):
        print("bench: a timed step missed 1e-4 (%s); the value is not valid" % checks,
              file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
