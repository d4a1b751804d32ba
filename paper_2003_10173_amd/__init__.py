"""MI355X-native H2 Hessian construction, HGEMV and Newton-Schulz inversion.

Thin Python layer over the C ABI in include/h2.h (libh2hip.so): it marshals
arguments only.  Device memory and streams come from PyTorch (ROCm); every step
of construction, product and inversion runs in the library's HIP kernels.
Implements arXiv 2003.10173 (Sec. 3 construction and operations, Appendix A
Newton-Schulz) -- see the header for the passage behind each entry point.
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import (BATCHED_SAMPLER_FN, H2_BF16, H2_FP32, H2_FP64, H2BuildStats, H2Error,
                   H2NSOpts, H2NSStats, H2Opts, SAMPLER_FN, check, lib)

__all__ = ["Tree", "H2Matrix", "build", "newton_schulz", "residual_norm", "KernelSampler",
           "DiffusionSampler", "AdvDiffSampler", "MinSurfSampler", "H2Sampler", "PythonSampler", "opts",
           "ns_opts", "H2_FP64", "H2_FP32", "H2_BF16", "H2Error", "lib"]


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Tree:
    """Cluster tree + admissibility lists (host C++; bit-exact with the oracle)."""

    def __init__(self, points, leaf_size, eta=0.7):
        pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64))
        if pts.ndim == 1:
            pts = pts.reshape(-1, 1)
        self.points = pts
        h = C.c_void_p()
        check(lib().h2_tree_create(pts.ctypes.data, pts.shape[0], pts.shape[1], int(leaf_size),
                                   float(eta), C.byref(h)), "h2_tree_create")
        self.handle = h
        n, L, lf, d = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        check(lib().h2_tree_info(h, C.byref(n), C.byref(L), C.byref(lf), C.byref(d)), "info")
        self.n, self.L, self.leaf_size, self.dim = n.value, L.value, lf.value, d.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().h2_tree_destroy(h)
            except Exception:  # noqa: BLE001 - interpreter shutdown
                pass
            self.handle = None

    @property
    def perm(self):
        p = np.empty(self.n, dtype=np.int64)
        check(lib().h2_tree_perm(self.handle, p.ctypes.data), "h2_tree_perm")
        return p

    def offsets(self, level):
        o = np.empty((1 << level) + 1, dtype=np.int64)
        check(lib().h2_tree_offsets(self.handle, level, o.ctypes.data), "h2_tree_offsets")
        return o

    def pairs(self, level):
        """Far pairs at `level` (0..L) or near pairs (level=-1), sorted (t, s)."""
        cnt = C.c_int64()
        check(lib().h2_tree_pair_count(self.handle, level, C.byref(cnt)), "pair_count")
        out = np.empty((cnt.value, 2), dtype=np.int32)
        if cnt.value:
            check(lib().h2_tree_pairs(self.handle, level, out.ctypes.data), "pairs")
        return out

    def nclusters(self):
        return (2 << self.L) - 1


class H2Matrix:
    """Device-resident H2 matrix handle."""

    def __init__(self, handle, tree):
        self.handle = handle
        self.tree = tree          # keep the tree alive as long as the matrix

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().h2_destroy(h)
            except Exception:  # noqa: BLE001 - interpreter shutdown
                pass
            self.handle = None

    # -- construction from host arrays (packed layout of include/h2.h)
    @staticmethod
    def from_host(tree, ranks, U, E, S, D):
        ranks = np.ascontiguousarray(ranks, dtype=np.int32)
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (U, E, S, D)]
        ptrs = [a.ctypes.data if a.size else None for a in arrs]
        h = C.c_void_p()
        check(lib().h2_matrix_import(tree.handle, ranks.ctypes.data, *ptrs, C.byref(h)),
              "h2_matrix_import")
        return H2Matrix(h, tree)

    @staticmethod
    def identity(tree, alpha):
        h = C.c_void_p()
        check(lib().h2_matrix_identity(tree.handle, float(alpha), C.byref(h)), "identity")
        return H2Matrix(h, tree)

    def ranks(self):
        r = np.empty(self.tree.nclusters(), dtype=np.int32)
        check(lib().h2_matrix_ranks(self.handle, r.ctypes.data), "h2_matrix_ranks")
        return r

    def sizes(self):
        r = self.ranks()
        out = [C.c_int64() for _ in range(4)]
        check(lib().h2_matrix_sizes(self.tree.handle, r.ctypes.data, *[C.byref(o) for o in out]),
              "h2_matrix_sizes")
        return [o.value for o in out]

    def export(self):
        nU, nE, nS, nD = self.sizes()
        arrs = [np.empty(max(k, 1)) for k in (nU, nE, nS, nD)]
        check(lib().h2_matrix_export(self.handle, *[a.ctypes.data for a in arrs]), "export")
        return self.ranks(), arrs[0][:nU], arrs[1][:nE], arrs[2][:nS], arrs[3][:nD]

    def words(self):
        w, b = C.c_int64(), C.c_int64()
        check(lib().h2_matrix_words(self.handle, C.byref(w), C.byref(b)), "h2_matrix_words")
        return w.value, b.value

    def convert(self, prec):
        h = C.c_void_p()
        check(lib().h2_matrix_convert(self.handle, int(prec), C.byref(h)), "h2_matrix_convert")
        return H2Matrix(h, self.tree)

    def scaled(self, alpha):
        h = C.c_void_p()
        check(lib().h2_matrix_scale(self.handle, float(alpha), C.byref(h)), "h2_matrix_scale")
        return H2Matrix(h, self.tree)

    # -- products (torch CUDA tensors, column-major = torch (nv, n) row-major)
    def gemv(self, x, y=None, alpha=1.0, beta=0.0, stream=None):
        """y = alpha A x + beta y for x of shape (n,) or (nv, n) (columns = rows of x)."""
        import torch
        xv = x.reshape(-1, self.tree.n)
        assert xv.is_contiguous() and xv.is_cuda
        if y is None:
            y = torch.empty_like(xv)
            beta = 0.0
        yv = y.reshape(-1, self.tree.n)
        nv = xv.shape[0]
        if xv.dtype == torch.float64:
            check(lib().h2_gemv(self.handle, nv, float(alpha), _ptr(xv), self.tree.n, float(beta),
                                _ptr(yv), self.tree.n, _stream(stream)), "h2_gemv")
        elif xv.dtype == torch.float32:
            check(lib().h2_gemv_f32(self.handle, nv, float(alpha), _ptr(xv), self.tree.n,
                                    float(beta), _ptr(yv), self.tree.n, _stream(stream)),
                  "h2_gemv_f32")
        else:
            raise TypeError("vectors must be float64 or float32")
        return y

    def gemv_noalloc(self, x, y, alpha=1.0, beta=0.0, stream=None):
        """y = alpha A x + beta y (FP64) through h2_gemv_noalloc: no device
        allocation; the library's fixed per-GPU workspace is used instead."""
        import torch
        xv = x.reshape(-1, self.tree.n)
        yv = y.reshape(-1, self.tree.n)
        assert xv.is_contiguous() and yv.is_contiguous() and xv.is_cuda and yv.is_cuda
        assert xv.dtype == torch.float64 and yv.dtype == torch.float64
        assert xv.shape == yv.shape
        check(lib().h2_gemv_noalloc(self.handle, xv.shape[0], float(alpha), _ptr(xv),
                                    self.tree.n, float(beta), _ptr(yv), self.tree.n,
                                    _stream(stream)), "h2_gemv_noalloc")
        return y

    def norm2(self, max_iter=30, rel=1e-2, seed=1, stream=None):
        out = C.c_double()
        check(lib().h2_norm2(self.handle, max_iter, rel, seed, _stream(stream), C.byref(out)),
              "h2_norm2")
        return out.value


# ---------------------------------------------------------------- samplers
class _SamplerBase:
    fn = None      # ctypes function pointer (h2_sampler_fn)
    ctx = None

    def __call__(self, omega, stream=None):
        """Apply to a (ncols, n) float64 CUDA tensor (columns = rows)."""
        import torch
        y = torch.empty_like(omega)
        rc = self.fn(self.ctx, omega.shape[1], omega.shape[0], _ptr(omega), omega.shape[1],
                     _ptr(y), omega.shape[1], _stream(stream))
        if rc != 0:
            raise RuntimeError("sampler failed with %d" % rc)
        return y


class _NativeSampler(_SamplerBase):
    apply_name = None

    def _finish(self, h):
        self.ctx = h
        self.fn = C.cast(getattr(lib()._dll, self.apply_name), C.c_void_p).value
        self.fn = SAMPLER_FN(self.fn)

    def __del__(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            try:
                lib().h2_sampler_destroy(self.ctx)
            except Exception:  # noqa: BLE001 - interpreter shutdown
                pass
            self.ctx = None


class KernelSampler(_NativeSampler):
    """H_ij = exp(-|p_i - p_j|/ell) + shift delta_ij (HIP kernel)."""
    apply_name = "h2_sampler_kernel_apply"

    def __init__(self, points, ell, shift):
        pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64))
        if pts.ndim == 1:
            pts = pts.reshape(-1, 1)
        h = C.c_void_p()
        check(lib().h2_sampler_kernel_create(pts.ctypes.data, pts.shape[0], pts.shape[1],
                                             float(ell), float(shift), C.byref(h)), "kernel")
        self._finish(h)


class DiffusionSampler(_NativeSampler):
    apply_name = "h2_sampler_diffusion_apply"

    def __init__(self, cfg):
        steps = np.ascontiguousarray(cfg["obs_steps"], dtype=np.int32)
        oi = np.ascontiguousarray(cfg["obs_index"], dtype=np.int32)
        h = C.c_void_p()
        check(lib().h2_sampler_diffusion_create(cfg["grid"], cfg["kappa"], cfg["dt"],
                                                cfg["steps"], steps.ctypes.data, len(steps),
                                                oi.ctypes.data, len(oi), cfg["sigma"],
                                                cfg["gamma"], cfg["beta"], C.byref(h)),
              "diffusion")
        self._finish(h)


class AdvDiffSampler(_NativeSampler):
    apply_name = "h2_sampler_advdiff_apply"

    def __init__(self, cfg):
        steps = np.ascontiguousarray(cfg["obs_steps"], dtype=np.int32)
        pts = np.ascontiguousarray(cfg["obs_points"], dtype=np.float64)
        a = np.ascontiguousarray(cfg["mode_a"], dtype=np.int32)
        b = np.ascontiguousarray(cfg["mode_b"], dtype=np.int32)
        s = np.ascontiguousarray(cfg["mode_s"], dtype=np.float64)
        h = C.c_void_p()
        check(lib().h2_sampler_advdiff_create(cfg["grid"], cfg["kappa"], cfg["steps"],
                                              steps.ctypes.data, len(steps), pts.ctypes.data,
                                              len(pts), cfg["sigma"], a.ctypes.data,
                                              b.ctypes.data, s.ctypes.data, len(a), C.byref(h)),
              "advdiff")
        self._finish(h)


class MinSurfSampler(_NativeSampler):
    """Hessian of the discrete minimal-surface area at the surface
    cfg["heights"] ((g+2) x (g+2) node heights, boundary included)."""
    apply_name = "h2_sampler_minsurf_apply"

    def __init__(self, cfg):
        g = int(cfg["grid"])
        hts = np.ascontiguousarray(cfg["heights"], dtype=np.float64)
        if hts.shape != (g + 2, g + 2):
            raise ValueError("heights must be (g+2) x (g+2)")
        h = C.c_void_p()
        check(lib().h2_sampler_minsurf_create(g, hts.ctypes.data, C.byref(h)), "minsurf")
        self._finish(h)


class H2Sampler(_SamplerBase):
    """Sampler applying an existing H2 matrix (for rebuild / idempotence checks)."""

    def __init__(self, mat):
        self.mat = mat
        self.ctx = mat.handle
        self.fn = SAMPLER_FN(C.cast(lib()._dll.h2_sampler_h2_apply, C.c_void_p).value)


class PythonSampler(_SamplerBase):
    """Wrap a Python callable f(omega_tensor (ncols, n)) -> y_tensor on the device.

    For tests (counting / failing wrappers); the callable must enqueue its work on
    the current torch stream.
    """

    def __init__(self, n, func):
        import torch
        self.n = n
        self.func = func
        self.calls = 0
        self.columns = 0

        def cb(ctx, n_, ncols, om, ldo, y, ldy, stream):
            try:
                self.calls += 1
                self.columns += ncols
                omv = _wrap(om, ncols, ldo)
                yv = _wrap(y, ncols, ldy)
                out = func(omv[:, :n_])
                if out is None:
                    return 1
                yv[:, :n_].copy_(out)
                return 0
            except Exception:  # noqa: BLE001 - reported as a callback failure
                return 1

        def _wrap(ptr, ncols, ld):
            return _tensor_from_ptr(ptr, ncols, ld)

        self._cb = SAMPLER_FN(cb)
        self.fn = self._cb
        self.ctx = None


def _tensor_from_ptr(ptr, ncols, ld):
    import torch

    class _Iface:
        def __init__(self):
            self.__cuda_array_interface__ = {
                "shape": (ncols, ld), "typestr": "<f8", "data": (ptr, False), "version": 2,
                "strides": None}
    return torch.as_tensor(_Iface(), device="cuda")


# ---------------------------------------------------------------- construction
def opts(**kw):
    o = H2Opts()
    lib().h2_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "learned":
            o._mlp = v                      # keep the network alive with the options
            v = v.handle.value if v is not None else None
        setattr(o, k, v)
    return o


def ns_opts(**kw):
    """h2_ns_opts with defaults; x0_matrix takes an H2Matrix (warm start,
    x0 = 2), kept alive with the options."""
    o = H2NSOpts()
    lib().h2_ns_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "x0_matrix":
            o._x0 = v
            v = v.handle.value if v is not None else None
        setattr(o, k, v)
    return o


def stats_dict(st, levels):
    return dict(levels=st.levels, weak_rank=list(st.weak_rank[1:levels + 1]),
                range_cols=list(st.range_cols[1:levels + 1]),
                rounds=list(st.rounds[1:levels + 1]),
                strong_rank=list(st.strong_rank[:levels + 1]), applies=st.applies,
                norm_applies=st.norm_applies,
                norm=st.norm, converged=bool(st.converged), cap_hit=bool(st.cap_hit),
                time_ms=list(st.time_ms), first_cols=list(st.first_cols[1:levels + 1]),
                global_rank=st.global_rank, global_applies=st.global_applies,
                update_applies=st.update_applies)


def build(tree, sampler, o=None, stream=None, allow_not_converged=True):
    """Peeling + recompression (h2_build); returns (H2Matrix, stats dict)."""
    if o is None:
        o = opts()
    h = C.c_void_p()
    st = H2BuildStats()
    allow = (0, 1) if allow_not_converged else (0,)
    check(lib().h2_build(tree.handle, C.cast(sampler.fn, C.c_void_p), sampler.ctx, C.byref(o),
                         _stream(stream), C.byref(h), C.byref(st)), "h2_build", allow)
    return H2Matrix(h, tree), stats_dict(st, tree.L)


def build_lowrank(tree, sampler, global_rank, o=None, stream=None, allow_not_converged=True):
    """Global low-rank pre-pass B B^T, construction of H - B B^T, and B B^T
    added back (h2_build_lowrank); returns (H2Matrix, stats dict)."""
    if o is None:
        o = opts()
    h = C.c_void_p()
    st = H2BuildStats()
    allow = (0, 1) if allow_not_converged else (0,)
    check(lib().h2_build_lowrank(tree.handle, C.cast(sampler.fn, C.c_void_p), sampler.ctx,
                                 C.byref(o), int(global_rank), _stream(stream), C.byref(h),
                                 C.byref(st)), "h2_build_lowrank", allow)
    return H2Matrix(h, tree), stats_dict(st, tree.L)


def build_batched(trees, samplers, opts_list, stream=None):
    """Level-synchronous construction of several problems (h2_build_batched);
    returns ([H2Matrix], [stats dict], status)."""
    n = len(trees)
    assert len(samplers) == n and len(opts_list) == n
    th = (C.c_void_p * n)(*[t.handle.value for t in trees])
    fns = (C.c_void_p * n)(*[C.cast(s.fn, C.c_void_p).value for s in samplers])
    ctxs = (C.c_void_p * n)(*[s.ctx.value if isinstance(s.ctx, C.c_void_p) else s.ctx
                              for s in samplers])
    oa = (H2Opts * n)(*opts_list)
    out = (C.c_void_p * n)()
    st = (H2BuildStats * n)()
    rc = lib().h2_build_batched(n, th, fns, ctxs, oa, _stream(stream), out, st)
    check(rc, "h2_build_batched", (0, 1))
    mats = [H2Matrix(C.c_void_p(out[i]), trees[i]) for i in range(n)]
    return mats, [stats_dict(st[i], trees[i].L) for i in range(n)], rc


class KernelBatchSampler:
    """One h2_batched_sampler_fn for several kernel matrices (packed layout;
    one HIP launch per call).  calls counts the calls."""

    def __init__(self, point_sets, ells, shifts):
        pts = [np.asarray(p, dtype=np.float64).reshape(len(p), -1) for p in point_sets]
        dim = pts[0].shape[1]
        self.row_off = np.concatenate([[0], np.cumsum([len(p) for p in pts])]).astype(np.int64)
        P = np.ascontiguousarray(np.concatenate(pts))
        e = np.ascontiguousarray(ells, dtype=np.float64)
        sh = np.ascontiguousarray(shifts, dtype=np.float64)
        h = C.c_void_p()
        check(lib().h2_sampler_kernel_batched_create(len(pts), self.row_off.ctypes.data,
                                                     P.ctypes.data, dim, e.ctypes.data,
                                                     sh.ctypes.data, C.byref(h)), "kernel_batched")
        self.ctx = h
        self.calls = 0
        native = C.cast(lib()._dll.h2_sampler_kernel_batched_apply, C.c_void_p).value
        self._native = BATCHED_SAMPLER_FN(native)

        def counted(ctx, nprob, off, act, ncols, om, ld, y, stream):
            self.calls += 1
            return self._native(ctx, nprob, off, act, ncols, om, ld, y, stream)
        self.fn = BATCHED_SAMPLER_FN(counted)

    def __del__(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            try:
                lib().h2_sampler_destroy(self.ctx)
            except Exception:  # noqa: BLE001 - interpreter shutdown
                pass
            self.ctx = None


def build_batched_packed(trees, sampler, opts_list, stream=None):
    """Batched construction with one batched sampler over the packed layout
    (h2_build_batched_packed); returns ([H2Matrix], [stats dict], status,
    sampler calls)."""
    n = len(trees)
    th = (C.c_void_p * n)(*[t.handle.value for t in trees])
    oa = (H2Opts * n)(*opts_list)
    out = (C.c_void_p * n)()
    st = (H2BuildStats * n)()
    calls = C.c_int64()
    rc = lib().h2_build_batched_packed(n, th, C.cast(sampler.fn, C.c_void_p), sampler.ctx, oa,
                                       _stream(stream), out, st, C.byref(calls))
    check(rc, "h2_build_batched_packed", (0, 1))
    mats = [H2Matrix(C.c_void_p(out[i]), trees[i]) for i in range(n)]
    return mats, [stats_dict(st[i], trees[i].L) for i in range(n)], rc, calls.value


def newton_schulz_batched(As, opts_list, stream=None):
    """Newton-Schulz of several matrices in lock step (h2_newton_schulz_batched);
    returns ([X], [info dict])."""
    n = len(As)
    ah = (C.c_void_p * n)(*[A.handle.value for A in As])
    oa = (H2NSOpts * n)(*opts_list)
    out = (C.c_void_p * n)()
    st = (H2NSStats * n)()
    status = (C.c_int * n)()
    check(lib().h2_newton_schulz_batched(n, ah, oa, _stream(stream), out, st, status),
          "h2_newton_schulz_batched")
    Xs, infos = [], []
    for i in range(n):
        k = st[i].iterations
        infos.append(dict(iterations=k, norm=st[i].norm, resid=list(st[i].resid[:k + 1]),
                          applies=list(st[i].applies[:k]), max_rank=list(st[i].max_rank[:k]),
                          time_ms=list(st[i].time_ms), status=status[i],
                          low_iterations=st[i].low_iterations))
        Xs.append(H2Matrix(C.c_void_p(out[i]), As[i].tree))
    return Xs, infos


def residual_norm_batched(As, Xs, rel=1e-2, max_iter=30, seed=1, iteration=0, graph=True,
                          stream=None):
    """||I - A_i X_i||_2 for several pairs in lock step; returns (E, iters,
    history (n x max_iter))."""
    n = len(As)
    ah = (C.c_void_p * n)(*[a.handle.value for a in As])
    xh = (C.c_void_p * n)(*[x.handle.value for x in Xs])
    out = np.zeros(n)
    its = np.zeros(n, dtype=np.int32)
    hist = np.zeros((n, max_iter))
    check(lib().h2_residual_norm_batched(n, ah, xh, rel, max_iter, seed, iteration,
                                         1 if graph else 0, _stream(stream), out.ctypes.data,
                                         its.ctypes.data, hist.ctypes.data),
          "h2_residual_norm_batched")
    return out, its, hist


def newton_schulz(A, o=None, stream=None):
    """Hierarchical Newton-Schulz (h2_newton_schulz); returns (X, stats dict, status)."""
    if o is None:
        o = ns_opts()
    h = C.c_void_p()
    st = H2NSStats()
    rc = lib().h2_newton_schulz(A.handle, C.byref(o), _stream(stream), C.byref(h), C.byref(st))
    check(rc, "h2_newton_schulz", (0, 1, 2))
    k = st.iterations
    info = dict(iterations=k, norm=st.norm, resid=list(st.resid[:k + 1]),
                applies=list(st.applies[:k]), max_rank=list(st.max_rank[:k]),
                time_ms=list(st.time_ms), status=rc, low_iterations=st.low_iterations)
    return H2Matrix(h, A.tree), info


def residual_norm(A, X, rel=1e-2, max_iter=30, seed=1, iteration=0, stream=None):
    out = C.c_double()
    check(lib().h2_residual_norm(A.handle, X.handle, rel, max_iter, seed, iteration,
                                 _stream(stream), C.byref(out)), "h2_residual_norm")
    return out.value


def timing_enable(on=True):
    """Start (clearing totals) or stop bracketing the library's timed kernel
    launches with HIP events on their own streams."""
    check(lib().h2_timing_enable(1 if on else 0), "h2_timing_enable")


def timing_read(kernel):
    """(launches, total ms, algorithmic work) of a timed kernel since enable."""
    n = C.c_int64()
    ms = C.c_double()
    w = C.c_double()
    check(lib().h2_timing_read(kernel.encode(), C.byref(n), C.byref(ms), C.byref(w)),
          "h2_timing_read")
    return n.value, ms.value, w.value


def stream_copy(src, dst):
    """dst[:] = src[:] for contiguous CUDA float64 tensors by the library's
    plain copy kernel, on torch's current stream."""
    import torch
    assert src.dtype == torch.float64 and dst.dtype == torch.float64
    assert src.is_contiguous() and dst.is_contiguous() and src.numel() == dst.numel()
    s = torch.cuda.current_stream().cuda_stream
    check(lib().h2_stream_copy(src.data_ptr(), dst.data_ptr(), src.numel(), s), "h2_stream_copy")


# ------------------------------------------------------------------ learned counts
MLP_FEATURES = 16
MLP_HIDDEN = 64
MLP_PARAMS = 5313


class MLP:
    """Rank predictor (h2_mlp): 16 -> 64 -> 64 -> 1, BF16 weights in the
    products, FP32 masters trained by Adam on the GPU."""

    def __init__(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.shape != (MLP_PARAMS,):
            raise ValueError("expected %d packed parameters" % MLP_PARAMS)
        self.handle = C.c_void_p()
        check(lib().h2_mlp_create(p.ctypes.data, C.byref(self.handle)), "h2_mlp_create")

    @staticmethod
    def he_init(seed):
        """Packed He-normal weights (FP32) and zero biases."""
        g = np.random.Generator(np.random.PCG64(seed))
        parts = [g.standard_normal((MLP_HIDDEN, MLP_FEATURES)) * np.sqrt(2.0 / MLP_FEATURES),
                 np.zeros(MLP_HIDDEN),
                 g.standard_normal((MLP_HIDDEN, MLP_HIDDEN)) * np.sqrt(2.0 / MLP_HIDDEN),
                 np.zeros(MLP_HIDDEN),
                 g.standard_normal(MLP_HIDDEN) * np.sqrt(2.0 / MLP_HIDDEN),
                 np.zeros(1)]
        return np.concatenate([a.ravel() for a in parts]).astype(np.float32)

    def params(self):
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        check(lib().h2_mlp_params(self.handle, out.ctypes.data), "h2_mlp_params")
        return out

    def forward(self, X, stream=None):
        import torch
        X = X.contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        check(lib().h2_mlp_forward(self.handle, X.shape[0], X.data_ptr(), y.data_ptr(),
                                   _stream(stream)), "h2_mlp_forward")
        return y

    def gradient(self, X, T, stream=None):
        import torch
        X, T = X.contiguous(), T.contiguous()
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        check(lib().h2_mlp_gradient(self.handle, X.shape[0], X.data_ptr(), T.data_ptr(),
                                    g.data_ptr(), loss.data_ptr(), _stream(stream)),
              "h2_mlp_gradient")
        return g, loss

    def train_step(self, X, T, lr, stream=None):
        check(lib().h2_mlp_train_step(self.handle, X.shape[0], X.data_ptr(), T.data_ptr(),
                                      C.c_float(lr), _stream(stream)), "h2_mlp_train_step")

    def last_loss(self):
        v = C.c_float()
        check(lib().h2_mlp_last_loss(self.handle, C.byref(v)), "h2_mlp_last_loss")
        return v.value

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None and self.handle.value:
                lib().h2_mlp_destroy(self.handle)
                self.handle = None
        except Exception:  # noqa: BLE001
            pass


def records_enable(on=True):
    check(lib().h2_records_enable(1 if on else 0), "h2_records_enable")


def records_read():
    """(features (count x 16), targets (count,)) recorded since enable."""
    n = C.c_int64()
    check(lib().h2_records_read(C.byref(n), None, None), "h2_records_read")
    F = np.zeros((n.value, MLP_FEATURES), dtype=np.float32)
    T = np.zeros(n.value, dtype=np.float32)
    check(lib().h2_records_read(C.byref(n), F.ctypes.data, T.ctypes.data), "h2_records_read")
    return F, T
