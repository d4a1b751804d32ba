"""ctypes binding of the C ABI declared in include/h2.h (argument marshalling only).

The shared library libh2hip.so is built in-tree by paper_2003_10173_amd.build;
loading fails loudly when it is missing -- there is no fallback path.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libh2hip.so")

H2_OK, H2_EINVAL, H2_ENOMEM, H2_EDEVICE, H2_ECALLBACK, H2_ENUMERIC = 0, -1, -2, -3, -4, -5
H2_ENOTCONVERGED, H2_EDIVERGED = 1, 2
H2_FP64, H2_FP32, H2_BF16 = 0, 1, 2
H2_MAX_LEVELS = 32
H2_MAX_NS_ITERS = 128

vp = C.c_void_p
i32, i64, u32, u64, dbl, flt = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double, C.c_float
P = C.POINTER

SAMPLER_FN = C.CFUNCTYPE(C.c_int, vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp)
BATCHED_SAMPLER_FN = C.CFUNCTYPE(C.c_int, vp, C.c_int, vp, vp, C.c_int, vp, C.c_int, vp, vp)


class H2Opts(C.Structure):
    _fields_ = [("rank_cap", C.c_int), ("oversample", C.c_int), ("tol", dbl),
                ("adaptive", C.c_int), ("max_rounds", C.c_int), ("seed", u64),
                ("iteration", u32), ("norm", dbl), ("prec", C.c_int), ("learned", vp)]


class H2BuildStats(C.Structure):
    _fields_ = [("levels", C.c_int), ("weak_rank", C.c_int * H2_MAX_LEVELS),
                ("range_cols", C.c_int * H2_MAX_LEVELS), ("rounds", C.c_int * H2_MAX_LEVELS),
                ("strong_rank", C.c_int * H2_MAX_LEVELS), ("applies", i64),
                ("norm_applies", i64), ("norm", dbl),
                ("converged", C.c_int), ("cap_hit", C.c_int), ("time_ms", dbl * 8),
                ("first_cols", C.c_int * H2_MAX_LEVELS), ("global_rank", C.c_int),
                ("global_applies", i64), ("update_applies", i64)]


class H2NSOpts(C.Structure):
    _fields_ = [("eps", dbl), ("max_iter", C.c_int), ("x0", C.c_int), ("dynamic", C.c_int),
                ("eps_build", dbl), ("norm_rel", dbl), ("resid_rel", dbl), ("rank_cap", C.c_int),
                ("oversample", C.c_int), ("adaptive", C.c_int), ("max_rounds", C.c_int),
                ("seed", u64), ("prec", C.c_int), ("order", C.c_int), ("unroll", C.c_int),
                ("x0_matrix", vp)]


class H2NSStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("norm", dbl), ("resid", dbl * (H2_MAX_NS_ITERS + 1)),
                ("applies", i64 * H2_MAX_NS_ITERS), ("max_rank", C.c_int * H2_MAX_NS_ITERS),
                ("time_ms", dbl * 4), ("low_iterations", C.c_int)]


# name -> (restype, argtypes)
SIGNATURES = {
    "h2_status_string": (C.c_char_p, [C.c_int]),
    "h2_last_error": (C.c_char_p, []),
    "h2_tree_create": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, dbl, P(vp)]),
    "h2_tree_destroy": (None, [vp]),
    "h2_tree_info": (C.c_int, [vp, P(C.c_int), P(C.c_int), P(C.c_int), P(C.c_int)]),
    "h2_tree_perm": (C.c_int, [vp, vp]),
    "h2_tree_offsets": (C.c_int, [vp, C.c_int, vp]),
    "h2_tree_pair_count": (C.c_int, [vp, C.c_int, P(i64)]),
    "h2_tree_pairs": (C.c_int, [vp, C.c_int, vp]),
    "h2_opts_default": (None, [P(H2Opts)]),
    "h2_build": (C.c_int, [vp, vp, vp, P(H2Opts), vp, P(vp), P(H2BuildStats)]),
    "h2_build_batched_packed": (C.c_int, [C.c_int, vp, vp, vp, vp, vp, vp, vp, P(i64)]),
    "h2_sampler_kernel_batched_create": (C.c_int, [C.c_int, vp, vp, C.c_int, vp, vp, P(vp)]),
    "h2_sampler_kernel_batched_apply": (C.c_int, [vp, C.c_int, vp, vp, C.c_int, vp, C.c_int, vp,
                                                  vp]),
    "h2_build_lowrank": (C.c_int, [vp, vp, vp, P(H2Opts), C.c_int, vp, P(vp), P(H2BuildStats)]),
    "h2_gemv": (C.c_int, [vp, C.c_int, dbl, vp, C.c_int, dbl, vp, C.c_int, vp]),
    "h2_gemv_f32": (C.c_int, [vp, C.c_int, flt, vp, C.c_int, flt, vp, C.c_int, vp]),
    "h2_gemv_noalloc": (C.c_int, [vp, C.c_int, dbl, vp, C.c_int, dbl, vp, C.c_int, vp]),
    "h2_norm2": (C.c_int, [vp, C.c_int, dbl, u64, vp, P(dbl)]),
    "h2_matrix_convert": (C.c_int, [vp, C.c_int, P(vp)]),
    "h2_matrix_scale": (C.c_int, [vp, dbl, P(vp)]),
    "h2_matrix_identity": (C.c_int, [vp, dbl, P(vp)]),
    "h2_destroy": (None, [vp]),
    "h2_matrix_sizes": (C.c_int, [vp, vp, P(i64), P(i64), P(i64), P(i64)]),
    "h2_matrix_import": (C.c_int, [vp, vp, vp, vp, vp, vp, P(vp)]),
    "h2_matrix_ranks": (C.c_int, [vp, vp]),
    "h2_matrix_export": (C.c_int, [vp, vp, vp, vp, vp]),
    "h2_matrix_words": (C.c_int, [vp, P(i64), P(i64)]),
    "h2_ns_opts_default": (None, [P(H2NSOpts)]),
    "h2_timing_enable": (C.c_int, [C.c_int]),
    "h2_build_batched": (C.c_int, [C.c_int, vp, vp, vp, vp, vp, vp, vp]),
    "h2_residual_norm_batched": (C.c_int, [C.c_int, vp, vp, dbl, C.c_int, u64, u32, C.c_int, vp,
                                           vp, vp, vp]),
    "h2_newton_schulz_batched": (C.c_int, [C.c_int, vp, vp, vp, vp, vp, vp]),
    "h2_mlp_create": (C.c_int, [vp, P(vp)]),
    "h2_mlp_params": (C.c_int, [vp, vp]),
    "h2_mlp_forward": (C.c_int, [vp, C.c_int, vp, vp, vp]),
    "h2_mlp_gradient": (C.c_int, [vp, C.c_int, vp, vp, vp, vp, vp]),
    "h2_mlp_train_step": (C.c_int, [vp, C.c_int, vp, vp, C.c_float, vp]),
    "h2_mlp_last_loss": (C.c_int, [vp, P(C.c_float)]),
    "h2_mlp_destroy": (None, [vp]),
    "h2_records_enable": (C.c_int, [C.c_int]),
    "h2_records_read": (C.c_int, [vp, vp, vp]),
    "h2_stream_copy": (C.c_int, [vp, vp, i64, vp]),
    "h2_timing_read": (C.c_int, [C.c_char_p, P(i64), P(dbl), P(dbl)]),
    "h2_newton_schulz": (C.c_int, [vp, P(H2NSOpts), vp, P(vp), P(H2NSStats)]),
    "h2_residual_norm": (C.c_int, [vp, vp, dbl, C.c_int, u64, u32, vp, P(dbl)]),
    "h2_sampler_kernel_create": (C.c_int, [vp, C.c_int, C.c_int, dbl, dbl, P(vp)]),
    "h2_sampler_kernel_apply": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "h2_sampler_diffusion_create": (C.c_int, [C.c_int, dbl, dbl, C.c_int, vp, C.c_int, vp,
                                              C.c_int, dbl, dbl, dbl, P(vp)]),
    "h2_sampler_diffusion_apply": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "h2_sampler_advdiff_create": (C.c_int, [C.c_int, dbl, C.c_int, vp, C.c_int, vp, C.c_int, dbl,
                                            vp, vp, vp, C.c_int, P(vp)]),
    "h2_sampler_advdiff_apply": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "h2_sampler_minsurf_create": (C.c_int, [C.c_int, vp, P(vp)]),
    "h2_sampler_minsurf_apply": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "h2_sampler_h2_apply": (C.c_int, [vp, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp]),
    "h2_sampler_destroy": (None, [vp]),
    # test hooks (include/h2_testing.h)
    "h2_test_gemm": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, dbl, vp, C.c_int, vp,
                               C.c_int, dbl, vp, C.c_int]),
    "h2_test_qr": (C.c_int, [C.c_int, C.c_int, vp, vp, vp]),
    "h2_test_svd": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, vp]),
    "h2_test_svd_batch": (C.c_int, [C.c_int, vp, vp, vp, vp, vp, vp]),
    "h2_test_mfma_layout": (C.c_int, [C.c_int, vp]),
    "h2_test_wave_sum": (C.c_int, [vp, vp]),
    "h2_test_svd_spin_limit": (None, [C.c_int]),
    "h2_test_gemv_tile": (C.c_int, [vp, C.c_int, vp, vp, C.c_int]),
    "h2_test_tuned_tile": (C.c_int, [vp, C.c_int]),
    "h2_test_gemv_split_groups": (C.c_int, [vp, C.c_int]),
    "h2_test_cholqr": (C.c_int, [C.c_int, C.c_int, vp, vp, vp, C.c_int]),
    "h2_test_keep_factors": (None, [C.c_int]),
    "h2_test_factors": (C.c_int, [C.c_int, vp, vp, vp]),
}


class _Lib:
    def __init__(self):
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libh2hip.so is not built (expected at %s); run "
                "`python -m paper_2003_10173_amd.build` -- there is no fallback" % LIB_PATH)
        self._dll = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)

    def __getattr__(self, name):
        if name not in SIGNATURES:
            raise AttributeError(name)
        fn = getattr(self._dll, name)
        res, args = SIGNATURES[name]
        fn.restype = res
        fn.argtypes = args
        setattr(self, name, fn)
        return fn

    def has(self, name):
        try:
            getattr(self._dll, name)
            return True
        except AttributeError:
            return False


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = _Lib()
    return _LIB


class H2Error(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        L = lib()
        msg = L.h2_last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (where, L.h2_status_string(status).decode(), msg))


def check(status, where, allow=(H2_OK,)):
    if status not in allow:
        raise H2Error(status, where)
    return status
