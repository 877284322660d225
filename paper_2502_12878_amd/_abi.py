"""ctypes declarations of the C ABI in include/rbf.h (argument marshalling only).

The module-level functions keep the C names.  Loading fails loudly when the
HIP library has not been built: there is no fallback implementation.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbf_mi355x.so")

RBF_OK = 0
RBF_EINVAL = 1
RBF_ENOMEM = 2
RBF_ESINGULAR = 3
RBF_EDIVERGED = 4
RBF_ENOTCONVERGED = 5
RBF_EOVERFLOW = 6
RBF_EHIP = 7
RBF_MODE_FP64 = 0
RBF_MODE_MIXED = 1

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class rbf_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class rbf_iter_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("max_steps", C.c_int64), ("tol_rel", C.c_double), ("chunk", C.c_int32),
                ("mode", C.c_int32), ("inner_steps", C.c_int32), ("stall_chunks", C.c_int32),
                ("u_ref_dev", C.c_void_p), ("err_target", C.c_double)]


class rbf_iter_report(C.Structure):
    _fields_ = [("steps", C.c_int64), ("res0", C.c_double), ("res_last", C.c_double), ("res_final", C.c_double),
                ("fnorm", C.c_double), ("err_inf", C.c_double), ("err_mean_abs", C.c_double),
                ("seconds", C.c_double), ("diverged_step", C.c_int64), ("converged", C.c_int32),
                ("diverged", C.c_int32), ("err_met", C.c_int32), ("checks", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rbf_operator_info(C.Structure):
    _fields_ = [("n_interior", C.c_int64), ("n_neumann", C.c_int64), ("slices", C.c_int64), ("slots", C.c_int64),
                ("coded_slices", C.c_int64), ("max_len", C.c_int32), ("layout", C.c_int32),
                ("f64_waves", C.c_int32), ("f64_unroll", C.c_int32), ("f64_xcd_remap", C.c_int32),
                ("f64_pipeline", C.c_int32), ("f64_zigzag", C.c_int32), ("f64_codes", C.c_int32),
                ("f32_waves", C.c_int32), ("f32_unroll", C.c_int32), ("f32_xcd_remap", C.c_int32),
                ("f32_pipeline", C.c_int32), ("f32_zigzag", C.c_int32), ("f32_codes", C.c_int32),
                ("stream_bytes_f64", C.c_double), ("stream_bytes_f32", C.c_double),
                ("f64_temporal", C.c_int32), ("f32_temporal", C.c_int32), ("f32_quad", C.c_int32),
                ("code_mismatches", C.c_int32), ("t_slices", C.c_int64), ("t_slots", C.c_int64),
                ("t_coded_slices", C.c_int64), ("t_code_mismatches", C.c_int64), ("t_max_len", C.c_int32),
                ("t_waves", C.c_int32), ("t_unroll", C.c_int32), ("t_codes", C.c_int32),
                ("ns_systems", C.c_int64), ("elim_systems", C.c_int64),
                ("t_lane_order", C.c_int32), ("t_masked", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_h = C.c_void_p
_p = C.c_void_p
_st = C.c_int32

SIGNATURES = {
    "rbf_create": (_st, [C.POINTER(C.c_void_p), C.c_int, _p, C.POINTER(rbf_allocator)]),
    "rbf_destroy": (_st, [_h]),
    "rbf_set_stream": (_st, [_h, _p]),
    "rbf_status_string": (C.c_char_p, [_st]),
    "rbf_last_error": (C.c_char_p, [_h]),
    "rbf_version": (C.c_char_p, []),
    "rbf_get_sizes": (_st, [_h, C.POINTER(C.c_int), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                            C.POINTER(C.c_int32)]),
    "rbf_build_nodes": (_st, [_h, C.c_int, C.c_int64, C.c_double, C.c_uint64, _p, _p]),
    "rbf_set_nodes": (_st, [_h, C.c_int, C.c_int64, _p, _p]),
    "rbf_set_normals": (_st, [_h, _p]),
    "rbf_build_stencils": (_st, [_h, C.c_int32, _p]),
    "rbf_compute_weights": (_st, [_h, C.c_int32, _p, C.c_int]),
    "rbf_iterate": (_st, [_h, _p, _p, C.POINTER(rbf_iter_params), C.POINTER(rbf_iter_report)]),
    "rbf_apply": (_st, [_h, _p, _p]),
    "rbf_apply_transpose": (_st, [_h, _p, _p]),
    "rbf_residual": (_st, [_h, _p, _p, C.POINTER(C.c_double)]),
    "rbf_residual_noalloc": (_st, [_h, _p, _p, _p]),
    "rbf_forward_ckpt": (_st, [_h, _p, _p, C.c_int64, C.c_int64, _p, _p, C.c_double]),
    "rbf_adjoint_f": (_st, [_h, _p, C.c_int64, C.c_int64, _p, _p, C.c_double]),
    "rbf_get_stencils": (_st, [_h, _p]),
    "rbf_get_weights": (_st, [_h, _p]),
    "rbf_set_stencils": (_st, [_h, _p, C.c_int32]),
    "rbf_set_weights": (_st, [_h, _p, C.c_int]),
    "rbf_autotune": (_st, [_h]),
    "rbf_last_sweep_time": (_st, [_h, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "rbf_get_operator_info": (_st, [_h, C.POINTER(rbf_operator_info)]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """The loaded HIP library (raises LibraryMissing if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} not found: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def __getattr__(name):
    if name in SIGNATURES:
        return getattr(lib(), name)
    raise AttributeError(name)
