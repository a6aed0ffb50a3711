"""ctypes declarations for libmrrr.so (include/mrrr.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrrr.so")

RANGE_ALL, RANGE_VALUE, RANGE_INDEX = 0, 1, 2

STATUS = {
    0: "MRRR_OK", 1: "MRRR_WARN_UNVERIFIED", 2: "MRRR_ENOMEM", 3: "MRRR_ENOCONV",
    4: "MRRR_EHIP", 6: "MRRR_ETIMEOUT", 7: "MRRR_EINTERNAL",
}

#: every symbol include/mrrr.h declares
EXPORTS = (
    "mrrr_create", "mrrr_destroy", "mrrr_set_stream", "mrrr_default_options",
    "mrrr_status_string", "mrrr_dstemr", "mrrr_dstemr_batched", "mrrr_default_options_mixed",
    "mrrr_sstemr", "mrrr_dsyevr",
    "mrrr_dstemr_backward", "mrrr_dstemr_backward_batched", "mrrr_dstemr_backward_noalloc",
    "mrrr_diag_quotient",
)


class Options(ctypes.Structure):
    _fields_ = [
        ("jobz", ctypes.c_int32), ("sign_convention", ctypes.c_int32),
        ("gaptol", ctypes.c_double), ("rtol_class", ctypes.c_double),
        ("perturb_xi", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("max_rqi", ctypes.c_int32), ("max_shift_tries", ctypes.c_int32),
        ("max_depth", ctypes.c_int32), ("workers", ctypes.c_int32),
        ("slice_min", ctypes.c_int32), ("slice_max", ctypes.c_int32),
        ("timeout_s", ctypes.c_double), ("arena_scale", ctypes.c_double),
        ("trace", ctypes.c_void_p), ("trace_cap", ctypes.c_int64),
        ("lanes_per_eig", ctypes.c_int32), ("bundle", ctypes.c_int32),
        ("tune", ctypes.c_void_p), ("check_tol", ctypes.c_double), ("cond_growth_k", ctypes.c_double),
        ("bundle_helpers", ctypes.c_int32), ("pass_helpers", ctypes.c_int32),
    ]


#: numpy dtype of one mrrr_trace_t record
TRACE_FIELDS = [("type", "<i4"), ("worker", "<i4"), ("node", "<i4"), ("depth", "<i4"),
                ("a", "<i4"), ("b", "<i4"), ("t0", "<i8"), ("t1", "<i8"),
                ("x0", "<f8"), ("x1", "<f8"), ("flags", "<i4"), ("child", "<i4")]
TRACE_BYTES = 64


class Stats(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n_blocks", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
        ("largest_cluster", ctypes.c_int64), ("dmax", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("n_unverified_rrr", ctypes.c_int64), ("n_bisect_fallback", ctypes.c_int64),
        ("n_nan_retry", ctypes.c_int64), ("qd_steps", ctypes.c_int64), ("n_tasks", ctypes.c_int64),
        ("n_singleton_tasks", ctypes.c_int64), ("n_rqi_iters", ctypes.c_int64),
        ("arena_bytes", ctypes.c_int64), ("ms", ctypes.c_double), ("tree_ms", ctypes.c_double),
        ("n_sturm_guarded", ctypes.c_int64), ("n_checked", ctypes.c_int64),
        ("n_reorthogonalized", ctypes.c_int64), ("n_check_failed", ctypes.c_int64),
        ("n_check_wide", ctypes.c_int64), ("n_cond_checked", ctypes.c_int64),
        ("n_cond_failed", ctypes.c_int64), ("max_cond_growth", ctypes.c_double),
        ("n_factor_quotient", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


_lib = None


def load():
    """Load libmrrr.so; raises (never falls back) when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmrrr.so not built at {LIB_PATH}; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    p64 = ctypes.POINTER(ctypes.c_int64)
    lib.mrrr_create.argtypes = [ctypes.POINTER(vp), i32]
    lib.mrrr_create.restype = i32
    lib.mrrr_destroy.argtypes = [vp]
    lib.mrrr_destroy.restype = i32
    lib.mrrr_set_stream.argtypes = [vp, vp]
    lib.mrrr_set_stream.restype = i32
    lib.mrrr_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.mrrr_default_options.restype = None
    lib.mrrr_status_string.argtypes = [i32]
    lib.mrrr_status_string.restype = ctypes.c_char_p
    lib.mrrr_dstemr.argtypes = [vp, i64, vp, vp, i32, dbl, dbl, i64, i64, ctypes.POINTER(Options),
                                p64, vp, vp, i64, ctypes.POINTER(Stats)]
    lib.mrrr_dstemr.restype = i32
    lib.mrrr_default_options_mixed.argtypes = [ctypes.POINTER(Options)]
    lib.mrrr_default_options_mixed.restype = None
    lib.mrrr_sstemr.argtypes = [vp, i64, vp, vp, i32, ctypes.c_float, ctypes.c_float, i64, i64,
                                ctypes.POINTER(Options), p64, vp, vp, i64, ctypes.POINTER(Stats)]
    lib.mrrr_sstemr.restype = i32
    lib.mrrr_dsyevr.argtypes = [vp, i64, vp, i64, i32, dbl, dbl, i64, i64, ctypes.POINTER(Options), p64, vp, vp,
                                i64, ctypes.POINTER(Stats)]
    lib.mrrr_dsyevr.restype = i32
    lib.mrrr_dstemr_batched.argtypes = [vp, i64, p64, vp, vp, p64, ctypes.POINTER(Options), vp, vp,
                                        ctypes.POINTER(Stats)]
    lib.mrrr_dstemr_batched.restype = i32
    lib.mrrr_dstemr_backward.argtypes = [vp, i64, vp, vp, i64, vp, vp, i64, dbl, vp, vp, p64]
    lib.mrrr_dstemr_backward.restype = i32
    lib.mrrr_dstemr_backward_batched.argtypes = [vp, i64, p64, vp, vp, p64, vp, vp, dbl, vp, vp, p64]
    lib.mrrr_dstemr_backward_batched.restype = i32
    lib.mrrr_dstemr_backward_noalloc.argtypes = [vp, i64, vp, vp, i64, vp, vp, i64, dbl, vp, vp, p64]
    lib.mrrr_dstemr_backward_noalloc.restype = i32
    lib.mrrr_diag_quotient.argtypes = [vp, i64, vp, vp, vp]
    lib.mrrr_diag_quotient.restype = i32
    _lib = lib
    return lib


def default_options(mixed: bool = False, **overrides) -> Options:
    """The library's default options (mixed=True: those of the single/double
    form), with the given fields overridden."""
    o = Options()
    (load().mrrr_default_options_mixed if mixed else load().mrrr_default_options)(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class MrrrError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = load().mrrr_status_string(code).decode()
        name = STATUS.get(code, f"argument {-code}" if code < 0 else str(code))
        super().__init__(f"{where}: {name} ({msg})")


def check(code: int, where: str, allow_warn: bool = True) -> int:
    if code == 0 or (allow_warn and code == 1):
        return code
    raise MrrrError(code, where)
