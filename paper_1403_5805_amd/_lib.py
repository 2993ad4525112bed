"""ctypes declarations for libjacobi.so (include/jacobi.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjacobi.so")

# jacobi_status
OK = 0
NOT_CONVERGED = 1
DIVERGED = 2
PENDING = 3
CANCELLED = 4
ERR_INVALID_ARG = -1
ERR_ZERO_DIAGONAL = -2
ERR_NONFINITE_INPUT = -3
ERR_OUT_OF_MEMORY = -4
ERR_DEVICE = -5
ERR_REJECTED = -6
ERR_INTERNAL = -7

# jacobi_dtype
F64 = 0
F32 = 1
BF16 = 2

NORM_INF = 0
NORM_L2 = 1
MODE_PLAIN = 0
MODE_REFINE = 1


class Options(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("norm", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("sweep_dtype", ctypes.c_int32),
        ("inner_rel_tol", ctypes.c_double),
        ("max_inner", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("refine_tol", ctypes.c_double),
        ("sync_every", ctypes.c_int32),
        ("profile", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("outer_iterations", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("bad_index", ctypes.c_int64),
        ("final_delta", ctypes.c_double),
        ("rel_residual", ctypes.c_double),
        ("device_ms", ctypes.c_double),
        ("sweep_kernel_ms", ctypes.c_double),
        ("sweep_kernel_launches", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name in _INFO_KEYS}


_INFO_KEYS = tuple(name for name, _ in Info._fields_)


class System(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("k", ctypes.c_int64),
        ("A", ctypes.c_void_p),
        ("lda", ctypes.c_int64),
        ("B", ctypes.c_void_p),
        ("ldb", ctypes.c_int64),
        ("X0", ctypes.c_void_p),
        ("X", ctypes.c_void_p),
        ("ldx", ctypes.c_int64),
    ]


class ServeConfig(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("max_active", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("inner_max", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("inner_rel_tol", ctypes.c_double),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("k", ctypes.c_int64),
        ("A", ctypes.c_void_p),
        ("lda", ctypes.c_int64),
        ("B", ctypes.c_void_p),
        ("ldb", ctypes.c_int64),
        ("X", ctypes.c_void_p),
        ("ldx", ctypes.c_int64),
        ("sweep_dtype", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("rel_tol", ctypes.c_double),
    ]


class ServeStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("rejected", ctypes.c_uint64),
        ("failed", ctypes.c_uint64),
        ("active", ctypes.c_uint64),
        ("queued", ctypes.c_uint64),
        ("hbm_in_use", ctypes.c_uint64),
        ("hbm_peak", ctypes.c_uint64),
        ("steps", ctypes.c_uint64),
        ("solves_per_s", ctypes.c_double),
        ("p50_ms", ctypes.c_double),
        ("p99_ms", ctypes.c_double),
        ("p50_device_ms", ctypes.c_double),
        ("p99_device_ms", ctypes.c_double),
        ("elapsed_s", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load():
    """Load libjacobi.so (built by paper_1403_5805_amd.build / __graft_entry__.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libjacobi.so not found at {LIB_PATH}: build it with "
            "`python -m paper_1403_5805_amd.build` (there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.jacobi_options_default.restype = None
    lib.jacobi_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.jacobi_ctx_create.restype = i32
    lib.jacobi_ctx_create.argtypes = [i32, ctypes.POINTER(vp)]
    lib.jacobi_ctx_destroy.restype = i32
    lib.jacobi_ctx_destroy.argtypes = [vp]
    lib.jacobi_solve.restype = i32
    lib.jacobi_solve.argtypes = [vp, i64, i64, i32, vp, i64, vp, i64, vp, vp, i64,
                                 ctypes.POINTER(Options), vp, ctypes.POINTER(Info)]
    lib.jacobi_status_string.restype = ctypes.c_char_p
    lib.jacobi_status_string.argtypes = [i32]
    lib.jacobi_last_error.restype = ctypes.c_char_p
    lib.jacobi_last_error.argtypes = []
    if hasattr(lib, "jacobi_solve_batched"):
        lib.jacobi_solve_batched.restype = i32
        lib.jacobi_solve_batched.argtypes = [vp, i32, ctypes.POINTER(System), i32,
                                             ctypes.POINTER(Options), vp, ctypes.POINTER(Info)]
    if hasattr(lib, "jacobi_serve_create"):
        lib.jacobi_serve_config_default.restype = None
        lib.jacobi_serve_config_default.argtypes = [ctypes.POINTER(ServeConfig)]
        lib.jacobi_serve_create.restype = i32
        lib.jacobi_serve_create.argtypes = [ctypes.POINTER(ServeConfig), ctypes.POINTER(vp)]
        lib.jacobi_serve_submit.restype = i32
        lib.jacobi_serve_submit.argtypes = [vp, ctypes.POINTER(Request),
                                            ctypes.POINTER(ctypes.c_uint64)]
        lib.jacobi_serve_poll.restype = i32
        lib.jacobi_serve_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Info)]
        lib.jacobi_serve_wait.restype = i32
        lib.jacobi_serve_wait.argtypes = [vp, ctypes.c_uint64, i64, ctypes.POINTER(Info)]
        lib.jacobi_serve_stats_get.restype = i32
        lib.jacobi_serve_stats_get.argtypes = [vp, ctypes.POINTER(ServeStats)]
        lib.jacobi_serve_destroy.restype = i32
        lib.jacobi_serve_destroy.argtypes = [vp]
    lib.jacobi_solve_noalloc.restype = i32
    lib.jacobi_solve_noalloc.argtypes = [i64, i64, i32, vp, i64, vp, i64, vp, vp, i64,
                                         ctypes.POINTER(Options), vp, ctypes.POINTER(Info)]
    lib.jacobi_shutdown.restype = i32
    lib.jacobi_shutdown.argtypes = []
    lib.jacobi_matrix_create.restype = i32
    lib.jacobi_matrix_create.argtypes = [vp, i64, i32, vp, i64, i32, vp, ctypes.POINTER(vp)]
    lib.jacobi_solve_prepared.restype = i32
    lib.jacobi_solve_prepared.argtypes = [vp, i64, vp, i64, vp, vp, i64,
                                          ctypes.POINTER(Options), vp, ctypes.POINTER(Info)]
    lib.jacobi_matrix_destroy.restype = i32
    lib.jacobi_matrix_destroy.argtypes = [vp]
    lib.jacobi_stream_probe.restype = i32
    lib.jacobi_stream_probe.argtypes = [vp, i64, i32, vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(i32)]
    _lib = lib
    atexit.register(_shutdown)
    return lib


# Servers and contexts still open at interpreter exit.  They are closed, and
# the library's default contexts released, by an exit hook that runs before
# the HIP runtime is torn down (Python's exit hooks run before the C
# library's), so no device memory, event or worker thread outlives it.
_open_handles: "weakref.WeakSet" = weakref.WeakSet()


def track(obj) -> None:
    """Register an object with a close() method for the exit hook."""
    _open_handles.add(obj)


def _shutdown() -> None:
    for obj in list(_open_handles):
        try:
            obj.close()
        except Exception:
            pass
    if _lib is not None:
        _lib.jacobi_shutdown()
