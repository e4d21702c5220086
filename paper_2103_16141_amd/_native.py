"""ctypes declarations for libsivf.so (include/sivf.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsivf.so")

SIVF_OK = 0
STATUS = {0: "SIVF_OK", -1: "SIVF_E_INVALID", -2: "SIVF_E_SHAPE", -3: "SIVF_E_UNSORTED", -4: "SIVF_E_RANGE",
          -5: "SIVF_E_NONFINITE", -6: "SIVF_E_NOMEM", -7: "SIVF_E_HIP", -8: "SIVF_E_UNSUPPORTED"}
SIVF_F32, SIVF_F64, SIVF_BF16 = 0, 1, 2
SIVF_MODE_SIVF, SIVF_MODE_IVF, SIVF_MODE_CBICP, SIVF_MODE_RELAXED = 0, 1, 2, 3


class sivf_csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("val_dtype", ctypes.c_int)]


class sivf_options(ctypes.Structure):
    _fields_ = [("posting_dtype", ctypes.c_int), ("filter_mode", ctypes.c_int32), ("k_tile", ctypes.c_int32),
                ("certify", ctypes.c_int32), ("workspace_cap_bytes", ctypes.c_size_t),
                ("head_density", ctypes.c_float), ("tiles_per_launch", ctypes.c_int32),
                ("exact_objective", ctypes.c_int32)]


class sivf_iter_stats(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("n_invariant", ctypes.c_int32), ("multadds", ctypes.c_int64),
                ("moved", ctypes.c_int64), ("icp_objects", ctypes.c_int64), ("rescored_objects", ctypes.c_int64),
                ("rescored_candidates", ctypes.c_int64), ("full_rescored", ctypes.c_int64),
                ("objective_fast", ctypes.c_double), ("t_walk_ms", ctypes.c_float),
                ("t_assign_ms", ctypes.c_float), ("t_update_ms", ctypes.c_float), ("head_rows", ctypes.c_int64),
                ("relaxed_objects", ctypes.c_int64), ("objective", ctypes.c_double), ("walk_bytes", ctypes.c_int64),
                ("walk_wide_bytes", ctypes.c_int64),
                ("walk_launches", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class SivfError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__("%s: %s" % (self.name, msg))


_lib = None


def load(path: str = LIB_PATH):
    """Load libsivf.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libsivf.so not built at %s: run `python -m paper_2103_16141_amd.build`" % path)
    lib = ctypes.CDLL(path)
    P, vp, i32, i64, f32 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    st = ctypes.c_int
    csr_p = P(sivf_csr)
    stats_p = P(sivf_iter_stats)
    sig = {
        "sivf_default_options": ([P(sivf_options)], st),
        "sivf_create": ([P(vp), ctypes.c_int, vp, P(sivf_options)], st),
        "sivf_destroy": ([vp], st),
        "sivf_last_error": ([vp], ctypes.c_char_p),
        "sivf_validate_csr": ([vp, csr_p], st),
        "sivf_init_centroids": ([vp, csr_p, i32, vp, P(vp)], st),
        "sivf_build_centroid_ivf": ([vp, csr_p, vp, P(vp)], st),
        "sivf_ivf_free": ([vp, vp], st),
        "sivf_ivf_sizes": ([vp, vp, P(i32), P(i64), P(i64), P(i32), P(i32)], st),
        "sivf_ivf_export": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, vp], st),
        "sivf_assign": ([vp, csr_p, vp, i32, vp, vp, vp, vp, stats_p], st),
        "sivf_assign_noalloc": ([vp, csr_p, vp, i32, vp, vp, vp, vp, stats_p], st),
        "sivf_update": ([vp, csr_p, vp, vp, vp, stats_p], st),
        "sivf_run_lloyd": ([vp, csr_p, i32, vp, i32, vp, vp, P(vp), stats_p, P(i32)], st),
        "sivf_resume": ([vp, csr_p, csr_p, vp, vp, P(vp), vp, vp], st),
        "sivf_soft_assign_fwd": ([vp, csr_p, vp, i32, f32, vp, P(ctypes.c_double)], st),
        "sivf_soft_assign_bwd": ([vp, csr_p, vp, i32, f32, vp, f32, vp, vp], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(ctx, status):
    if status != SIVF_OK:
        msg = load().sivf_last_error(ctx) if ctx else b""
        raise SivfError(status, (msg or b"").decode(errors="replace"))
