"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds input generation only (no clustering arithmetic).  The heavy lifting is
``synth.c`` (SplitMix64 counter-based streams, OpenMP over rows); this module
compiles it with gcc on demand and wraps it with ctypes.

Workloads mirror the shapes of the paper's corpora (Section 5.1: PubMed,
L2-normalised tf-idf, ~59 nonzeros/row, D ~ 141k; NYT, D ~ 496k, ~226
nonzeros/row).  Those corpora are not available, so seeded Zipf/Poisson/
lognormal rows stand in for them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile synth.c into libsynth.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, u64, f64, vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
        lib.synth_row_counts.argtypes = [i64, i64, f64, u64, vp]
        lib.synth_row_counts.restype = ctypes.c_int
        lib.synth_fill.argtypes = [i64, i64, f64, u64, vp, vp, vp, ctypes.c_int]
        lib.synth_fill.restype = ctypes.c_int
        lib.synth_dense_centroids.argtypes = [i64, ctypes.c_int32, vp, vp, vp, vp, f64, u64, vp]
        lib.synth_dense_centroids.restype = ctypes.c_int
        lib.synth_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Corpus:
    """CSR matrix: row_ptr int64[N+1], col int32[nnz] (ascending per row), val f32|f64[nnz]."""
    n: int
    d: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def make_corpus(n: int, d: int, lam: float, zipf_s: float, dtype=np.float32, seed: int = 0) -> Corpus:
    """Generate N rows over D terms (recipe in synth.c's header)."""
    lib = _load()
    counts = np.empty(n, dtype=np.int64)
    rc = lib.synth_row_counts(n, d, float(lam), int(seed), _ptr(counts))
    if rc != 0:
        raise ValueError("synth_row_counts failed (%d)" % rc)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    dtype = np.dtype(dtype)
    if dtype not in (np.dtype(np.float32), np.dtype(np.float64)):
        raise ValueError("dtype must be float32 or float64")
    val = np.empty(nnz, dtype=dtype)
    rc = lib.synth_fill(n, d, float(zipf_s), int(seed), _ptr(row_ptr), _ptr(col), _ptr(val),
                        1 if dtype == np.float64 else 0)
    if rc != 0:
        raise RuntimeError("synth_fill failed (%d)" % rc)
    return Corpus(n, d, row_ptr, col, val)


def init_ids(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct object ids drawn uniformly by seed, in draw order (int32)."""
    if not (1 <= k <= n):
        raise ValueError("need 1 <= k <= n")
    return np.random.Generator(np.random.PCG64(seed)).choice(n, k, replace=False).astype(np.int32)


def dense_centroids(corpus: Corpus, ids: np.ndarray, noise: float = 1e-3, seed: int = 0) -> np.ndarray:
    """Dense k x D f32 rows: normalise(dense(x_id) + noise*|N(0,1)|).  Soft-assignment workload."""
    if corpus.val.dtype != np.float32:
        raise ValueError("dense_centroids expects an f32 corpus")
    lib = _load()
    ids64 = np.ascontiguousarray(ids, dtype=np.int64)
    out = np.empty((len(ids64), corpus.d), dtype=np.float32)
    lib.synth_dense_centroids(corpus.d, len(ids64), _ptr(corpus.row_ptr), _ptr(corpus.col),
                              _ptr(corpus.val), _ptr(ids64), float(noise), int(seed), _ptr(out))
    return out


def num_threads() -> int:
    return int(_load().synth_num_threads())


# Workloads (sizes of the paper-shaped configurations).  data_seed = 16141 + c,
# init_seed = 2103 + c for configuration number c.
WORKLOADS = {
    "small-f64": dict(n=10_000, d=5_000, lam=50, zipf_s=1.0, dtype=np.float64, k=100, iters=10, c=1),
    "1m-f32": dict(n=1_000_000, d=100_000, lam=100, zipf_s=1.1, dtype=np.float32, k=1_000, iters=50, c=2),
    "8m-f32": dict(n=8_000_000, d=140_000, lam=90, zipf_s=1.1, dtype=np.float32, k=10_000, iters=30, c=3),
    "8m-bf16-k20k": dict(n=8_000_000, d=140_000, lam=90, zipf_s=1.1, dtype=np.float32, k=20_000, iters=30, c=4),
    "soft-262k": dict(n=262_144, d=100_000, lam=100, zipf_s=1.1, dtype=np.float32, k=4_096, iters=1, c=5),
    # second corpus shape the paper uses (NYT articles: N, D and mean nonzeros per row)
    "nyt-f32": dict(n=1_285_944, d=495_714, lam=226, zipf_s=1.1, dtype=np.float32, k=10_000, iters=30, c=6),
}


def workload(name: str, **override):
    w = dict(WORKLOADS[name])
    w.update(override)
    corpus = make_corpus(w["n"], w["d"], w["lam"], w["zipf_s"], w["dtype"], seed=16141 + w["c"])
    ids = init_ids(w["n"], w["k"], seed=2103 + w["c"])
    return corpus, ids, w
