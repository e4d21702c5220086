"""FP64 CPU oracle for structured inverted-file spherical k-means.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU path: the arithmetic lives in ``sivf_oracle.c`` (plain C, FP64,
``-ffp-contract=off``) and this module only marshals numpy arrays into it and
writes out the Lloyd loop of Alg. 1 with the SIVF bookkeeping of Alg. 4/5.

Pinned by ``tests/test_oracle_*.py`` against exact rational brute force,
Euclidean cross-checks, dense numpy means, closed forms, the ICP
filtered == unfiltered invariant, monotone objective and special cases.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sivf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(path):
    """Load a built oracle library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    i32, i64, f64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    ci = ctypes.c_int
    lib.orc_assign.argtypes = [i64, i64, vp, vp, vp, ci, i32, vp, vp, vp, vp, i64, ci, vp, vp, vp,
                               ci, vp, vp, vp, vp]
    lib.orc_assign.restype = ci
    lib.orc_pair_sims.argtypes = [i64, vp, vp, vp, ci, vp, vp, vp, vp, vp, i64, vp]
    lib.orc_pair_sims.restype = ci
    lib.orc_update.argtypes = [i64, i64, vp, vp, vp, ci, i32, vp, vp, vp, vp, vp, vp, vp, i64, vp]
    lib.orc_update.restype = i64
    lib.orc_build_ivf.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_build_ivf.restype = ci
    lib.orc_multadds.argtypes = [i64, vp, vp, vp, vp, vp, ci, vp, vp, ci, vp, vp, vp]
    lib.orc_multadds.restype = ci
    lib.orc_soft_forward.argtypes = [i64, vp, vp, vp, ci, i32, vp, f64, vp, i64, vp]
    lib.orc_soft_forward.restype = ci
    lib.orc_soft_backward.argtypes = [i64, vp, vp, vp, ci, i32, vp, f64, f64, vp, i64, vp, vp, vp]
    lib.orc_soft_backward.restype = ci
    lib.orc_num_threads.restype = ci
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _bind(_LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _xval(corpus):
    v = corpus.val
    if v.dtype == np.float64:
        return v, 1
    if v.dtype == np.float32:
        return v, 0
    raise ValueError("corpus values must be float32 or float64")


def num_threads() -> int:
    return int(_load().orc_num_threads())


@dataclass
class Centroids:
    """k x d centroid set as CSR (ascending columns), FP64 values."""
    k: int
    d: int
    ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    def dense(self) -> np.ndarray:
        out = np.zeros((self.k, self.d), dtype=np.float64)
        rows = np.repeat(np.arange(self.k), np.diff(self.ptr))
        out[rows, self.col] = self.val
        return out


@dataclass
class Ivf:
    """Structured inverted file in the paper's layout: per term, moving then invariant."""
    term_ptr: np.ndarray
    split: np.ndarray
    cid: np.ndarray
    val: np.ndarray


def init_centroids(corpus, ids) -> Centroids:
    """mu_j^(0) = x_{ids[j]} as stored (widened to f64), j in draw order."""
    ids = np.asarray(ids, dtype=np.int64)
    lens = corpus.row_ptr[ids + 1] - corpus.row_ptr[ids]
    ptr = np.zeros(len(ids) + 1, dtype=np.int64)
    np.cumsum(lens, out=ptr[1:])
    col = np.concatenate([corpus.col[corpus.row_ptr[i]:corpus.row_ptr[i + 1]] for i in ids]) \
        if len(ids) else np.zeros(0, np.int32)
    val = np.concatenate([corpus.val[corpus.row_ptr[i]:corpus.row_ptr[i + 1]].astype(np.float64)
                          for i in ids]) if len(ids) else np.zeros(0)
    return Centroids(len(ids), corpus.d, ptr, np.ascontiguousarray(col, np.int32),
                     np.ascontiguousarray(val, np.float64))


def assign(corpus, cents: Centroids, rows=None, icp=False, lam_prev=None, a_prev=None, own_prev=None,
           relaxed=False, want_branch=False):
    """Returns (a, own, top2) for the selected rows (all rows if None), and the
    branch each row took (0 all centroids, 1 ICP, 2 relaxed ICP) if want_branch."""
    lib = _load()
    val, f64 = _xval(corpus)
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = corpus.n if rows_a is None else len(rows_a)
    a = np.empty(m, dtype=np.int32)
    own = np.empty(m, dtype=np.float64)
    top2 = np.empty((m, 2), dtype=np.float64)
    lam_prev = None if lam_prev is None else np.ascontiguousarray(lam_prev, np.uint8)
    a_prev = None if a_prev is None else np.ascontiguousarray(a_prev, np.int32)
    own_prev = None if own_prev is None else np.ascontiguousarray(own_prev, np.float64)
    branch = np.empty(m, dtype=np.uint8)
    rc = lib.orc_assign(corpus.n, corpus.d, _p(corpus.row_ptr), _p(corpus.col), _p(val), f64, cents.k,
                        _p(cents.ptr), _p(cents.col), _p(cents.val), _p(rows_a), m, 1 if icp else 0,
                        _p(lam_prev), _p(a_prev), _p(own_prev), 1 if relaxed else 0, _p(a), _p(own), _p(top2),
                        _p(branch))
    if rc != 0:
        raise RuntimeError("orc_assign failed (%d)" % rc)
    return (a, own, top2, branch) if want_branch else (a, own, top2)


def pair_sims(corpus, cents: Centroids, obj, cen) -> np.ndarray:
    lib = _load()
    val, f64 = _xval(corpus)
    obj = np.ascontiguousarray(obj, dtype=np.int64)
    cen = np.ascontiguousarray(cen, dtype=np.int32)
    out = np.empty(len(obj), dtype=np.float64)
    lib.orc_pair_sims(corpus.d, _p(corpus.row_ptr), _p(corpus.col), _p(val), f64, _p(cents.ptr),
                      _p(cents.col), _p(cents.val), _p(obj), _p(cen), len(obj), _p(out))
    return out


def update(corpus, a, prev: Centroids):
    """Returns (new centroids, cluster sizes)."""
    lib = _load()
    val, f64 = _xval(corpus)
    a = np.ascontiguousarray(a, dtype=np.int32)
    k = prev.k
    cap = max(1, min(corpus.nnz + len(prev.val), k * corpus.d))
    while True:
        ptr = np.empty(k + 1, dtype=np.int64)
        col = np.empty(cap, dtype=np.int32)
        v = np.empty(cap, dtype=np.float64)
        counts = np.empty(k, dtype=np.int32)
        rc = lib.orc_update(corpus.n, corpus.d, _p(corpus.row_ptr), _p(corpus.col), _p(val), f64, k,
                            _p(a), _p(prev.ptr), _p(prev.col), _p(prev.val), _p(ptr), _p(col), _p(v),
                            cap, _p(counts))
        if rc == 0:
            nnz = int(ptr[-1])
            return Centroids(k, corpus.d, ptr, col[:nnz].copy(), v[:nnz].copy()), counts
        if rc < 0:
            raise RuntimeError("orc_update failed (%d)" % rc)
        cap = int(rc)


def build_ivf(cents: Centroids, lam=None) -> Ivf:
    lib = _load()
    nnz = len(cents.val)
    tp = np.empty(cents.d + 1, dtype=np.int64)
    sp = np.empty(cents.d, dtype=np.int32)
    cid = np.empty(max(nnz, 1), dtype=np.int32)
    uv = np.empty(max(nnz, 1), dtype=np.float64)
    lam = None if lam is None else np.ascontiguousarray(lam, np.uint8)
    rc = lib.orc_build_ivf(cents.k, cents.d, _p(cents.ptr), _p(cents.col), _p(cents.val), _p(lam),
                           _p(tp), _p(sp), _p(cid), _p(uv))
    if rc != 0:
        raise RuntimeError("orc_build_ivf failed (%d)" % rc)
    return Ivf(tp, sp, cid[:nnz], uv[:nnz])


MODE_SIVF, MODE_CBICP, MODE_IVF = 0, 1, 2


def multadds(corpus, ivf: Ivf, icp=False, lam_prev=None, a_prev=None, mode=MODE_SIVF, per_row=False, branch=None):
    lib = _load()
    total = np.zeros(1, dtype=np.int64)
    pr = np.empty(corpus.n, dtype=np.int64) if per_row else None
    lam_prev = None if lam_prev is None else np.ascontiguousarray(lam_prev, np.uint8)
    a_prev = None if a_prev is None else np.ascontiguousarray(a_prev, np.int32)
    cid = ivf.cid if len(ivf.cid) else np.zeros(1, np.int32)
    branch = None if branch is None else np.ascontiguousarray(branch, np.uint8)
    lib.orc_multadds(corpus.n, _p(corpus.row_ptr), _p(corpus.col), _p(ivf.term_ptr), _p(ivf.split),
                     _p(cid), 1 if icp else 0, _p(lam_prev), _p(a_prev), mode, _p(branch), _p(pr), _p(total))
    return (int(total[0]), pr) if per_row else int(total[0])


def mark_invariant(a_old, a_new, k, first: bool):
    """lambda_j = 1 iff cluster j has the same members before and after (Alg. 4, mark
    invariant clusters); all zero on the first iteration.  Returns (lam, moved)."""
    a_new = np.asarray(a_new)
    if first:
        return np.zeros(k, dtype=np.uint8), int(len(a_new))
    a_old = np.asarray(a_old)
    mv = a_old != a_new
    changed = np.zeros(k, dtype=bool)
    changed[a_old[mv]] = True
    changed[a_new[mv]] = True
    return (~changed).astype(np.uint8), int(mv.sum())


def objective(corpus, cents: Centroids, a) -> float:
    """F = sum_i rho_{i,a_i}, the spherical k-means objective (summed exactly with fsum)."""
    sims = pair_sims(corpus, cents, np.arange(corpus.n), a)
    return math.fsum(sims.tolist())


@dataclass
class LloydTrace:
    assign: list = field(default_factory=list)       # a^[r], r = 1..R
    own: list = field(default_factory=list)          # rho_{i,a_i} cached per iteration
    lam: list = field(default_factory=list)          # lambda^[r]
    moved: list = field(default_factory=list)
    multadds: list = field(default_factory=list)     # SIVF posting mult-adds of assignment step r
    branch: list = field(default_factory=list)       # per object: 0 all centroids, 1 ICP, 2 relaxed ICP
    centroids: list = field(default_factory=list)    # mu^[r-1] used by assignment r (if keep_centroids)
    final: Centroids | None = None                   # centroids after the last update
    iters: int = 0
    converged: bool = False


@dataclass
class LloydState:
    """Where a Lloyd run stands after the update of iteration r (Alg. 1): the
    next assignment step is r + 1 and reads these values.

    cents: mu^[r]; a: a^[r]; lam: lambda^[r] (from a^[r-1] and a^[r]);
    own: rho of each object to mu^[r]_{a_i}.  For an object whose cluster is
    invariant (lam[a_i] = 1) that centroid did not change, so this is the
    cached own similarity the ICP branch starts from; the other objects' values
    are not read in the SIVF, IVF and IVF-CBICP modes.
    """
    r: int
    cents: Centroids
    a: np.ndarray
    own: np.ndarray
    lam: np.ndarray


def resume_state(corpus, cents: Centroids, a_prev, a_prev2=None, r=None) -> LloydState:
    """State to continue a run from its last two assignments and the centroids
    the last update produced (Alg. 1 restarted between iterations):
    lambda^[r] from (a^[r-1], a^[r]) -- all zero when a_prev2 is None, i.e.
    r = 1 -- and the own similarities rho(x_i, mu^[r]_{a_i}) recomputed with
    the same fold as the assignment step."""
    a_prev = np.ascontiguousarray(a_prev, np.int32)
    lam, _ = mark_invariant(a_prev2, a_prev, cents.k, first=a_prev2 is None)
    own = pair_sims(corpus, cents, np.arange(corpus.n), a_prev)
    return LloydState(r if r is not None else (1 if a_prev2 is None else 2), cents, a_prev, own, lam)


def lloyd(corpus, k, ids, max_iter, icp=True, keep_centroids=False, count_multadds=True, relaxed=False,
          start: LloydState | None = None, on_iter=None):
    """Spherical Lloyd with SIVF bookkeeping (Alg. 1 driver around Alg. 4 / Alg. 5).

    Iteration r: assignment against mu^[r-1] (ICP mode from r >= 2 when icp;
    with relaxed, also objects whose own centroid moved without their
    similarity to it decreasing compare moving centroids only), invariance
    flags lambda^[r], stop after an assignment step r >= 2 that moved nothing,
    else update to mu^[r].

    start: continue after iteration start.r instead of starting from the
    seeded objects (ids is then unused); the trace lists iterations
    start.r + 1 .. in order.  Relaxed ICP needs the similarities to the
    previous centroids, which a restart does not have, so it cannot resume.
    on_iter(info): called after each assignment step with a dict holding r, a,
    own, lam, moved, multadds, branch and, once the update ran, cents (mu^[r]).
    """
    if start is not None and relaxed:
        raise ValueError("relaxed ICP cannot resume from a saved state")
    if start is None:
        cents = init_centroids(corpus, ids)
        a_prev = own_prev = lam_prev = None
        r0 = 0
    else:
        cents, a_prev, own_prev, lam_prev, r0 = start.cents, start.a, start.own, start.lam, start.r
    tr = LloydTrace()
    for r in range(r0 + 1, max_iter + 1):
        if keep_centroids:
            tr.centroids.append(cents)
        use_icp = icp and r >= 2
        a, own, _, branch = assign(corpus, cents, icp=use_icp, lam_prev=lam_prev, a_prev=a_prev, own_prev=own_prev,
                                   relaxed=relaxed, want_branch=True)
        tr.branch.append(branch)
        m = None
        if count_multadds:
            ivf = build_ivf(cents, lam_prev)
            m = multadds(corpus, ivf, icp=use_icp, lam_prev=lam_prev, a_prev=a_prev,
                         branch=branch if use_icp else None)
            tr.multadds.append(m)
            del ivf
        lam, moved = mark_invariant(a_prev, a, k, first=(r == 1))
        tr.assign.append(a)
        tr.own.append(own)
        tr.lam.append(lam)
        tr.moved.append(moved)
        tr.iters = r
        info = dict(r=r, a=a, own=own, lam=lam, moved=moved, multadds=m, branch=branch, cents=None)
        if r >= 2 and moved == 0:
            tr.converged = True
            if on_iter:
                on_iter(info)
            break
        cents, _ = update(corpus, a, cents)
        a_prev, own_prev, lam_prev = a, own, lam
        if on_iter:
            info["cents"] = cents
            on_iter(info)
    tr.final = cents
    return tr


def soft_forward(corpus, C: np.ndarray, tau: float, rows=None):
    """lse_i for the selected rows; loss = -fsum(lse)."""
    lib = _load()
    val, f64 = _xval(corpus)
    C = np.ascontiguousarray(C, dtype=np.float64)
    rows = np.arange(corpus.n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, np.int64)
    lse = np.empty(len(rows), dtype=np.float64)
    lib.orc_soft_forward(corpus.d, _p(corpus.row_ptr), _p(corpus.col), _p(val), f64, C.shape[0], _p(C),
                         float(tau), _p(rows), len(rows), _p(lse))
    return lse


def soft_backward(corpus, C: np.ndarray, tau: float, g: float, lse, rows=None, want_dc=True, want_dx=True):
    """(dC dense k x d or None, dX on X's nonzeros of the selected rows or None)."""
    lib = _load()
    val, f64 = _xval(corpus)
    C = np.ascontiguousarray(C, dtype=np.float64)
    rows = np.arange(corpus.n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, np.int64)
    lse = np.ascontiguousarray(lse, dtype=np.float64)
    dx = np.zeros(corpus.nnz, dtype=np.float64) if want_dx else None
    dc = np.zeros(C.shape, dtype=np.float64) if want_dc else None
    lib.orc_soft_backward(corpus.d, _p(corpus.row_ptr), _p(corpus.col), _p(val), f64, C.shape[0], _p(C),
                          float(tau), float(g), _p(rows), len(rows), _p(lse), _p(dx), _p(dc))
    return dc, dx
