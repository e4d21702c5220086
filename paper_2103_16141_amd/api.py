"""Python binding of libsivf.so over torch tensors.

Argument marshalling only: every step of the method runs in the HIP kernels
of libsivf.so.  Tensors provide device memory; the context enqueues on the
torch stream that is current when it is created.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@dataclass
class DeviceCsr:
    """A CSR matrix in device memory (objects are rows)."""
    row_ptr: torch.Tensor   # int64 [n+1]
    col: torch.Tensor       # int32 [nnz]
    val: torch.Tensor       # float32 | float64 [nnz]
    n_cols: int

    @property
    def n_rows(self):
        return self.row_ptr.numel() - 1

    @property
    def nnz(self):
        return self.col.numel()

    def struct(self) -> N.sivf_csr:
        dt = {torch.float32: N.SIVF_F32, torch.float64: N.SIVF_F64}.get(self.val.dtype)
        if dt is None:
            raise TypeError("CSR values must be float32 or float64")
        for t, want in ((self.row_ptr, torch.int64), (self.col, torch.int32)):
            if t.dtype != want or not t.is_contiguous():
                raise TypeError("row_ptr must be contiguous int64 and col contiguous int32")
        return N.sivf_csr(self.n_rows, self.n_cols, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                          self.val.data_ptr(), dt)

    @staticmethod
    def from_numpy(row_ptr, col, val, n_cols, device="cuda"):
        return DeviceCsr(torch.from_numpy(np.ascontiguousarray(row_ptr, np.int64)).to(device),
                         torch.from_numpy(np.ascontiguousarray(col, np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(val)).to(device), int(n_cols))

    @staticmethod
    def from_corpus(corpus, device="cuda"):
        return DeviceCsr.from_numpy(corpus.row_ptr, corpus.col, corpus.val, corpus.d, device)


class Ivf:
    """Library-owned centroid set + structured inverted file."""

    def __init__(self, ctx: "Context", handle):
        self.ctx = ctx
        self.handle = handle

    def free(self):
        if self.handle:
            N.check(self.ctx.handle, N.load().sivf_ivf_free(self.ctx.handle, self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                N.load().sivf_ivf_free(self.ctx.handle, self.handle)
        except Exception:
            pass

    def sizes(self):
        k, d, nnz, T, kt = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        N.check(self.ctx.handle, N.load().sivf_ivf_sizes(self.ctx.handle, self.handle, ctypes.byref(k), ctypes.byref(d),
                                                         ctypes.byref(nnz), ctypes.byref(T), ctypes.byref(kt)))
        return dict(k=k.value, d=d.value, nnz=nnz.value, n_tiles=T.value, k_tile=kt.value)

    def export(self):
        """Centroids (CSR, FP64), flags, and the structured file in the paper's layout."""
        sz = self.sizes()
        dev = self.ctx.device
        k, d = sz["k"], sz["d"]
        lib = N.load()
        out = dict(c_ptr=torch.empty(k + 1, dtype=torch.int64, device=dev),
                   lam=torch.empty(k, dtype=torch.uint8, device=dev),
                   term_ptr=torch.empty(d + 1, dtype=torch.int64, device=dev),
                   split=torch.empty(d, dtype=torch.int32, device=dev))
        # first the offsets, then arrays sized from them
        N.check(self.ctx.handle, lib.sivf_ivf_export(self.ctx.handle, self.handle, _ptr(out["c_ptr"]), None, None,
                                                     _ptr(out["lam"]), _ptr(out["term_ptr"]), _ptr(out["split"]),
                                                     None, None))
        nc, npost = int(out["c_ptr"][-1]), int(out["term_ptr"][-1])
        out["c_col"] = torch.empty(max(nc, 1), dtype=torch.int32, device=dev)
        out["c_val"] = torch.empty(max(nc, 1), dtype=torch.float64, device=dev)
        out["p_cid"] = torch.empty(max(npost, 1), dtype=torch.int32, device=dev)
        out["p_val"] = torch.empty(max(npost, 1), dtype=torch.float64, device=dev)
        N.check(self.ctx.handle, lib.sivf_ivf_export(
            self.ctx.handle, self.handle, *[_ptr(out[n]) for n in
                                            ("c_ptr", "c_col", "c_val", "lam", "term_ptr", "split", "p_cid", "p_val")]))
        out["c_col"], out["c_val"] = out["c_col"][:nc], out["c_val"][:nc]
        out["p_cid"], out["p_val"] = out["p_cid"][:npost], out["p_val"][:npost]
        return out

    def centroids(self) -> DeviceCsr:
        """The centroids as a k x D FP64 CSR in device memory (a copy)."""
        ex = self.export()
        return DeviceCsr(ex["c_ptr"], ex["c_col"], ex["c_val"], self.sizes()["d"])


class Context:
    def __init__(self, device=0, posting_dtype="fp32", filter_mode="sivf", k_tile=0, certify=True,
                 workspace_cap_bytes=0, stream=None, head_density=None, tiles_per_launch=None,
                 exact_objective=False):
        lib = N.load()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = self.device.index if self.device.index is not None else 0
        opt = N.sivf_options()
        lib.sivf_default_options(ctypes.byref(opt))
        opt.posting_dtype = {"fp32": N.SIVF_F32, "bf16": N.SIVF_BF16}[posting_dtype]
        opt.filter_mode = {"sivf": N.SIVF_MODE_SIVF, "ivf": N.SIVF_MODE_IVF, "cbicp": N.SIVF_MODE_CBICP,
                           "relaxed": N.SIVF_MODE_RELAXED}[filter_mode]
        opt.k_tile = int(k_tile)
        opt.certify = 1 if certify else 0
        opt.workspace_cap_bytes = int(workspace_cap_bytes)
        if head_density is not None:
            opt.head_density = float(head_density)
        if tiles_per_launch is not None:
            opt.tiles_per_launch = int(tiles_per_launch)
        opt.exact_objective = 1 if exact_objective else 0
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib.sivf_create(ctypes.byref(h), idx, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(opt))
        if rc != N.SIVF_OK:
            raise N.SivfError(rc, "sivf_create failed")
        self.handle = h
        self.opt = opt

    def close(self):
        if self.handle:
            N.load().sivf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        N.check(self.handle, rc)

    def validate(self, X: DeviceCsr):
        s = X.struct()
        self._chk(N.load().sivf_validate_csr(self.handle, ctypes.byref(s)))

    def init_centroids(self, X: DeviceCsr, k: int, init_ids) -> Ivf:
        ids = np.ascontiguousarray(init_ids, dtype=np.int32)
        if len(ids) != k:
            raise ValueError("need k init ids")
        s = X.struct()
        h = ctypes.c_void_p()
        self._chk(N.load().sivf_init_centroids(self.handle, ctypes.byref(s), int(k),
                                               ids.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        return Ivf(self, h)

    def build_centroid_ivf(self, c_ptr, c_col, c_val, n_cols, lam=None) -> Ivf:
        C = DeviceCsr(c_ptr, c_col, c_val, n_cols)
        s = C.struct()
        h = ctypes.c_void_p()
        self._chk(N.load().sivf_build_centroid_ivf(self.handle, ctypes.byref(s), _ptr(lam), ctypes.byref(h)))
        return Ivf(self, h)

    def assign(self, X: DeviceCsr, ivf: Ivf, it: int, a, own, lam_out, stats=True, own64=None):
        s = X.struct()
        st = N.sivf_iter_stats()
        self._chk(N.load().sivf_assign(self.handle, ctypes.byref(s), ivf.handle, int(it), _ptr(a), _ptr(own),
                                       _ptr(own64), _ptr(lam_out), ctypes.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def assign_noalloc(self, X: DeviceCsr, ivf: Ivf, it: int, a, own, lam_out, stats=True, own64=None):
        """assign() through the entry point that allocates no device memory."""
        s = X.struct()
        st = N.sivf_iter_stats()
        self._chk(N.load().sivf_assign_noalloc(self.handle, ctypes.byref(s), ivf.handle, int(it), _ptr(a), _ptr(own),
                                               _ptr(own64), _ptr(lam_out), ctypes.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def update(self, X: DeviceCsr, a, lam, ivf: Ivf, stats=True):
        s = X.struct()
        st = N.sivf_iter_stats()
        self._chk(N.load().sivf_update(self.handle, ctypes.byref(s), _ptr(a), _ptr(lam), ivf.handle,
                                       ctypes.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def resume(self, X: DeviceCsr, centroids: DeviceCsr, a_prev, a_prev2=None):
        """Restart after the update of iteration r-1 from (mu^[r-1], a^[r-1],
        a^[r-2]): returns (file structured by lambda^[r-1], own similarities
        f32[N], exact own similarities f64[N] or None)."""
        n = X.n_rows
        own = torch.empty(n, dtype=torch.float32, device=self.device)
        relaxed = self.opt.filter_mode == N.SIVF_MODE_RELAXED
        own64 = torch.empty(n, dtype=torch.float64, device=self.device) if relaxed else None
        s, c = X.struct(), centroids.struct()
        h = ctypes.c_void_p()
        self._chk(N.load().sivf_resume(self.handle, ctypes.byref(s), ctypes.byref(c), _ptr(a_prev), _ptr(a_prev2),
                                       ctypes.byref(h), _ptr(own), _ptr(own64)))
        return Ivf(self, h), own, own64

    def run_lloyd(self, X: DeviceCsr, k: int, init_ids, max_iter: int, keep_centroids=True):
        ids = np.ascontiguousarray(init_ids, dtype=np.int32)
        a = torch.empty(X.n_rows, dtype=torch.int32, device=self.device)
        own = torch.empty(X.n_rows, dtype=torch.float32, device=self.device)
        stats = (N.sivf_iter_stats * max_iter)()
        done = ctypes.c_int32()
        h = ctypes.c_void_p()
        s = X.struct()
        self._chk(N.load().sivf_run_lloyd(self.handle, ctypes.byref(s), int(k), ids.ctypes.data_as(ctypes.c_void_p),
                                          int(max_iter), _ptr(a), _ptr(own),
                                          ctypes.byref(h) if keep_centroids else None, stats, ctypes.byref(done)))
        ivf = Ivf(self, h) if keep_centroids else None
        return a, own, ivf, [stats[r].as_dict() for r in range(done.value)]

    def soft_assign_fwd(self, X: DeviceCsr, C, tau: float):
        lse = torch.empty(X.n_rows, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        s = X.struct()
        self._chk(N.load().sivf_soft_assign_fwd(self.handle, ctypes.byref(s), _ptr(C), int(C.shape[0]), float(tau),
                                                _ptr(lse), ctypes.byref(loss)))
        return lse, loss.value

    def soft_assign_bwd(self, X: DeviceCsr, C, tau: float, lse, grad_loss: float, want_dc=True, want_dx=True):
        dC = torch.empty_like(C) if want_dc else None
        dX = torch.empty(X.nnz, dtype=torch.float32, device=self.device) if want_dx else None
        s = X.struct()
        self._chk(N.load().sivf_soft_assign_bwd(self.handle, ctypes.byref(s), _ptr(C), int(C.shape[0]), float(tau),
                                                _ptr(lse), float(grad_loss), _ptr(dC), _ptr(dX)))
        return dC, dX


class Lloyd:
    """Step-by-step Lloyd driver over the C ABI (Alg. 1): exposes every iteration's state."""

    def __init__(self, ctx: Context, X: DeviceCsr, k: int, init_ids):
        self.ctx, self.X, self.k = ctx, X, k
        self.ivf = ctx.init_centroids(X, k, init_ids)
        dev = ctx.device
        self.a = torch.zeros(X.n_rows, dtype=torch.int32, device=dev)
        self.own = torch.zeros(X.n_rows, dtype=torch.float32, device=dev)
        self.lam = torch.zeros(k, dtype=torch.uint8, device=dev)
        # exact own similarities, the state of the relaxed ICP filter
        relaxed = ctx.opt.filter_mode == N.SIVF_MODE_RELAXED
        self.own64 = torch.zeros(X.n_rows, dtype=torch.float64, device=dev) if relaxed else None
        self.r = 0

    @classmethod
    def resume(cls, ctx: Context, X: DeviceCsr, centroids: DeviceCsr, r_done: int, a_prev, a_prev2=None):
        """A driver continuing after the update of iteration r_done from the
        centroids mu^[r_done] and the assignments a^[r_done], a^[r_done - 1]."""
        self = cls.__new__(cls)
        self.ctx, self.X, self.k = ctx, X, centroids.n_rows
        self.ivf, self.own, self.own64 = ctx.resume(X, centroids, a_prev, a_prev2)
        self.a = a_prev.clone()
        self.lam = torch.zeros(self.k, dtype=torch.uint8, device=ctx.device)
        self.r = r_done
        return self

    def assign(self):
        self.r += 1
        return self.ctx.assign(self.X, self.ivf, self.r, self.a, self.own, self.lam, own64=self.own64)

    def update(self):
        return self.ctx.update(self.X, self.a, self.lam, self.ivf)


def run_lloyd(X: DeviceCsr, k: int, init_ids, max_iter: int, icp=True, precision="fp32", device=0, **options):
    """Spherical Lloyd from the given seeds (Alg. 1 around Alg. 4 / Alg. 5).

    icp selects the SIVF filter (else plain IVF, every posting), precision the
    posting values ("fp32" or "bf16"); the assignments are the same either way.
    Further keyword options go to Context.  Returns (assign int32[N] on the
    device, centroids as a FP64 DeviceCsr, per-iteration stats)."""
    ctx = Context(device, posting_dtype=precision, filter_mode="sivf" if icp else "ivf", **options)
    a, _, ivf, stats = ctx.run_lloyd(X, k, init_ids, max_iter)
    C = ivf.centroids()
    ivf.free()
    ctx.close()
    return a, C, stats
