"""The assignment entry point that allocates nothing (sivf_assign_noalloc)
against sivf_assign: same inputs, same results, bit for bit, on two calls in
a row -- the second with fewer objects, so it runs on what the first left in
the shared scratch block -- and on an ICP step; a request larger than the
block is refused before anything is written.  The ctx it runs on may hold no
device memory at all (workspace cap of one byte), so any allocation it
attempted would fail."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import device, log

pytestmark = pytest.mark.gpu


def _ctx(**kw):
    from paper_2103_16141_amd.api import Context
    return Context(0, **kw)


def _X(c):
    from paper_2103_16141_amd.api import DeviceCsr
    return DeviceCsr.from_corpus(c, device())


def _rows(c, lo, hi):
    return synth.Corpus(hi - lo, c.d, c.row_ptr[lo:hi + 1] - c.row_ptr[lo], c.col[c.row_ptr[lo]:c.row_ptr[hi]],
                        c.val[c.row_ptr[lo]:c.row_ptr[hi]])


def _both(ref_ctx, na_ctx, X, ivf, it, a0, own0, k, own64_0=None):
    out = []
    for ctx, call in ((ref_ctx, "assign"), (na_ctx, "assign_noalloc")):
        a, own = a0.clone(), own0.clone()
        lam = torch.full((k,), 7, dtype=torch.uint8, device=device())
        own64 = None if own64_0 is None else own64_0.clone()
        st = getattr(ctx, call)(X, ivf, it, a, own, lam, own64=own64)
        out.append((a.cpu().numpy(), own.cpu().numpy(), lam.cpu().numpy(), st,
                    None if own64 is None else own64.cpu().numpy()))
    (a1, o1, l1, s1, e1), (a2, o2, l2, s2, e2) = out
    assert np.array_equal(a1, a2)
    assert np.array_equal(o1.view(np.uint32), o2.view(np.uint32))
    assert np.array_equal(l1, l2)
    for key in ("multadds", "moved", "icp_objects", "rescored_objects", "full_rescored", "n_invariant",
                "relaxed_objects", "walk_bytes"):
        assert s1[key] == s2[key], key
    if e1 is not None:
        assert np.array_equal(e1.view(np.uint64), e2.view(np.uint64))
    return a1, o1, l1, s1


@pytest.mark.parametrize("posting,mode", [("fp32", "sivf"), ("bf16", "relaxed")])
def test_noalloc_assign_equals_assign(posting, mode):
    log("no-alloc assign vs assign, %s postings, filter %s" % (posting, mode))
    c = synth.make_corpus(24000, 5000, 30, 1.1, np.float32, seed=151)
    k = 300   # three tiles of 128 (the last ragged): per-object state between launches
    ids = synth.init_ids(c.n, k, 51)
    opts = dict(k_tile=128, posting_dtype=posting, filter_mode=mode)
    ref = _ctx(**opts)
    na = _ctx(workspace_cap_bytes=1, **opts)
    X = _X(c)
    ivf = ref.init_centroids(X, k, ids)
    a = torch.zeros(c.n, dtype=torch.int32, device=device())
    own = torch.zeros(c.n, dtype=torch.float32, device=device())
    own64 = torch.zeros(c.n, dtype=torch.float64, device=device()) if mode == "relaxed" else None
    lam = torch.zeros(k, dtype=torch.uint8, device=device())
    # call 1: all objects, iteration 1
    _, _, _, st1 = _both(ref, na, X, ivf, 1, a, own, k, own64)
    assert st1["moved"] == c.n
    # call 2 right after it: fewer objects (the first 9,000 rows), iteration 1
    X2 = _X(_rows(c, 0, 9000))
    _both(ref, na, X2, ivf, 1, a[:9000].clone(), own[:9000].clone(), k,
          None if own64 is None else own64[:9000].clone())
    # ICP steps: the reference state advances with sivf_assign / sivf_update,
    # and each step is also taken through the no-alloc entry point
    ref.assign(X, ivf, 1, a, own, lam, own64=own64)
    for r in (2, 3, 4):
        ref.update(X, a, lam, ivf)
        a_r, _, _, st = _both(ref, na, X, ivf, r, a, own, k, own64)
        ref.assign(X, ivf, r, a, own, lam, own64=own64)
        assert np.array_equal(a.cpu().numpy(), a_r)
    assert st["icp_objects"] > 0
    na.close()
    ref.close()


def test_noalloc_refuses_what_does_not_fit():
    from paper_2103_16141_amd._native import SivfError
    log("no-alloc assign: request above the scratch block")
    c = synth.make_corpus(260000, 2000, 4, 1.1, np.float32, seed=152)
    k = 200
    ctx = _ctx(k_tile=64)
    X = _X(c)
    ivf = ctx.init_centroids(X, k, synth.init_ids(c.n, k, 52))
    a = torch.full((c.n,), 3, dtype=torch.int32, device=device())
    own = torch.full((c.n,), 0.5, dtype=torch.float32, device=device())
    lam = torch.full((k,), 9, dtype=torch.uint8, device=device())
    with pytest.raises(SivfError) as e:
        ctx.assign_noalloc(X, ivf, 1, a, own, lam)
    assert e.value.name == "SIVF_E_UNSUPPORTED" and "scratch" in str(e.value)
    assert bool((a == 3).all()) and bool((own == 0.5).all()) and bool((lam == 9).all())
    # the same request through sivf_assign runs
    ctx.assign(X, ivf, 1, a, own, lam)
    assert int(a.max()) < k
