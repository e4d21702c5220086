"""Shared helpers for the GPU parity tests: drive the C ABI one Lloyd step at a
time and compare every step against the FP64 oracle."""
import sys

import numpy as np
import torch

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def centroids_from_export(ex, k, d):
    ptr = ex["c_ptr"].cpu().numpy()
    return oracle.Centroids(k, d, ptr, ex["c_col"].cpu().numpy()[: ptr[-1]], ex["c_val"].cpu().numpy()[: ptr[-1]])


def assert_centroids_equal(gpu: oracle.Centroids, ref: oracle.Centroids, what=""):
    assert np.array_equal(gpu.ptr, ref.ptr), "centroid sizes differ %s" % what
    assert np.array_equal(gpu.col, ref.col), "centroid supports differ %s" % what
    if not np.array_equal(gpu.val.view(np.uint64), ref.val.view(np.uint64)):
        rel = np.max(np.abs(gpu.val - ref.val) / np.maximum(np.abs(ref.val), 1e-300))
        n_diff = int(np.sum(gpu.val != ref.val))
        raise AssertionError("centroid values differ in %d entries (max rel %.3g) %s" % (n_diff, rel, what))


def lloyd_parity(ctx, X, corpus, k, ids, max_iter, icp=True, mode="sivf", check_centroids=True,
                 check_ivf_every=1):
    """Run GPU and oracle Lloyd side by side; assert identical trajectories."""
    from paper_2103_16141_amd.api import Lloyd
    tr = oracle.lloyd(corpus, k, ids, max_iter, icp=icp, keep_centroids=True, relaxed=(mode == "relaxed"))
    L = Lloyd(ctx, X, k, ids)
    gpu_stats = []
    for r in range(1, tr.iters + 1):
        st = L.assign()
        gpu_stats.append(st)
        a = L.a.cpu().numpy()
        ref = tr.assign[r - 1]
        nbad = int((a != ref).sum())
        assert nbad == 0, "iteration %d: %d assignments differ (first at %s)" % (r, nbad, np.nonzero(a != ref)[0][:5])
        assert np.array_equal(L.lam.cpu().numpy(), tr.lam[r - 1]), "iteration %d: flags differ" % r
        assert st["moved"] == tr.moved[r - 1]
        if mode == "ivf":
            ivf = oracle.build_ivf(tr.centroids[r - 1], tr.lam[r - 2] if r >= 2 else None)
            m_ref = oracle.multadds(corpus, ivf, icp=False, mode=oracle.MODE_IVF)
        else:
            m_ref = tr.multadds[r - 1]
        assert st["multadds"] == m_ref, "iteration %d: multadds %d vs %d" % (r, st["multadds"], m_ref)
        # own similarity: the fast-pass value (or the FP64 re-score rounded to
        # FP32), within the certificate's relative bound: 2^-24 (+ fold) for FP32
        # postings, 2^-8 + 2^-24 (+ fold) for BF16 postings
        own = L.own.cpu().numpy().astype(np.float64)
        rel = np.abs(own - tr.own[r - 1]) / np.maximum(np.abs(tr.own[r - 1]), 1e-30)
        tol = 4.0e-3 if ctx.opt.posting_dtype == 2 else 1e-5
        assert rel.max() < tol, "iteration %d: own similarity off by %.3g" % (r, rel.max())
        if r == tr.iters:
            break
        L.update()
        if check_centroids and (r % check_ivf_every == 0 or r + 1 == tr.iters):
            ex = L.ivf.export()
            ref_c = tr.centroids[r]
            gpu_c = centroids_from_export(ex, k, corpus.d)
            assert_centroids_equal(gpu_c, ref_c, "after update %d" % r)
            # structured file in the paper's layout
            ivf_ref = oracle.build_ivf(ref_c, tr.lam[r - 1])
            assert np.array_equal(ex["term_ptr"].cpu().numpy(), ivf_ref.term_ptr)
            assert np.array_equal(ex["split"].cpu().numpy(), ivf_ref.split)
            assert np.array_equal(ex["p_cid"].cpu().numpy(), ivf_ref.cid)
            assert np.array_equal(ex["p_val"].cpu().numpy(), ivf_ref.val)
            assert np.array_equal(ex["lam"].cpu().numpy(), tr.lam[r - 1])
    return tr, gpu_stats


def device():
    return torch.device("cuda", 0)
