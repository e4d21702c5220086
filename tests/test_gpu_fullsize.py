"""Full-size checks in the launch configuration bench.py times.

N = 8M objects, D = 140k, k = 10k, automatic tiles (the headline workload):
  * iterations 1-4 one step at a time against the oracle: from the GPU's
    previous assignment the oracle's update must give the GPU's centroids bit
    for bit, and sampled objects' assignments against them must match
    exactly; flags, moved counts and the exact mult-add count over all
    objects; the structured file after update 2;
  * sampled centroids after update 1 against dense FP64 numpy means (not the
    oracle);
  * SIVF, IVF, relaxed ICP and BF16 postings give identical assignments over
    3 iterations; the SIVF count never exceeds the IVF count, the relaxed
    count never exceeds the SIVF count, BF16 counts equal FP32 counts.
Soft form at its full shape (N = 262,144, D = 100k, k = 4,096): sampled rows'
lse and dX and sampled columns of dC against the oracle; the dC column-sum
identity over all columns.
The precision form at N = 8M, k = 20,000 with BF16 postings: iterations 1-3
one step at a time against the oracle.
N = 1M, D = 100k, k = 1,000 run to convergence or 50 iterations, each
iteration one step against the oracle.
NYT-shaped corpus (N = 1,285,944, D = 495,714, ~226 nonzeros per row, k =
10k): iteration 1 on sampled objects against the oracle; update 1 bit for bit
against the oracle's update of the GPU's assignment; iteration 2 on sampled
objects, flags and the exact mult-add count.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def headline():
    log("generating the 8M x 140k corpus")
    corpus, ids, w = synth.workload("8m-f32")
    from paper_2103_16141_amd.api import DeviceCsr
    X = DeviceCsr.from_corpus(corpus, torch.device("cuda", 0))
    torch.cuda.synchronize()
    return corpus, ids, w, X


def _export_centroids(ivf):
    ex = ivf.export()
    out = {key: ex[key].cpu().numpy() for key in ("c_ptr", "c_col", "c_val", "lam", "term_ptr", "split")}
    return ex, out


def test_headline_one_step_parity(headline):
    """Iterations 1-4 at full size, each checked against the oracle one step at
    a time: the oracle updates from the GPU's previous assignment, so its
    centroids must equal the GPU's bit for bit; sampled objects' assignments
    against them must match exactly; the invariance flags and the exact
    mult-add count are compared over all objects."""
    from paper_2103_16141_amd.api import Context, Lloyd
    corpus, ids, w, X = headline
    k = w["k"]
    ctx = Context(0)
    L = Lloyd(ctx, X, k, ids)
    rng = np.random.default_rng(1)
    cents = oracle.init_centroids(corpus, ids)
    a_prev = lam_prev = None
    for r in range(1, 5):
        log("iteration %d on the GPU" % r)
        st = L.assign()
        a = L.a.cpu().numpy()
        own = L.own.cpu().numpy().astype(np.float64)
        lam = L.lam.cpu().numpy()
        sample = np.sort(rng.choice(corpus.n, 1500, replace=False))
        log("oracle on %d sampled objects" % len(sample))
        ref, ref_own, _ = oracle.assign(corpus, cents, rows=sample)
        bad = np.nonzero(a[sample] != ref)[0]
        assert len(bad) == 0, "iteration %d: sampled objects %s differ" % (r, sample[bad][:5])
        rel = np.abs(own[sample] - ref_own) / np.maximum(np.abs(ref_own), 1e-30)
        assert rel.max() < 1e-5, "iteration %d: own similarity off by %.3g" % (r, rel.max())
        lam_ref, moved = oracle.mark_invariant(a_prev, a, k, first=(r == 1))
        assert np.array_equal(lam, lam_ref), "iteration %d: flags differ" % r
        assert st["moved"] == moved
        log("oracle mult-add count over all objects")
        m_ref = oracle.multadds(corpus, oracle.build_ivf(cents, lam_prev), icp=(r >= 2), lam_prev=lam_prev,
                                a_prev=a_prev)
        assert st["multadds"] == m_ref, "iteration %d: multadds %d vs %d" % (r, st["multadds"], m_ref)
        if r >= 3:      # flags after iteration 1 are all zero, so ICP starts at iteration 3
            assert st["icp_objects"] > 0
        log("update %d: GPU and oracle" % r)
        L.update()
        cents, _ = oracle.update(corpus, a, cents)
        ex, got = _export_centroids(L.ivf)
        assert np.array_equal(got["c_ptr"], cents.ptr), "update %d: centroid sizes differ" % r
        assert np.array_equal(got["c_col"], cents.col), "update %d: centroid supports differ" % r
        assert np.array_equal(got["c_val"], cents.val), "update %d: centroid values differ" % r
        assert np.array_equal(got["lam"], lam)
        if r == 2:
            log("structured file against the oracle's")
            ivf_ref = oracle.build_ivf(cents, lam)
            assert np.array_equal(got["term_ptr"], ivf_ref.term_ptr)
            assert np.array_equal(got["split"], ivf_ref.split)
            assert np.array_equal(ex["p_cid"].cpu().numpy(), ivf_ref.cid)
            assert np.array_equal(ex["p_val"].cpu().numpy(), ivf_ref.val)
            del ivf_ref
        if r == 1:
            # independent of the oracle: sampled centroids are the normalised
            # means (dense FP64 numpy) of the objects the GPU assigned to them
            sizes = np.bincount(a, minlength=k)
            cptr, ccol, cval = got["c_ptr"], got["c_col"], got["c_val"]
            for j in rng.choice(np.nonzero(sizes > 0)[0], 12, replace=False):
                mem = np.nonzero(a == j)[0]
                idx = np.concatenate([np.arange(corpus.row_ptr[i], corpus.row_ptr[i + 1]) for i in mem])
                w_ = np.zeros(corpus.d)
                np.add.at(w_, corpus.col[idx], corpus.val[idx].astype(np.float64))
                u = w_ / np.linalg.norm(w_)
                dense = np.zeros(corpus.d)
                dense[ccol[cptr[j]:cptr[j + 1]]] = cval[cptr[j]:cptr[j + 1]]
                assert np.array_equal(np.nonzero(dense)[0], np.nonzero(u)[0])
                np.testing.assert_allclose(dense, u, rtol=1e-12, atol=1e-300)
        del ex, got
        a_prev, lam_prev = a, lam
    ctx.close()


def test_precision_form_k20k_one_step_parity():
    """The precision form at its own configuration (N = 8M, D = 140k,
    k = 20,000, BF16 postings): iterations 1-3 one step at a time against the
    oracle, as for the headline workload."""
    from paper_2103_16141_amd.api import Context, DeviceCsr, Lloyd
    log("generating the 8M x 140k corpus for k = 20,000")
    corpus, ids, w = synth.workload("8m-bf16-k20k")
    k = w["k"]
    X = DeviceCsr.from_corpus(corpus, torch.device("cuda", 0))
    ctx = Context(0, posting_dtype="bf16")
    L = Lloyd(ctx, X, k, ids)
    rng = np.random.default_rng(11)
    cents = oracle.init_centroids(corpus, ids)
    a_prev = lam_prev = None
    for r in range(1, 4):
        log("iteration %d" % r)
        st = L.assign()
        a = L.a.cpu().numpy()
        lam = L.lam.cpu().numpy()
        sample = np.sort(rng.choice(corpus.n, 1000, replace=False))
        ref, _, _ = oracle.assign(corpus, cents, rows=sample)
        bad = np.nonzero(a[sample] != ref)[0]
        assert len(bad) == 0, "iteration %d: sampled objects %s differ" % (r, sample[bad][:5])
        lam_ref, moved = oracle.mark_invariant(a_prev, a, k, first=(r == 1))
        assert np.array_equal(lam, lam_ref) and st["moved"] == moved
        m_ref = oracle.multadds(corpus, oracle.build_ivf(cents, lam_prev), icp=(r >= 2), lam_prev=lam_prev,
                                a_prev=a_prev)
        assert st["multadds"] == m_ref
        assert st["rescored_objects"] > 0   # BF16 needs the FP64 re-score
        L.update()
        cents, _ = oracle.update(corpus, a, cents)
        ex, got = _export_centroids(L.ivf)
        assert np.array_equal(got["c_ptr"], cents.ptr)
        assert np.array_equal(got["c_col"], cents.col)
        assert np.array_equal(got["c_val"], cents.val)
        del ex, got
        a_prev, lam_prev = a, lam
    ctx.close()
    del X
    torch.cuda.empty_cache()


def test_headline_filter_modes_agree(headline):
    from paper_2103_16141_amd.api import Context
    corpus, ids, w, X = headline
    res = {}
    for mode, posting in (("sivf", "fp32"), ("ivf", "fp32"), ("relaxed", "fp32"), ("sivf", "bf16")):
        log("3 iterations, filter %s, %s postings" % (mode, posting))
        ctx = Context(0, filter_mode=mode, posting_dtype=posting)
        a, own, ivf, stats = ctx.run_lloyd(X, w["k"], ids, 3, keep_centroids=False)
        res[mode, posting] = (a.cpu().numpy(), [s["multadds"] for s in stats], [s["icp_objects"] for s in stats])
        ctx.close()
    base = res["sivf", "fp32"]
    for key, (a, m, icp) in res.items():
        assert np.array_equal(a, base[0]), key
    assert res["sivf", "bf16"][1] == base[1]
    assert all(s <= i for s, i in zip(base[1], res["ivf", "fp32"][1]))
    assert all(r <= s for r, s in zip(res["relaxed", "fp32"][1], base[1]))
    assert base[2][2] > 0 and res["ivf", "fp32"][2][2] == 0
    assert res["relaxed", "fp32"][2][2] >= base[2][2]


def test_config_1m_to_convergence():
    """N = 1M, D = 100k, Poisson(100), k = 1,000, run to convergence (no
    assignment change) or 50 iterations, every iteration checked one step at a
    time against the oracle: flags, moved count and the exact mult-add count
    over all objects, 2,000 sampled assignments, and the oracle's update of the
    GPU's assignment bitwise against the GPU's centroids."""
    from paper_2103_16141_amd.api import Context, DeviceCsr, Lloyd
    log("generating the 1M x 100k corpus")
    corpus, ids, w = synth.workload("1m-f32")
    k = w["k"]
    X = DeviceCsr.from_corpus(corpus, torch.device("cuda", 0))
    ctx = Context(0)
    L = Lloyd(ctx, X, k, ids)
    rng = np.random.default_rng(7)
    cents = oracle.init_centroids(corpus, ids)
    a_prev = lam_prev = None
    converged = False
    for r in range(1, w["iters"] + 1):
        st = L.assign()
        a = L.a.cpu().numpy()
        lam = L.lam.cpu().numpy()
        sample = np.sort(rng.choice(corpus.n, 2000, replace=False))
        ref, _, _ = oracle.assign(corpus, cents, rows=sample)
        bad = np.nonzero(a[sample] != ref)[0]
        assert len(bad) == 0, "iteration %d: sampled objects %s differ" % (r, sample[bad][:5])
        lam_ref, moved = oracle.mark_invariant(a_prev, a, k, first=(r == 1))
        assert np.array_equal(lam, lam_ref) and st["moved"] == moved, "iteration %d: flags or moved" % r
        m_ref = oracle.multadds(corpus, oracle.build_ivf(cents, lam_prev), icp=(r >= 2), lam_prev=lam_prev,
                                a_prev=a_prev)
        assert st["multadds"] == m_ref, "iteration %d: multadds %d vs %d" % (r, st["multadds"], m_ref)
        if r >= 2 and moved == 0:
            converged = True
            assert st["multadds"] == 0
            break
        L.update()
        cents, _ = oracle.update(corpus, a, cents)
        ex, got = _export_centroids(L.ivf)
        assert np.array_equal(got["c_ptr"], cents.ptr), "update %d: centroid sizes differ" % r
        assert np.array_equal(got["c_col"], cents.col), "update %d: centroid supports differ" % r
        assert np.array_equal(got["c_val"], cents.val), "update %d: centroid values differ" % r
        del ex, got
        a_prev, lam_prev = a, lam
    log("stopped after iteration %d (converged: %s)" % (r, converged))
    ctx.close()


def test_soft_fullsize_sampled():
    from paper_2103_16141_amd.api import Context, DeviceCsr
    log("soft form at N=262,144, D=100k, k=4,096")
    corpus, ids, w = synth.workload("soft-262k")
    C = synth.dense_centroids(corpus, ids, noise=1e-3, seed=2103 + 5)
    X = DeviceCsr.from_corpus(corpus, torch.device("cuda", 0))
    Cg = torch.from_numpy(C).cuda()
    ctx = Context(0)
    tau, g = 0.05, 1.0
    lse, loss = ctx.soft_assign_fwd(X, Cg, tau)
    dC, dX = ctx.soft_assign_bwd(X, Cg, tau, lse, g)
    torch.cuda.synchronize()
    lse_h, dX_h = lse.cpu().numpy(), dX.cpu().numpy()
    del Cg
    C64 = C.astype(np.float64)
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(corpus.n, 48, replace=False))
    log("oracle on sampled rows")
    lse_ref = oracle.soft_forward(corpus, C64, tau, rows=rows)
    np.testing.assert_allclose(lse_h[rows], lse_ref, rtol=0, atol=5e-4)
    _, dx_ref = oracle.soft_backward(corpus, C64, tau, g, lse_ref, rows=rows, want_dc=False)
    for i in rows:
        b, e = corpus.row_ptr[i], corpus.row_ptr[i + 1]
        np.testing.assert_allclose(dX_h[b:e], dx_ref[b:e], rtol=2e-3, atol=1e-9)
    # dC column sums: sum_j dC_j = -(g/tau) sum_i x_i (all D columns)
    dC_h = dC.cpu().numpy()
    xs = np.zeros(corpus.d)
    np.add.at(xs, corpus.col, corpus.val.astype(np.float64))
    np.testing.assert_allclose(dC_h.astype(np.float64).sum(0), -(g / tau) * xs, rtol=3e-3, atol=1e-5)
    # sampled dC columns of terms used by few objects, from exactly those rows
    df = np.bincount(corpus.col, minlength=corpus.d)
    cand = np.nonzero((df >= 2) & (df <= 6))[0]
    terms = rng.choice(cand, 4, replace=False)
    pos = np.nonzero(np.isin(corpus.col, terms))[0]
    rows_t = np.unique(np.searchsorted(corpus.row_ptr, pos, side="right") - 1)
    lse_t = oracle.soft_forward(corpus, C64, tau, rows=rows_t)
    dc_ref, _ = oracle.soft_backward(corpus, C64, tau, g, lse_t, rows=rows_t, want_dx=False)
    for t in terms:
        np.testing.assert_allclose(dC_h[:, t], dc_ref[:, t], rtol=2e-3, atol=1e-9)
    assert math.isfinite(loss)


def test_nyt_shape_sampled():
    from paper_2103_16141_amd.api import Context, DeviceCsr, Lloyd
    log("generating the NYT-shaped corpus")
    corpus, ids, w = synth.workload("nyt-f32")
    k = w["k"]
    X = DeviceCsr.from_corpus(corpus, torch.device("cuda", 0))
    L = Lloyd(Context(0), X, k, ids)
    log("iteration 1")
    L.assign()
    a1 = L.a.cpu().numpy()
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(corpus.n, 600, replace=False))
    ref, _, _ = oracle.assign(corpus, oracle.init_centroids(corpus, ids), rows=sample)
    assert np.array_equal(a1[sample], ref)
    log("update 1 against the oracle, iteration 2")
    L.update()
    cents, _ = oracle.update(corpus, a1, oracle.init_centroids(corpus, ids))
    ex, got = _export_centroids(L.ivf)
    assert np.array_equal(got["c_ptr"], cents.ptr)
    assert np.array_equal(got["c_col"], cents.col)
    assert np.array_equal(got["c_val"], cents.val)
    del ex, got
    st = L.assign()
    a2 = L.a.cpu().numpy()
    sample = np.sort(rng.choice(corpus.n, 600, replace=False))
    ref, _, _ = oracle.assign(corpus, cents, rows=sample)
    assert np.array_equal(a2[sample], ref)
    lam_ref, moved = oracle.mark_invariant(a1, a2, k, first=False)
    assert np.array_equal(L.lam.cpu().numpy(), lam_ref) and st["moved"] == moved
    m_ref = oracle.multadds(corpus, oracle.build_ivf(cents, np.zeros(k, np.uint8)), icp=True,
                            lam_prev=np.zeros(k, np.uint8), a_prev=a1)
    assert st["multadds"] == m_ref
