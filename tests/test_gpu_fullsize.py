"""Full-size checks in the launch configuration bench.py times.

N = 8M objects, D = 140k, k = 10k, automatic tiles (the headline workload):
  * iteration 1 on sampled objects against the oracle (its inputs are the
    seeded corpus and the seeded initial centroids only);
  * properties that hold at any size for later steps, checked on samples with
    dense FP64 numpy (not the oracle): each sampled centroid after update 1 is
    the normalised mean of the objects the GPU assigned to it; each sampled
    object's iteration-2 assignment maximises the FP64 similarity against the
    GPU's centroids; SIVF (ICP) and IVF (no filter) runs give identical
    assignments and the SIVF count never exceeds the IVF count.
Soft form at its full shape (N = 262,144, D = 100k, k = 4,096): sampled rows'
lse and dX and sampled columns of dC against the oracle; the dC column-sum
identity over all columns.
NYT-shaped corpus (N = 1,285,944, D = 495,714, ~226 nonzeros per row, k =
10k): iteration 1 on sampled objects against the oracle, iteration 2 against
dense FP64 numpy on samples.
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


def _rows_dense(corpus, rows, term_index):
    out = np.zeros((len(rows), len(term_index)), dtype=np.float64)
    for r, i in enumerate(rows):
        b, e = corpus.row_ptr[i], corpus.row_ptr[i + 1]
        out[r, [term_index[t] for t in corpus.col[b:e]]] = corpus.val[b:e]
    return out


def test_headline_sampled_parity_and_properties(headline):
    from paper_2103_16141_amd.api import Context, Lloyd
    corpus, ids, w, X = headline
    k = w["k"]
    ctx = Context(0)
    L = Lloyd(ctx, X, k, ids)
    log("iteration 1 on the GPU")
    st1 = L.assign()
    a1 = L.a.cpu().numpy()
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(corpus.n, 1500, replace=False))
    log("oracle on %d sampled objects" % len(sample))
    ref, _, _ = oracle.assign(corpus, oracle.init_centroids(corpus, ids), rows=sample)
    assert np.array_equal(a1[sample], ref)
    assert st1["moved"] == corpus.n

    log("update 1 and export")
    L.update()
    ex = L.ivf.export()
    cptr = ex["c_ptr"].cpu().numpy()
    ccol = ex["c_col"].cpu().numpy()
    cval = ex["c_val"].cpu().numpy()
    sizes = np.bincount(a1, minlength=k)
    for j in rng.choice(np.nonzero(sizes > 0)[0], 12, replace=False):
        mem = np.nonzero(a1 == j)[0]
        idx = np.concatenate([np.arange(corpus.row_ptr[i], corpus.row_ptr[i + 1]) for i in mem])
        w_ = np.zeros(corpus.d)
        np.add.at(w_, corpus.col[idx], corpus.val[idx].astype(np.float64))
        u = w_ / np.linalg.norm(w_)
        got = np.zeros(corpus.d)
        got[ccol[cptr[j]:cptr[j + 1]]] = cval[cptr[j]:cptr[j + 1]]
        assert np.array_equal(np.nonzero(got)[0], np.nonzero(u)[0])
        np.testing.assert_allclose(got, u, rtol=1e-12, atol=1e-300)

    log("iteration 2 on the GPU")
    L.assign()
    a2 = L.a.cpu().numpy()
    objs = np.sort(rng.choice(corpus.n, 200, replace=False))
    terms = np.unique(np.concatenate([corpus.col[corpus.row_ptr[i]:corpus.row_ptr[i + 1]] for i in objs]))
    tix = {int(t): r for r, t in enumerate(terms)}
    Xs = _rows_dense(corpus, objs, tix)
    M = np.zeros((len(terms), k))
    rows_of = np.repeat(np.arange(k), np.diff(cptr))
    keep = np.isin(ccol, terms)
    M[np.searchsorted(terms, ccol[keep]), rows_of[keep]] = cval[keep]
    rho = Xs @ M
    best = rho.max(1)
    got = rho[np.arange(len(objs)), a2[objs]]
    assert np.all(got >= best - 1e-12 * np.maximum(1.0, np.abs(best)))
    del M, rho


def test_headline_filter_modes_agree(headline):
    from paper_2103_16141_amd.api import Context
    corpus, ids, w, X = headline
    res = {}
    for mode in ("sivf", "ivf"):
        log("3 iterations, filter %s" % mode)
        ctx = Context(0, filter_mode=mode)
        a, own, ivf, stats = ctx.run_lloyd(X, w["k"], ids, 3, keep_centroids=False)
        res[mode] = (a.cpu().numpy(), [s["multadds"] for s in stats], [s["icp_objects"] for s in stats])
        ctx.close()
    assert np.array_equal(res["sivf"][0], res["ivf"][0])
    assert all(s <= i for s, i in zip(res["sivf"][1], res["ivf"][1]))
    assert res["sivf"][2][2] > 0 and res["ivf"][2][2] == 0


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
    log("update 1, iteration 2")
    L.update()
    ex = L.ivf.export()
    L.assign()
    a2 = L.a.cpu().numpy()
    cptr, ccol, cval = (ex[key].cpu().numpy() for key in ("c_ptr", "c_col", "c_val"))
    objs = np.sort(rng.choice(corpus.n, 120, replace=False))
    terms = np.unique(np.concatenate([corpus.col[corpus.row_ptr[i]:corpus.row_ptr[i + 1]] for i in objs]))
    tix = {int(t): r for r, t in enumerate(terms)}
    Xs = _rows_dense(corpus, objs, tix)
    M = np.zeros((len(terms), k))
    rows_of = np.repeat(np.arange(k), np.diff(cptr))
    keep = np.isin(ccol, terms)
    M[np.searchsorted(terms, ccol[keep]), rows_of[keep]] = cval[keep]
    rho = Xs @ M
    best = rho.max(1)
    got = rho[np.arange(len(objs)), a2[objs]]
    assert np.all(got >= best - 1e-12 * np.maximum(1.0, np.abs(best)))
