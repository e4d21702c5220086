"""GPU parity of the soft-assignment form against the FP64 oracle.

Tolerances from the arithmetic: S in FP32 over n <= ~200 products has
|dS| <= gamma_n(2^-24) * sum|x||c| <= ~1.2e-5 (rows and centroids unit norm);
lse adds |dS|/tau plus an FP32 sum of k exponentials (gamma_k(2^-24) relative),
so |d lse| <= 5e-4 at tau = 0.05, k <= 5000.  P = exp(S/tau - lse) then carries
a relative error <= ~1e-3, and dX, dC are sums of same-signed terms (dS <= 0,
X >= 0, C >= 0), so a relative tolerance of 2e-3 holds entrywise.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

TAU = 0.05


def _case(n, d, k, seed, lam=20):
    c = synth.make_corpus(n, d, lam, 1.1, np.float32, seed=seed)
    ids = synth.init_ids(n, k, seed + 7) if k <= n else np.arange(k) % n
    C = synth.dense_centroids(c, ids, noise=1e-3, seed=seed + 11)
    return c, C


def _dev(c, C):
    from paper_2103_16141_amd.api import DeviceCsr
    return DeviceCsr.from_corpus(c, torch.device("cuda", 0)), torch.from_numpy(C).cuda()


def _ctx():
    from paper_2103_16141_amd.api import Context
    return Context(0)


@pytest.mark.parametrize("n,d,k", [(300, 500, 50), (257, 800, 5003), (1000, 3000, 4096), (4000, 1500, 20000),
                                   (200, 400, 1), (200, 400, 3)])
def test_soft_forward_backward_match_oracle(n, d, k):
    log("soft n=%d d=%d k=%d" % (n, d, k))
    c, C = _case(n, d, k, seed=n + k)
    X, Cg = _dev(c, C)
    ctx = _ctx()
    lse, loss = ctx.soft_assign_fwd(X, Cg, TAU)
    lse_ref = oracle.soft_forward(c, C.astype(np.float64), TAU)
    np.testing.assert_allclose(lse.cpu().numpy(), lse_ref, rtol=0, atol=5e-4)
    loss_ref = -math.fsum(lse_ref.tolist())
    assert abs(loss - loss_ref) <= 5e-4 * n
    g = 0.8
    dC, dX = ctx.soft_assign_bwd(X, Cg, TAU, lse, g)
    dC_ref, dX_ref = oracle.soft_backward(c, C.astype(np.float64), TAU, g, lse_ref)
    np.testing.assert_allclose(dX.cpu().numpy(), dX_ref, rtol=2e-3, atol=1e-9)
    np.testing.assert_allclose(dC.cpu().numpy(), dC_ref, rtol=2e-3, atol=1e-7)
    # dC's column sums have a closed form: sum_j dC_j = -(g/tau) sum_i x_i
    xs = np.zeros(d)
    np.add.at(xs, c.col, c.val.astype(np.float64))
    np.testing.assert_allclose(dC.cpu().numpy().astype(np.float64).sum(0), -(g / TAU) * xs, rtol=2e-3, atol=1e-6)


@pytest.mark.parametrize("k", [300, 299])
def test_soft_rows_longer_than_one_lds_batch(k):
    # ~300 terms per row: the backward's long-row kernel stages a row's
    # centroid slices in batches of 136 terms (two or three per row); k = 300
    # ends on a partial 64-column block, k = 299 also takes the unaligned
    # gathers
    log("soft long rows k=%d" % k)
    c, C = _case(120, 2000, k, seed=77 + k, lam=300)
    assert np.diff(c.row_ptr).max() > 288
    X, Cg = _dev(c, C)
    ctx = _ctx()
    lse, _ = ctx.soft_assign_fwd(X, Cg, TAU)
    lse_ref = oracle.soft_forward(c, C.astype(np.float64), TAU)
    np.testing.assert_allclose(lse.cpu().numpy(), lse_ref, rtol=0, atol=5e-4)
    dC, dX = ctx.soft_assign_bwd(X, Cg, TAU, lse, 1.3)
    dC_ref, dX_ref = oracle.soft_backward(c, C.astype(np.float64), TAU, 1.3, lse_ref)
    np.testing.assert_allclose(dX.cpu().numpy(), dX_ref, rtol=2e-3, atol=1e-9)
    np.testing.assert_allclose(dC.cpu().numpy(), dC_ref, rtol=2e-3, atol=1e-7)


@pytest.mark.parametrize("k", [512, 299])
def test_soft_rows_on_both_sides_of_the_register_limit(k):
    # Poisson(128) rows: rows of at most 128 terms go to the register-held
    # rows kernel, longer ones to the LDS-staged one, in the same call
    log("soft mixed rows k=%d" % k)
    c, C = _case(600, 3000, k, seed=91 + k, lam=128)
    lens = np.diff(c.row_ptr)
    assert (lens <= 128).sum() > 100 and (lens > 128).sum() > 100
    assert 128 in lens and 129 in lens
    X, Cg = _dev(c, C)
    ctx = _ctx()
    lse, _ = ctx.soft_assign_fwd(X, Cg, TAU)
    lse_ref = oracle.soft_forward(c, C.astype(np.float64), TAU)
    np.testing.assert_allclose(lse.cpu().numpy(), lse_ref, rtol=0, atol=5e-4)
    dC, dX = ctx.soft_assign_bwd(X, Cg, TAU, lse, 0.6)
    dC_ref, dX_ref = oracle.soft_backward(c, C.astype(np.float64), TAU, 0.6, lse_ref)
    np.testing.assert_allclose(dX.cpu().numpy(), dX_ref, rtol=2e-3, atol=1e-9)
    np.testing.assert_allclose(dC.cpu().numpy(), dC_ref, rtol=2e-3, atol=1e-7)


@pytest.mark.parametrize("k", [16384, 16383])
def test_soft_hot_terms_cut_at_row_blocks(k):
    # 40 terms, 20 per row: at k = 16384 the dS chunks hold 4096 rows, and in
    # the first one 15 terms have more than 2048 entries (summed in 512-row
    # blocks across terms), 25 have 257..2048 (2048-row blocks); the second
    # chunk (1904 rows) has none above 2048; k = 16383 takes the unaligned
    # gathers
    log("soft hot terms k=%d" % k)
    c = synth.make_corpus(6000, 40, 20, 1.1, np.float32, seed=123)
    C = synth.dense_centroids(c, np.arange(k) % c.n, noise=1e-3, seed=7)
    rc = (64 << 20) // k
    cnt = np.bincount(c.col[:c.row_ptr[rc]], minlength=c.d)
    assert rc == 4096 and (cnt > 2048).sum() >= 10 and ((cnt > 256) & (cnt <= 2048)).sum() >= 10
    X, Cg = _dev(c, C)
    ctx = _ctx()
    lse, _ = ctx.soft_assign_fwd(X, Cg, TAU)
    lse_ref = oracle.soft_forward(c, C.astype(np.float64), TAU)
    np.testing.assert_allclose(lse.cpu().numpy(), lse_ref, rtol=0, atol=5e-4)
    dC, dX = ctx.soft_assign_bwd(X, Cg, TAU, lse, 0.9)
    dC_ref, dX_ref = oracle.soft_backward(c, C.astype(np.float64), TAU, 0.9, lse_ref)
    np.testing.assert_allclose(dX.cpu().numpy(), dX_ref, rtol=2e-3, atol=1e-9)
    np.testing.assert_allclose(dC.cpu().numpy(), dC_ref, rtol=2e-3, atol=1e-7)
    again = ctx.soft_assign_bwd(X, Cg, TAU, lse, 0.9)
    assert torch.equal(again[0], dC) and torch.equal(again[1], dX)


def test_soft_empty_rows():
    # rows without terms have S = 0, so lse = log k, and add nothing to dC;
    # empty rows first, last and in a run, in a chunk with ordinary rows
    log("soft empty rows")
    c = synth.make_corpus(300, 500, 20, 1.1, np.float32, seed=31)
    empty = {0, 7, 100, 101, 102, 103, 104, 299}
    cols, vals, rp = [], [], [0]
    for i in range(c.n):
        if i not in empty:
            cols.append(c.col[c.row_ptr[i]:c.row_ptr[i + 1]])
            vals.append(c.val[c.row_ptr[i]:c.row_ptr[i + 1]])
        rp.append(rp[-1] + (0 if i in empty else int(c.row_ptr[i + 1] - c.row_ptr[i])))
    e = synth.Corpus(c.n, c.d, np.array(rp, np.int64), np.concatenate(cols).astype(np.int32),
                     np.concatenate(vals).astype(np.float32))
    C = synth.dense_centroids(c, synth.init_ids(c.n, 40, 5), noise=1e-3, seed=9)
    X, Cg = _dev(e, C)
    ctx = _ctx()
    lse, _ = ctx.soft_assign_fwd(X, Cg, TAU)
    lse_ref = oracle.soft_forward(e, C.astype(np.float64), TAU)
    np.testing.assert_allclose(lse.cpu().numpy(), lse_ref, rtol=0, atol=5e-4)
    assert abs(float(lse[0]) - math.log(40)) < 1e-5
    dC, dX = ctx.soft_assign_bwd(X, Cg, TAU, lse, 0.8)
    dC_ref, dX_ref = oracle.soft_backward(e, C.astype(np.float64), TAU, 0.8, lse_ref)
    np.testing.assert_allclose(dX.cpu().numpy(), dX_ref, rtol=2e-3, atol=1e-9)
    np.testing.assert_allclose(dC.cpu().numpy(), dC_ref, rtol=2e-3, atol=1e-7)


def test_soft_backward_is_deterministic_and_partial_outputs():
    c, C = _case(800, 1200, 300, seed=3)
    X, Cg = _dev(c, C)
    ctx = _ctx()
    lse, _ = ctx.soft_assign_fwd(X, Cg, TAU)
    a = ctx.soft_assign_bwd(X, Cg, TAU, lse, 1.0)
    b = ctx.soft_assign_bwd(X, Cg, TAU, lse, 1.0)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    dC_only, none_x = ctx.soft_assign_bwd(X, Cg, TAU, lse, 1.0, want_dx=False)
    assert none_x is None and torch.equal(dC_only, a[0])


def test_autograd_function_and_finite_differences():
    from paper_2103_16141_amd.soft_assign import soft_assign_loss
    c, C = _case(200, 300, 40, seed=5)
    X, Cg = _dev(c, C)
    Cp = Cg.clone().requires_grad_(True)
    X.val.requires_grad_(True)
    loss = soft_assign_loss(X, Cp, TAU)
    loss.backward()
    lse_ref = oracle.soft_forward(c, C.astype(np.float64), TAU)
    dC_ref, dX_ref = oracle.soft_backward(c, C.astype(np.float64), TAU, 1.0, lse_ref)
    np.testing.assert_allclose(Cp.grad.cpu().numpy(), dC_ref, rtol=2e-3, atol=1e-7)
    np.testing.assert_allclose(X.val.grad.cpu().numpy(), dX_ref, rtol=2e-3, atol=1e-9)
    # FP64 central differences of the oracle's loss agree with the GPU gradient
    rng = np.random.default_rng(1)
    h = 1e-5
    for _ in range(5):
        j, t = int(rng.integers(40)), int(c.col[rng.integers(c.nnz)])
        Cp_, Cm_ = C.astype(np.float64), C.astype(np.float64)
        Cp_[j, t] += h
        Cm_[j, t] -= h
        fd = (-math.fsum(oracle.soft_forward(c, Cp_, TAU).tolist()) + math.fsum(oracle.soft_forward(c, Cm_, TAU).tolist())) / (2 * h)
        assert abs(fd - float(Cp.grad[j, t])) <= 2e-3 * abs(fd) + 1e-5


def test_soft_errors():
    from paper_2103_16141_amd._native import SivfError
    c, C = _case(50, 80, 10, seed=9)
    X, Cg = _dev(c, C)
    ctx = _ctx()
    with pytest.raises(SivfError) as e:
        ctx.soft_assign_fwd(X, Cg, 0.0)
    assert e.value.name == "SIVF_E_INVALID"
    c64 = synth.Corpus(c.n, c.d, c.row_ptr, c.col, c.val.astype(np.float64))
    X64, _ = _dev(c64, C)
    with pytest.raises(SivfError) as e:
        ctx.soft_assign_fwd(X64, Cg, TAU)
    assert e.value.name == "SIVF_E_UNSUPPORTED"
