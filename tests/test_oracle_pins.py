"""Pins for the FP64 oracle: each test checks it against something other than
itself (exact rationals, closed forms, dense numpy in another formulation,
invariants the paper states, special cases with known answers)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests.util import corpus_from_dense, corpus_from_rows, exact_sims, gamma

GOLD = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2.0 ** -53


def _tiny(seed, n=48, d=24, lam=6, k=6, dtype=np.float64):
    c = synth.make_corpus(n, d, lam, 1.0, dtype, seed=seed)
    ids = synth.init_ids(n, k, seed + 1000)
    return c, ids


# --------------------------------------------------------------------------
# similarity + argmax against exact rational brute force
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_assign_matches_exact_rational_argmax(seed):
    c, ids = _tiny(seed)
    cents = oracle.init_centroids(c, ids)
    a, own, _ = oracle.assign(c, cents)
    ex = exact_sims(c, cents)
    for i in range(c.n):
        n_i = int(c.row_ptr[i + 1] - c.row_ptr[i])
        # |fl(rho) - rho| <= gamma_n * sum |v||u| <= gamma_n * ||x|| ||u|| ~ gamma_n
        bound = gamma(n_i + 1, U64) * 1.01
        best = max(ex[i])
        exact_arg = ex[i].index(best)  # lowest index among exact maxima
        assert abs(Fraction(own[i]) - ex[i][a[i]]) <= Fraction(bound)
        srt = sorted(set(ex[i]), reverse=True)
        if len(srt) == 1 or float(srt[0] - srt[1]) > 2 * bound:
            assert a[i] == exact_arg
        assert abs(own[i] - float(best)) <= 2 * bound


def test_dyadic_golden_iteration_by_iteration():
    g = json.load(open(os.path.join(GOLD, "dyadic_8x8.json")))
    c = corpus_from_rows(g["rows"], g["d"], g["value"])
    ids = np.array(g["init_ids"])
    exp = g["expected"]
    cents0 = oracle.init_centroids(c, ids)
    a1, own1, _ = oracle.assign(c, cents0)
    assert a1.tolist() == exp["a1"]
    ex = exact_sims(c, cents0)
    for i, row in enumerate(exp["rho1"]):
        assert [Fraction(s) for s in row] == ex[i]
        assert Fraction(own1[i]) == Fraction(row[a1[i]])  # exact: dyadic values
    tr = oracle.lloyd(c, 3, ids, 10, icp=True)
    assert tr.assign[0].tolist() == exp["a1"]
    assert tr.assign[1].tolist() == exp["a2"]
    assert tr.iters == exp["converged_at"] and tr.converged
    assert tr.multadds == exp["multadds"]
    mu1, _ = oracle.update(c, a1, cents0)
    for j, spec in exp["mu1_squared"].items():
        j = int(j)
        terms = mu1.col[mu1.ptr[j]:mu1.ptr[j + 1]].tolist()
        vals = mu1.val[mu1.ptr[j]:mu1.ptr[j + 1]]
        assert terms == spec["terms"]
        for v, sq in zip(vals, spec["sq"]):
            want = math.sqrt(float(Fraction(sq)))  # sqrt correctly rounded of a rounded rational
            assert abs(v - want) <= 4 * np.spacing(want)


def test_exact_ties_break_to_lowest_index():
    # duplicate centroids: x0 == x1 == x2 as init; every object ties among 0,1,2
    rows = [[0, 1], [0, 1], [0, 1], [1, 2], [0, 2], [2, 3]]
    c = corpus_from_rows(rows, 4, 2 ** -0.5)
    cents = oracle.init_centroids(c, [2, 1, 0, 5])
    a, _, top2 = oracle.assign(c, cents)
    ex = exact_sims(c, cents)
    for i in range(c.n):
        best = max(ex[i])
        assert a[i] == ex[i].index(best)
    assert a[0] == 0 and a[3] == 0  # three-way ties resolved to centroid 0


def test_euclidean_argmin_equals_cosine_argmax():
    # Section 1 / Section 2.2: on the unit sphere argmin ||x - mu||^2 = argmax <x, mu>
    c = synth.make_corpus(400, 60, 12, 1.0, np.float64, seed=21)
    ids = synth.init_ids(400, 9, 4)
    cents = oracle.init_centroids(c, ids)
    mu1, _ = oracle.update(c, oracle.assign(c, cents)[0], cents)
    a, _, top2 = oracle.assign(c, mu1)
    x = np.zeros((c.n, c.d))
    x[np.repeat(np.arange(c.n), np.diff(c.row_ptr)), c.col] = c.val
    m = mu1.dense()
    dist = ((x[:, None, :] - m[None, :, :]) ** 2).sum(-1)
    clear = (top2[:, 0] - top2[:, 1]) > 1e-9
    assert clear.mean() > 0.95
    assert np.array_equal(np.argmin(dist, 1)[clear], a[clear])


# --------------------------------------------------------------------------
# update against dense numpy (different formulation), norms, support
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_update_matches_dense_numpy(dtype):
    c = synth.make_corpus(600, 80, 10, 1.0, dtype, seed=31)
    ids = synth.init_ids(600, 12, 8)
    cents = oracle.init_centroids(c, ids)
    a, _, _ = oracle.assign(c, cents)
    mu, counts = oracle.update(c, a, cents)
    x = np.zeros((c.n, c.d))
    x[np.repeat(np.arange(c.n), np.diff(c.row_ptr)), c.col] = c.val.astype(np.float64)
    dense = mu.dense()
    for j in range(12):
        mem = np.nonzero(a == j)[0]
        assert counts[j] == len(mem)
        if len(mem) == 0:
            continue
        w = x[mem].sum(0) / len(mem)
        u = w / np.linalg.norm(w)
        np.testing.assert_allclose(dense[j], u, rtol=1e-14, atol=1e-16)
        support = np.unique(c.col[np.concatenate([np.arange(c.row_ptr[i], c.row_ptr[i + 1]) for i in mem])])
        assert np.array_equal(mu.col[mu.ptr[j]:mu.ptr[j + 1]], support)  # nonnegative data
        assert abs(math.fsum((mu.val[mu.ptr[j]:mu.ptr[j + 1]] ** 2).tolist()) - 1.0) < 1e-15


def test_update_single_member_and_k1_closed_form():
    c = synth.make_corpus(300, 50, 8, 1.0, np.float64, seed=41)
    # k = 1: mu = normalise(sum x); converged at r = 2
    tr = oracle.lloyd(c, 1, [17], 5)
    x = np.zeros((c.n, c.d))
    x[np.repeat(np.arange(c.n), np.diff(c.row_ptr)), c.col] = c.val
    s = x.sum(0)
    np.testing.assert_allclose(tr.final.dense()[0], s / np.linalg.norm(s), rtol=1e-13)
    assert tr.converged and tr.iters == 2 and tr.moved == [300, 0]


def test_empty_cluster_keeps_previous_centroid():
    # D = 1: every object and centroid is the same unit vector -> all a_i = 0,
    # clusters 1..k-1 empty and must keep their previous centroid bitwise
    c = corpus_from_rows([[0]] * 7, 1, 1.0)
    ids = [3, 1, 5]
    cents = oracle.init_centroids(c, ids)
    a, _, _ = oracle.assign(c, cents)
    assert a.tolist() == [0] * 7
    mu, counts = oracle.update(c, a, cents)
    assert counts.tolist() == [7, 0, 0]
    assert np.array_equal(mu.ptr, cents.ptr) and np.array_equal(mu.val, cents.val)


def test_k_equals_n_assigns_each_object_to_itself():
    c = synth.make_corpus(40, 30, 6, 1.0, np.float64, seed=5)
    ids = np.arange(40)
    a, _, top2 = oracle.assign(c, oracle.init_centroids(c, ids))
    # distinct unit rows: <x_i, x_i> > <x_i, x_j> (strict Cauchy-Schwarz) unless collinear
    dup = {}
    for i in range(c.n):
        key = tuple(c.col[c.row_ptr[i]:c.row_ptr[i + 1]])
        dup.setdefault(key, []).append(i)
    assert all(len(v) == 1 for v in dup.values())
    assert a.tolist() == list(range(40))


# --------------------------------------------------------------------------
# ICP: filtered == unfiltered, counts (Section 2.1 ICP; Alg. 3 vs Alg. 4)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_icp_filtered_equals_unfiltered_every_iteration(seed):
    c = synth.make_corpus(3000, 400, 20, 1.0, np.float64, seed=seed)
    ids = synth.init_ids(3000, 40, seed)
    t1 = oracle.lloyd(c, 40, ids, 25, icp=True)
    t0 = oracle.lloyd(c, 40, ids, 25, icp=False)
    assert t1.iters == t0.iters
    for r in range(t1.iters):
        assert np.array_equal(t1.assign[r], t0.assign[r])
        assert np.array_equal(t1.own[r], t0.own[r])  # cached own similarity is bit-exact
        assert t1.multadds[r] <= t0.multadds[r]
    assert sum(t1.multadds) < sum(t0.multadds)
    assert sum(int(l.sum()) for l in t1.lam) > 0  # some clusters became invariant


@pytest.mark.parametrize("seed", [3, 4])
def test_relaxed_icp_equals_unfiltered_every_iteration(seed):
    # Relaxed ICP (Section 2.1, after Bottesch et al.): an object whose own
    # centroid moved but got no less similar skips the invariant centroids.
    # Plain Lloyd's assignments (unfiltered, by definition) must not change,
    # the relaxed branch must occur, and it may only lower the count.
    c = synth.make_corpus(3000, 400, 20, 1.0, np.float64, seed=seed)
    ids = synth.init_ids(3000, 40, seed)
    t2 = oracle.lloyd(c, 40, ids, 25, icp=True, relaxed=True, keep_centroids=True)
    t1 = oracle.lloyd(c, 40, ids, 25, icp=True)
    t0 = oracle.lloyd(c, 40, ids, 25, icp=False)
    assert t2.iters == t0.iters
    for r in range(t2.iters):
        assert np.array_equal(t2.assign[r], t0.assign[r])
        assert np.array_equal(t2.own[r], t0.own[r])
        assert t2.multadds[r] <= t1.multadds[r]
        if r >= 1:
            # exactly the objects whose own cluster moved and whose FP64
            # similarity to it did not decrease take the relaxed branch
            a_prev = t2.assign[r - 1]
            moving_own = t2.lam[r - 1][a_prev] == 0
            now = oracle.pair_sims(c, t2.centroids[r], np.arange(c.n), a_prev)
            want = moving_own & (now >= t2.own[r - 1])
            assert np.array_equal(t2.branch[r] == 2, want)
            assert np.array_equal(t2.branch[r] == 1, ~moving_own)
    assert sum(int((b == 2).sum()) for b in t2.branch) > 0
    assert sum(t2.multadds) < sum(t1.multadds)


def test_sivf_and_cbicp_counts_equal_and_not_above_ivf():
    c = synth.make_corpus(2000, 300, 15, 1.0, np.float64, seed=9)
    ids = synth.init_ids(2000, 30, 9)
    tr = oracle.lloyd(c, 30, ids, 8, icp=True, keep_centroids=True)
    for r in range(1, tr.iters):
        lam_prev, a_prev = tr.lam[r - 1], tr.assign[r - 1]
        ivf = oracle.build_ivf(tr.centroids[r], lam_prev)
        kw = dict(icp=True, lam_prev=lam_prev, a_prev=a_prev)
        m_sivf = oracle.multadds(c, ivf, mode=oracle.MODE_SIVF, **kw)
        m_cb = oracle.multadds(c, ivf, mode=oracle.MODE_CBICP, **kw)
        m_ivf = oracle.multadds(c, ivf, mode=oracle.MODE_IVF, **kw)
        assert m_sivf == m_cb == tr.multadds[r]
        assert m_sivf <= m_ivf


def test_converged_iteration_costs_zero_multadds():
    c = synth.make_corpus(500, 100, 10, 1.0, np.float64, seed=13)
    ids = synth.init_ids(500, 6, 13)
    tr = oracle.lloyd(c, 6, ids, 200, icp=True)
    assert tr.converged
    # once every flag is set, the ICP bound of every list is zero (Section 4)
    lam_all = np.ones(6, dtype=np.uint8)
    ivf = oracle.build_ivf(tr.final, lam_all)
    assert oracle.multadds(c, ivf, icp=True, lam_prev=lam_all, a_prev=tr.assign[-1]) == 0


# --------------------------------------------------------------------------
# objective is monotone across both half steps (Section 1, Lloyd)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [4, 5])
def test_objective_monotone(seed):
    c = synth.make_corpus(1500, 200, 15, 1.0, np.float64, seed=seed)
    ids = synth.init_ids(1500, 20, seed)
    tr = oracle.lloyd(c, 20, ids, 12, icp=True, keep_centroids=True)
    prev = None
    for r in range(tr.iters):
        mu = tr.centroids[r]
        f_assign = oracle.objective(c, mu, tr.assign[r])
        if r > 0:
            f_before = oracle.objective(c, mu, tr.assign[r - 1])
            assert f_assign >= f_before  # exact on computed values
            assert f_before >= prev - 1e-12 * abs(prev)  # update half-step
        prev = f_assign


# --------------------------------------------------------------------------
# restart between iterations (Alg. 1): the state after an update is the
# centroids and the last two assignments; continuing from it must reproduce
# the uninterrupted run bitwise (assignments, cached own similarities, flags,
# counts, centroids)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("r_done", [1, 2, 5])
def test_resume_reproduces_the_trajectory(r_done):
    c = synth.make_corpus(1200, 300, 14, 1.0, np.float64, seed=21)
    ids = synth.init_ids(1200, 30, 22)
    full = oracle.lloyd(c, 30, ids, 12, icp=True, keep_centroids=True)
    assert full.iters > r_done + 2
    cents = full.centroids[r_done]          # mu^[r_done]: what assignment r_done + 1 reads
    a2 = full.assign[r_done - 2] if r_done >= 2 else None
    st = oracle.resume_state(c, cents, full.assign[r_done - 1], a2)
    assert np.array_equal(st.lam, full.lam[r_done - 1])
    # own similarities of the ICP objects equal the cached ones bitwise
    # (their centroid did not move, and the fold is the assignment's)
    icp = st.lam[st.a] == 1
    assert np.array_equal(st.own[icp].view(np.uint64), full.own[r_done - 1][icp].view(np.uint64))
    st.r = r_done
    res = oracle.lloyd(c, 30, None, 12, icp=True, keep_centroids=True, start=st)
    assert res.iters == full.iters and len(res.assign) == full.iters - r_done
    for q, r in enumerate(range(r_done + 1, full.iters + 1)):
        assert np.array_equal(res.assign[q], full.assign[r - 1]), r
        assert np.array_equal(res.own[q].view(np.uint64), full.own[r - 1].view(np.uint64)), r
        assert np.array_equal(res.lam[q], full.lam[r - 1]), r
        assert res.multadds[q] == full.multadds[r - 1], r
        assert res.moved[q] == full.moved[r - 1], r
    assert np.array_equal(res.final.val.view(np.uint64), full.final.val.view(np.uint64))


def test_resume_without_flags_is_not_a_restart():
    """A restart that forgets the flags (treats every cluster as moving) still
    gives the same assignments -- the ICP filter only skips comparisons -- but
    more mult-adds: the counts pin that the flags are part of the state."""
    c = synth.make_corpus(1200, 300, 14, 1.0, np.float64, seed=23)
    ids = synth.init_ids(1200, 30, 24)
    full = oracle.lloyd(c, 30, ids, 10, icp=True, keep_centroids=True)
    r_done = 4
    st = oracle.resume_state(c, full.centroids[r_done], full.assign[r_done - 1], full.assign[r_done - 2])
    assert st.lam.sum() > 0
    st.lam = np.zeros_like(st.lam)
    st.r = r_done
    res = oracle.lloyd(c, 30, None, r_done + 1, icp=True, start=st)
    assert np.array_equal(res.assign[0], full.assign[r_done])
    assert res.multadds[0] > full.multadds[r_done]


def test_relaxed_icp_cannot_resume():
    c = synth.make_corpus(200, 50, 6, 1.0, np.float64, seed=25)
    ids = synth.init_ids(200, 5, 26)
    full = oracle.lloyd(c, 5, ids, 3, icp=True, keep_centroids=True)
    st = oracle.resume_state(c, full.centroids[2], full.assign[1], full.assign[0])
    with pytest.raises(ValueError):
        oracle.lloyd(c, 5, None, 5, icp=True, relaxed=True, start=st)


# --------------------------------------------------------------------------
# structured inverted file (Section 4, Alg. 5)
# --------------------------------------------------------------------------
def test_ivf_layout_and_roundtrip():
    c = synth.make_corpus(800, 120, 12, 1.0, np.float64, seed=17)
    ids = synth.init_ids(800, 25, 3)
    cents = oracle.init_centroids(c, ids)
    mu, _ = oracle.update(c, oracle.assign(c, cents)[0], cents)
    lam = (np.arange(25) % 3 == 0).astype(np.uint8)
    ivf = oracle.build_ivf(mu, lam)
    assert ivf.term_ptr[-1] == len(mu.val)
    back = {}
    for s in range(mu.d):
        lo, mid, hi = ivf.term_ptr[s], ivf.term_ptr[s] + ivf.split[s], ivf.term_ptr[s + 1]
        front, rear = ivf.cid[lo:mid], ivf.cid[mid:hi]
        assert np.all(lam[front] == 0) and np.all(lam[rear] == 1)
        assert np.all(np.diff(front) > 0) and np.all(np.diff(rear) > 0)
        assert ivf.split[s] == sum(1 for j in range(25) if lam[j] == 0 and s in
                                   set(mu.col[mu.ptr[j]:mu.ptr[j + 1]].tolist()))
        for q in range(lo, hi):
            back[(int(ivf.cid[q]), s)] = ivf.val[q]
    for j in range(25):
        for p in range(mu.ptr[j], mu.ptr[j + 1]):
            assert back.pop((j, int(mu.col[p]))) == mu.val[p]
    assert not back


# --------------------------------------------------------------------------
# soft assignment: closed forms and finite differences
# --------------------------------------------------------------------------
def _soft_case(seed=3, n=30, d=20, k=7):
    c = synth.make_corpus(n, d, 6, 1.0, np.float64, seed=seed)
    rng = np.random.default_rng(seed)
    C = np.abs(rng.standard_normal((k, d)))
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    return c, C


def _dense_x(c):
    x = np.zeros((c.n, c.d))
    x[np.repeat(np.arange(c.n), np.diff(c.row_ptr)), c.col] = c.val
    return x


def test_soft_forward_matches_scipy_logsumexp():
    from scipy.special import logsumexp
    c, C = _soft_case()
    tau = 0.05
    lse = oracle.soft_forward(c, C, tau)
    S = _dense_x(c) @ C.T
    np.testing.assert_allclose(lse, logsumexp(S / tau, axis=1), rtol=1e-13)


def test_soft_backward_finite_differences():
    c, C = _soft_case()
    tau, g = 0.05, 1.0
    lse = oracle.soft_forward(c, C, tau)
    dC, dX = oracle.soft_backward(c, C, tau, g, lse)

    def loss(Cm, vals):
        cc = synth.Corpus(c.n, c.d, c.row_ptr, c.col, vals)
        return -math.fsum(oracle.soft_forward(cc, Cm, tau).tolist())

    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(8):
        j, t = rng.integers(C.shape[0]), rng.integers(c.d)
        Cp, Cm = C.copy(), C.copy()
        Cp[j, t] += h
        Cm[j, t] -= h
        fd = (loss(Cp, c.val) - loss(Cm, c.val)) / (2 * h)
        assert abs(fd - dC[j, t]) <= 1e-5 * max(1.0, abs(fd))
    for p in rng.integers(0, c.nnz, 8):
        vp, vm = c.val.copy(), c.val.copy()
        vp[p] += h
        vm[p] -= h
        fd = (loss(C, vp) - loss(C, vm)) / (2 * h)
        assert abs(fd - dX[p]) <= 1e-5 * max(1.0, abs(fd))


def test_soft_backward_closed_form_identities():
    c, C = _soft_case(seed=8, n=60, d=25, k=9)
    tau, g = 0.05, 0.7
    lse = oracle.soft_forward(c, C, tau)
    dC, dX = oracle.soft_backward(c, C, tau, g, lse)
    x = _dense_x(c)
    S = x @ C.T
    P = np.exp(S / tau - lse[:, None])
    # sum_j P_ij = 1  =>  sum_j dC_j = -(g / tau) sum_i x_i
    np.testing.assert_allclose(dC.sum(0), -(g / tau) * x.sum(0), rtol=1e-10, atol=1e-10)
    # Euler homogeneity in x_i: sum_t dX_it x_it = -(g/tau) sum_j P_ij S_ij
    rows = np.repeat(np.arange(c.n), np.diff(c.row_ptr))
    lhs = np.bincount(rows, weights=dX * c.val, minlength=c.n)
    np.testing.assert_allclose(lhs, -(g / tau) * (P * S).sum(1), rtol=1e-10, atol=1e-12)
    # and in C: sum_{j,t} dC_jt C_jt = -(g/tau) sum_ij P_ij S_ij
    assert abs((dC * C).sum() + (g / tau) * (P * S).sum()) < 1e-9 * abs((P * S).sum() / tau)


def test_soft_small_tau_limit_is_hard_assignment():
    c, C = _soft_case(seed=12, n=40, d=30, k=6)
    # rows of C as centroids in CSR form
    k, d = C.shape
    cents = oracle.Centroids(k, d, np.arange(0, k * d + 1, d, dtype=np.int64),
                             np.tile(np.arange(d, dtype=np.int32), k), C.ravel().copy())
    a, own, _ = oracle.assign(c, cents)
    lse = oracle.soft_forward(c, C, 1e-4)
    # tau -> 0: tau * lse -> max_j S_ij
    np.testing.assert_allclose(1e-4 * lse, own, atol=1e-4 * math.log(k) + 1e-12)
