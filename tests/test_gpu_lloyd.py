"""GPU parity: the HIP path through the C ABI against the FP64 oracle, step by
step (assignments bit-exact, flags and mult-add counts equal, FP64 centroids
and the structured file bitwise equal)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import device, log, lloyd_parity
from tests.util import corpus_from_rows

pytestmark = pytest.mark.gpu


def _ctx(**kw):
    from paper_2103_16141_amd.api import Context
    return Context(0, **kw)


def _X(corpus):
    from paper_2103_16141_amd.api import DeviceCsr
    return DeviceCsr.from_corpus(corpus, device())


@pytest.mark.parametrize("k_tile,posting", [(0, "fp32"), (64, "fp32"), (64, "bf16")])
def test_small_f64_trajectory(k_tile, posting):
    log("small f64 trajectory k_tile=%d posting=%s" % (k_tile, posting))
    c = synth.make_corpus(3000, 900, 25, 1.0, np.float64, seed=101)
    ids = synth.init_ids(3000, 150, 7)  # 150 = 64 + 64 + 22: several tiles with a ragged tail
    ctx = _ctx(k_tile=k_tile, posting_dtype=posting)
    tr, st = lloyd_parity(ctx, _X(c), c, 150, ids, 12)
    assert tr.iters >= 5


@pytest.mark.parametrize("mode", ["sivf", "ivf", "cbicp", "relaxed"])
def test_filter_modes_same_assignments(mode):
    log("filter mode %s" % mode)
    c = synth.make_corpus(2500, 700, 20, 1.0, np.float64, seed=102)
    ids = synth.init_ids(2500, 90, 8)
    ctx = _ctx(k_tile=64, filter_mode=mode)
    lloyd_parity(ctx, _X(c), c, 90, ids, 15, mode=mode)


def test_small_config_f64_k100_ten_iterations():
    # N=10,000, D=5,000, Poisson(50), Zipf 1.0, f64, k=100, 10 iterations with ICP
    log("N=10k D=5k k=100 f64")
    c, ids, w = synth.workload("small-f64")
    for kt in (0, 64):
        lloyd_parity(_ctx(k_tile=kt), _X(c), c, w["k"], ids, w["iters"])


def test_mid_f32_trajectory():
    log("N=40k D=20k k=300 f32")
    c = synth.make_corpus(40000, 20000, 60, 1.1, np.float32, seed=103)
    ids = synth.init_ids(40000, 300, 9)
    lloyd_parity(_ctx(k_tile=128), _X(c), c, 300, ids, 8, check_ivf_every=3)


def test_bf16_matches_fp32_trajectory_and_counts():
    log("bf16 vs fp32 counts")
    c = synth.make_corpus(20000, 8000, 40, 1.1, np.float32, seed=104)
    ids = synth.init_ids(20000, 200, 10)
    _, s32 = lloyd_parity(_ctx(posting_dtype="fp32"), _X(c), c, 200, ids, 8, check_ivf_every=4)
    _, s16 = lloyd_parity(_ctx(posting_dtype="bf16"), _X(c), c, 200, ids, 8, check_ivf_every=4)
    assert [s["multadds"] for s in s32] == [s["multadds"] for s in s16]
    assert sum(s["rescored_objects"] for s in s16) >= sum(s["rescored_objects"] for s in s32)


# --------------------------------------------------------------------- edge cases
def test_empty_rows_k1_and_duplicates():
    log("edge: empty rows, duplicates, k=1")
    rows = [[0, 3], [], [1, 2, 3], [0, 3], [], [2], [0, 1, 2, 3], [0, 3]]
    vals = [[0.6, 0.8], [], [0.5, 0.5, 0.7071067811865476], [0.6, 0.8], [], [1.0], [0.5] * 4, [0.6, 0.8]]
    c = corpus_from_rows(rows, 4, vals)
    lloyd_parity(_ctx(), _X(c), c, 3, [0, 3, 7], 6)   # three identical seeds: exact ties
    lloyd_parity(_ctx(), _X(c), c, 1, [2], 4)
    lloyd_parity(_ctx(), _X(c), c, 8, list(range(8)), 4)


def test_single_term_dimension():
    log("edge: D=1")
    c = corpus_from_rows([[0]] * 9, 1, 1.0)
    lloyd_parity(_ctx(), _X(c), c, 4, [3, 1, 5, 0], 4)


def test_signed_values_use_the_absolute_bound():
    log("edge: signed values")
    c = synth.make_corpus(1500, 300, 15, 1.0, np.float64, seed=105)
    rng = np.random.default_rng(0)
    c.val *= np.where(rng.random(c.nnz) < 0.3, -1.0, 1.0)
    ids = synth.init_ids(1500, 70, 11)
    lloyd_parity(_ctx(k_tile=64), _X(c), c, 70, ids, 8)


def test_long_rows_over_64_terms():
    log("edge: rows longer than 64 terms")
    c = synth.make_corpus(2000, 3000, 150, 0.8, np.float32, seed=106)
    ids = synth.init_ids(2000, 80, 12)
    lloyd_parity(_ctx(k_tile=64), _X(c), c, 80, ids, 6)


def test_rows_longer_than_the_staged_terms():
    # rows of ~300 terms: the walk reads terms past the 128 it stages in LDS
    # from X, and the update reads nonzeros past the 256 it holds in registers
    # chunk by chunk
    log("edge: rows longer than 256 terms")
    c = synth.make_corpus(1500, 4000, 300, 0.9, np.float32, seed=111)
    assert np.diff(c.row_ptr).max() > 256
    ids = synth.init_ids(1500, 60, 17)
    for posting in ("fp32", "bf16"):
        lloyd_parity(_ctx(k_tile=64, posting_dtype=posting, head_density=0.3), _X(c), c, 60, ids, 6)


def test_run_lloyd_matches_stepwise_and_is_deterministic():
    log("run_lloyd determinism")
    c = synth.make_corpus(8000, 3000, 30, 1.1, np.float32, seed=107)
    ids = synth.init_ids(8000, 120, 13)
    X = _X(c)
    ctx = _ctx()
    a1, own1, ivf1, st1 = ctx.run_lloyd(X, 120, ids, 20)
    a2, own2, ivf2, st2 = ctx.run_lloyd(X, 120, ids, 20)
    assert torch.equal(a1, a2) and torch.equal(own1, own2)
    e1, e2 = ivf1.export(), ivf2.export()
    for key in e1:
        assert torch.equal(e1[key], e2[key]), key
    tr = oracle.lloyd(c, 120, ids, 20, icp=True)
    assert len(st1) == tr.iters
    assert np.array_equal(a1.cpu().numpy(), tr.assign[-1])
    assert [s["multadds"] for s in st1] == tr.multadds
    # the module-level convenience call: same assignments, centroids as CSR
    from paper_2103_16141_amd import run_lloyd
    for precision, icp in (("bf16", True), ("fp32", False)):
        a3, C3, st3 = run_lloyd(X, 120, ids, 20, icp=icp, precision=precision)
        assert np.array_equal(a3.cpu().numpy(), tr.assign[-1])
        assert len(st3) == tr.iters
        assert torch.equal(C3.row_ptr, e1["c_ptr"]) and torch.equal(C3.col, e1["c_col"])
        assert torch.equal(C3.val, e1["c_val"]) and C3.n_cols == c.d


@pytest.mark.parametrize("posting", ["fp32", "bf16"])
@pytest.mark.parametrize("k,k_tile", [(200, 0), (600, 512), (1100, 1024), (700, 576), (1300, 1280)])
def test_dense_head_rows_same_trajectory(posting, k, k_tile):
    # Dense head rows for terms held by >= 10% or by all centroids, or none at
    # all: every variant matches the oracle step by step (assignments, flags,
    # mult-add counts, centroids), and the rows are really read when enabled.
    # Rows are read in 512-centroid batches: tiles of 512 and 1024 take whole
    # batches, 256 (automatic for k = 200), 576 and 1280 end in a batch that
    # is partly outside the tile.
    log("dense head rows posting=%s k=%d k_tile=%d" % (posting, k, k_tile))
    c = synth.make_corpus(20000, 3000, 40, 1.1, np.float32, seed=104)
    ids = synth.init_ids(20000, k, 10)
    rows = {}
    for hd in (0.0, 0.1, 1.0):
        ctx = _ctx(k_tile=k_tile, posting_dtype=posting, head_density=hd)
        tr, st = lloyd_parity(ctx, _X(c), c, k, ids, 6)
        rows[hd] = [s["head_rows"] for s in st]
        ctx.close()
    assert all(r == 0 for r in rows[0.0])
    assert max(rows[0.1]) > 0
    assert all(a >= b for a, b in zip(rows[0.1], rows[1.0]))


@pytest.mark.parametrize("posting", ["fp32", "bf16"])
def test_widest_tile_full_length_segments(posting):
    # The largest tile (4096 centroids) and a term every object holds: its
    # list segment in a tile is as long as the tile, the longest a segment
    # record describes.  k = 4500 leaves a ragged second tile of 404.  Lists
    # only (no dense rows) and with dense rows.
    log("widest tile, full-length segments, posting=%s" % posting)
    c0 = synth.make_corpus(9000, 800, 12, 1.0, np.float32, seed=109)
    rows, vals = [], []
    for i in range(c0.n):
        t = c0.col[c0.row_ptr[i]:c0.row_ptr[i + 1]].tolist()
        v = c0.val[c0.row_ptr[i]:c0.row_ptr[i + 1]].astype(np.float64)
        if t[0] != 0:
            t = [0] + t
            v = np.concatenate([[0.3], v])
        v = v / np.linalg.norm(v)
        rows.append(t)
        vals.append(v.astype(np.float32).tolist())
    c = corpus_from_rows(rows, c0.d, vals, np.float32)
    ids = synth.init_ids(c.n, 4500, 15)
    for hd in (0.0, 0.5):
        ctx = _ctx(k_tile=4096, posting_dtype=posting, head_density=hd)
        tr, st = lloyd_parity(ctx, _X(c), c, 4500, ids, 4)
        assert (max(s["head_rows"] for s in st) > 0) == (hd > 0)
        ctx.close()


def test_more_than_65536_centroids():
    # k = 70,000: 69 tiles of 1024 (centroid ids are 16-bit and tile-local,
    # so the file holds any k); most clusters have one or two members.
    log("k = 70,000")
    c = synth.make_corpus(75000, 4000, 8, 1.0, np.float32, seed=112)
    ids = synth.init_ids(c.n, 70000, 18)
    tr, st = lloyd_parity(_ctx(), _X(c), c, 70000, ids, 2, check_ivf_every=2)
    assert tr.iters == 2


@pytest.mark.parametrize("posting", ["fp32", "bf16"])
def test_moving_prefix_tiles(posting):
    # The file numbers the moving centroids first: objects in the ICP branch
    # read the moving prefix of each tile and skip the tiles past it.  k = 300
    # in 64-centroid tiles: 85% of the clusters are invariant by iteration 6,
    # so most launches are past the prefix and the boundary moves inside a
    # tile.  k = 5,000 in one 4096-centroid tile and a ragged one: 542 moving
    # centroids at iteration 3, then fewer than one 512-centroid batch.  With
    # head rows and without, one tile per launch and all in one launch, the
    # runs match the oracle step by step (the exported file is compared in
    # centroid ids).
    log("moving-prefix tiles posting=%s" % posting)
    for (n, d, lam, k, kt, it, seed) in ((6000, 1500, 25, 300, 64, 14, 113), (20000, 3000, 30, 5000, 4096, 6, 115)):
        c = synth.make_corpus(n, d, lam, 1.0, np.float32, seed=seed)
        ids = synth.init_ids(c.n, k, 19)
        for hd, tpl in ((0.2, 0), (0.0, 0), (0.2, 64)):
            ctx = _ctx(k_tile=kt, posting_dtype=posting, head_density=hd, tiles_per_launch=tpl)
            tr, st = lloyd_parity(ctx, _X(c), c, k, ids, it, check_ivf_every=3)
            assert sum(s["icp_objects"] for s in st) > 0
            assert (max(s["head_rows"] for s in st) > 0) == (hd > 0)
            ctx.close()


@pytest.mark.parametrize("tiles_per_launch", [1, 2, 64])
def test_tile_launch_split_with_ties_and_overflow(tiles_per_launch):
    # 100 identical seeds spread over five 64-centroid tiles: objects near them
    # carry more than kCandCap candidates across tile launches (overflow, then
    # the FP64 re-score over all eligible centroids with lowest-index ties).
    # One tile per launch, two, or all five in one launch: identical runs.
    log("tile launches: %d tiles per launch" % tiles_per_launch)
    c = synth.make_corpus(3000, 500, 20, 1.0, np.float64, seed=108)
    rows = [c.col[c.row_ptr[i]:c.row_ptr[i + 1]] for i in range(c.n)]
    vals = [c.val[c.row_ptr[i]:c.row_ptr[i + 1]] for i in range(c.n)]
    for i in range(1, 100):
        rows[i], vals[i] = rows[0], vals[0]
    c2 = corpus_from_rows(rows, c.d, vals)
    ids = list(range(100)) + [int(x) for x in synth.init_ids(2900, 200, 14) + 100]
    ctx = _ctx(k_tile=64, tiles_per_launch=tiles_per_launch)
    tr, st = lloyd_parity(ctx, _X(c2), c2, 300, ids, 6)
    assert sum(s["full_rescored"] for s in st) > 0


@pytest.mark.parametrize("posting", ["fp32", "bf16"])
def test_icp_objects_reading_head_rows(posting):
    # Objects in the ICP branch read the moving prefix of the dense head rows
    # (head rows at 0.2 or 0.05 of the centroids) or walk every term's list
    # (none): identical trajectories, flags and mult-add counts.
    log("ICP objects and head rows, posting=%s" % posting)
    c = synth.make_corpus(20000, 3000, 40, 1.1, np.float32, seed=110)
    ids = synth.init_ids(20000, 400, 16)
    icp_seen = 0
    for hd in (0.2, 0.05, 0.0):
        ctx = _ctx(k_tile=128, posting_dtype=posting, head_density=hd)
        tr, st = lloyd_parity(ctx, _X(c), c, 400, ids, 12, check_ivf_every=4)
        icp_seen = max(icp_seen, sum(s["icp_objects"] for s in st))
        ctx.close()
    assert icp_seen > 0


@pytest.mark.parametrize("posting,tiles_per_launch", [("fp32", 0), ("bf16", 0), ("fp32", 64)])
def test_relaxed_icp_trajectory(posting, tiles_per_launch):
    # Relaxed ICP (Section 2.1): objects whose own centroid moved but got no
    # less similar (exact FP64) skip invariant centroids.  Assignments, flags,
    # mult-add counts and centroids match the oracle's relaxed run step by
    # step; the branch is taken; one launch per tile or all tiles at once.
    log("relaxed ICP posting=%s tiles_per_launch=%d" % (posting, tiles_per_launch))
    c = synth.make_corpus(20000, 3000, 40, 1.1, np.float32, seed=112)
    ids = synth.init_ids(20000, 300, 18)
    ctx = _ctx(k_tile=128, posting_dtype=posting, filter_mode="relaxed", tiles_per_launch=tiles_per_launch)
    tr, st = lloyd_parity(ctx, _X(c), c, 300, ids, 12, mode="relaxed", check_ivf_every=4)
    assert sum(s["relaxed_objects"] for s in st) > 0
    assert [s["relaxed_objects"] for s in st] == [int((b == 2).sum()) for b in tr.branch[:len(st)]]


@pytest.mark.parametrize("posting,mode,tiles_per_launch,signed", [("fp32", "sivf", 0, False), ("bf16", "sivf", 0, False),
                                                                 ("fp32", "sivf", 64, False),
                                                                 ("fp32", "cbicp", 0, False), ("fp32", "sivf", 0, True)])
def test_flag_patterns_on_a_built_file(posting, mode, tiles_per_launch, signed):
    # The file numbers the moving centroids first.  A file built from given
    # centroids under chosen flags -- no moving centroid, all moving, one
    # moving, alternating, a boundary inside a tile, random -- then one ICP
    # assignment step: assignments, output flags and the mult-add count equal
    # the oracle's, and the exported file (in centroid ids) equals the
    # oracle's structured file.  k = 200 in tiles of 64, 64, 64 and 8.  The
    # centroids are those after one update and the previous assignment that
    # of the initial ones, so the restriction to moving centroids changes the
    # result (147 to 743 objects end elsewhere than under the full argmax).
    # Signed values take the bound through each centroid's norm, looked up by
    # centroid id from the position.
    log("flag patterns posting=%s mode=%s tiles_per_launch=%d signed=%s" % (posting, mode, tiles_per_launch, signed))
    c = synth.make_corpus(4000, 1200, 25, 1.0, np.float32, seed=117)
    if signed:
        c.val *= np.where(np.random.default_rng(1).random(c.nnz) < 0.3, -1.0, 1.0).astype(c.val.dtype)
    k = 200
    a0, _, _ = oracle.assign(c, oracle.init_centroids(c, synth.init_ids(c.n, k, 21)))
    cents, _ = oracle.update(c, a0, oracle.init_centroids(c, synth.init_ids(c.n, k, 21)))
    own0 = oracle.pair_sims(c, cents, np.arange(c.n), a0)   # exact similarity to the own centroid now
    rng = np.random.default_rng(5)
    patterns = {
        "none moving": np.ones(k, np.uint8),
        "all moving": np.zeros(k, np.uint8),
        "one moving": np.r_[np.ones(k - 1, np.uint8), np.zeros(1, np.uint8)],
        "one invariant": np.r_[np.ones(1, np.uint8), np.zeros(k - 1, np.uint8)],
        "alternating": (np.arange(k) % 2).astype(np.uint8),
        "first 150 invariant": (np.arange(k) < 150).astype(np.uint8),
        "random 70% invariant": (rng.random(k) < 0.7).astype(np.uint8),
    }
    X = _X(c)
    dev = device()
    ctx = _ctx(k_tile=64, posting_dtype=posting, head_density=0.2, filter_mode=mode,
               tiles_per_launch=tiles_per_launch)
    for name, lam in patterns.items():
        log("  pattern: %s" % name)
        ivf = ctx.build_centroid_ivf(torch.from_numpy(cents.ptr.astype(np.int64)).to(dev),
                                     torch.from_numpy(cents.col.astype(np.int32)).to(dev),
                                     torch.from_numpy(cents.val.astype(np.float64)).to(dev), c.d,
                                     torch.from_numpy(lam).to(dev))
        ex = ivf.export()
        ref_ivf = oracle.build_ivf(cents, lam)
        assert np.array_equal(ex["term_ptr"].cpu().numpy(), ref_ivf.term_ptr), name
        assert np.array_equal(ex["split"].cpu().numpy(), ref_ivf.split), name
        assert np.array_equal(ex["p_cid"].cpu().numpy(), ref_ivf.cid), name
        assert np.array_equal(ex["p_val"].cpu().numpy(), ref_ivf.val), name
        a = torch.from_numpy(a0.astype(np.int32)).to(dev)
        own = torch.from_numpy(own0.astype(np.float32)).to(dev)
        lam_out = torch.empty(k, dtype=torch.uint8, device=dev)
        st = ctx.assign(X, ivf, 2, a, own, lam_out)
        ref_a, _, _ = oracle.assign(c, cents, icp=True, lam_prev=lam, a_prev=a0, own_prev=own0)
        got = a.cpu().numpy()
        assert np.array_equal(got, ref_a), "%s: %d assignments differ" % (name, int((got != ref_a).sum()))
        assert np.array_equal(lam_out.cpu().numpy(), oracle.mark_invariant(a0, ref_a, k, False)[0]), name
        m_ref = oracle.multadds(c, ref_ivf, icp=True, lam_prev=lam, a_prev=a0,
                                mode=oracle.MODE_CBICP if mode == "cbicp" else oracle.MODE_SIVF)
        assert st["multadds"] == m_ref, "%s: multadds %d vs %d" % (name, st["multadds"], m_ref)
        assert st["icp_objects"] == int(lam[a0].astype(bool).sum()), name
        ivf.free()
    ctx.close()


@pytest.mark.parametrize("posting", ["fp32", "bf16"])
def test_every_term_dense(posting):
    """Full-expression centroids (the paper's Lloyd-ICP baseline, Section 3.1
    and Section 5): with head_density near 0 every term held by any centroid
    gets a dense row, so the walk multiplies objects against dense centroids
    and reads no structured list; ICP objects read the moving prefix of each
    row.  Same trajectory and counts as the structured file."""
    log("every term dense, %s postings" % posting)
    c = synth.make_corpus(4000, 1500, 30, 1.0, np.float32, seed=141)
    ids = synth.init_ids(4000, 150, 41)
    tr, st = lloyd_parity(_ctx(k_tile=64, posting_dtype=posting, head_density=1e-6), _X(c), c, 150, ids, 8)
    used = np.unique(c.col).size
    assert st[0]["head_rows"] == np.unique(np.concatenate(
        [c.col[c.row_ptr[i]:c.row_ptr[i + 1]] for i in ids])).size
    assert all(0 < s["head_rows"] <= used for s in st)
    assert sum(s["icp_objects"] for s in st) > 0
