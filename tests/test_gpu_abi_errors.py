"""Every status the boundary reports, forced from the host, and outputs left
untouched on validation errors.  Validation itself runs on the device, so
these tests need the GPU; no case makes a kernel fault: invalid inputs are
rejected before any kernel indexes with them."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import device, log
from tests.util import corpus_from_rows

pytestmark = pytest.mark.gpu


def _ctx(**kw):
    from paper_2103_16141_amd.api import Context
    return Context(0, **kw)


def _X(c):
    from paper_2103_16141_amd.api import DeviceCsr
    return DeviceCsr.from_corpus(c, torch.device("cuda", 0))


def _status(fn):
    from paper_2103_16141_amd._native import SivfError
    with pytest.raises(SivfError) as e:
        fn()
    return e.value.name


def _good():
    return synth.make_corpus(200, 100, 8, 1.0, np.float32, seed=1)


def test_invalid_csr_statuses():
    log("abi errors: csr")
    ctx = _ctx()
    c = _good()
    bad = _good()
    bad.col = bad.col.copy()
    r = int(np.argmax(np.diff(bad.row_ptr) >= 2))
    a = bad.row_ptr[r]
    bad.col[a], bad.col[a + 1] = bad.col[a + 1], bad.col[a]       # unsorted row
    assert _status(lambda: ctx.validate(_X(bad))) == "SIVF_E_UNSORTED"
    rng = _good()
    rng.col = rng.col.copy()
    rng.col[rng.row_ptr[3 + 1] - 1] = rng.d + 5                   # column out of range (last in its row)
    assert _status(lambda: ctx.validate(_X(rng))) == "SIVF_E_RANGE"
    nan = _good()
    nan.val = nan.val.copy()
    nan.val[17] = np.nan
    assert _status(lambda: ctx.validate(_X(nan))) == "SIVF_E_NONFINITE"
    ok = _X(c)
    ctx.validate(ok)
    assert _status(lambda: ctx.init_centroids(ok, 0, [])) == "SIVF_E_SHAPE"
    assert _status(lambda: ctx.init_centroids(ok, 201, list(range(201)))) == "SIVF_E_SHAPE"
    assert _status(lambda: ctx.init_centroids(ok, 2, [0, 999])) == "SIVF_E_RANGE"


def test_outputs_untouched_on_error():
    log("abi errors: outputs untouched")
    from paper_2103_16141_amd.api import DeviceCsr
    ctx = _ctx()
    c = _good()
    X = _X(c)
    ivf = ctx.init_centroids(X, 5, [0, 1, 2, 3, 4])
    a = torch.full((c.n,), 7, dtype=torch.int32, device="cuda")   # 7 >= k: invalid a^[r-1]
    own = torch.full((c.n,), 0.25, dtype=torch.float32, device="cuda")
    lam = torch.full((5,), 9, dtype=torch.uint8, device="cuda")
    assert _status(lambda: ctx.assign(X, ivf, 2, a, own, lam)) == "SIVF_E_RANGE"
    assert bool((a == 7).all()) and bool((own == 0.25).all()) and bool((lam == 9).all())
    assert _status(lambda: ctx.update(X, a, lam, ivf)) == "SIVF_E_RANGE"
    # column-count mismatch
    c2 = synth.make_corpus(50, 60, 8, 1.0, np.float32, seed=2)
    X2 = DeviceCsr.from_corpus(c2, torch.device("cuda", 0))
    a2 = torch.zeros(c2.n, dtype=torch.int32, device="cuda")
    own2 = torch.zeros(c2.n, dtype=torch.float32, device="cuda")
    assert _status(lambda: ctx.assign(X2, ivf, 1, a2, own2, lam)) == "SIVF_E_SHAPE"
    assert bool((lam == 9).all())
    # a valid call after the errors still works
    st = ctx.assign(X, ivf, 1, a, own, lam)
    assert st["moved"] == c.n and int(a.max()) < 5


def test_null_pointers_and_bad_options():
    from paper_2103_16141_amd import _native as N
    lib = N.load()
    h = ctypes.c_void_p()
    opt = N.sivf_options()
    lib.sivf_default_options(ctypes.byref(opt))
    opt.k_tile = 100                                              # not a multiple of 64
    assert lib.sivf_create(ctypes.byref(h), 0, None, ctypes.byref(opt)) == -1
    opt.k_tile = 0
    opt.posting_dtype = N.SIVF_F64                                # postings are f32 or bf16
    assert lib.sivf_create(ctypes.byref(h), 0, None, ctypes.byref(opt)) == -1
    lib.sivf_default_options(ctypes.byref(opt))
    assert lib.sivf_create(ctypes.byref(h), 999, None, None) == -7
    assert lib.sivf_create(None, 0, None, None) == -1
    ctx = _ctx()
    assert lib.sivf_validate_csr(ctx.handle, None) == -1
    assert b"NULL" in lib.sivf_last_error(ctx.handle)
    st = N.sivf_iter_stats()
    assert lib.sivf_assign(ctx.handle, None, None, 1, None, None, None, None, ctypes.byref(st)) == -1
    assert lib.sivf_destroy(None) == 0 and lib.sivf_ivf_free(ctx.handle, None) == 0


def test_workspace_cap_reports_nomem():
    log("abi errors: workspace cap")
    ctx = _ctx(workspace_cap_bytes=4096)
    c = _good()
    X = _X(c)
    assert _status(lambda: ctx.init_centroids(X, 5, [0, 1, 2, 3, 4])) == "SIVF_E_NOMEM"
    ctx2 = _ctx(workspace_cap_bytes=1 << 30)
    a, own, ivf, stats = ctx2.run_lloyd(X, 5, [0, 1, 2, 3, 4], 5)
    assert len(stats) >= 1


def test_relaxed_filter_needs_own64():
    log("abi errors: relaxed filter without own64")
    ctx = _ctx(filter_mode="relaxed")
    c = _good()
    X = _X(c)
    ivf = ctx.init_centroids(X, 5, [0, 1, 2, 3, 4])
    a = torch.zeros(c.n, dtype=torch.int32, device=device())
    own = torch.zeros(c.n, dtype=torch.float32, device=device())
    lam = torch.zeros(5, dtype=torch.uint8, device=device())
    assert _status(lambda: ctx.assign(X, ivf, 1, a, own, lam)) == "SIVF_E_INVALID"
    # with the state it runs, and run_lloyd keeps the state itself
    own64 = torch.zeros(c.n, dtype=torch.float64, device=device())
    ctx.assign(X, ivf, 1, a, own, lam, own64=own64)
    a2, own2, ivf2, stats = ctx.run_lloyd(X, 5, [0, 1, 2, 3, 4], 6)
    assert len(stats) >= 1


def test_empty_matrix_and_zero_rows():
    log("abi: empty X")
    ctx = _ctx()
    c = corpus_from_rows([[0], [1]], 3, 1.0, dtype=np.float32)
    X = _X(c)
    a, own, ivf, stats = ctx.run_lloyd(X, 2, [0, 1], 3)
    assert a.cpu().tolist() == [0, 1] and stats[-1]["moved"] == 0


def test_in_place_edits_are_validated_again():
    """X edited in place (same pointers, same sizes) after a successful call
    is checked again before any kernel indexes with it: an out-of-range
    column is rejected with the outputs untouched, and values whose sign
    changed switch the certificate to the signed-data bound, so the next
    assignment still equals the oracle's."""
    import oracle
    log("abi: in-place edits of a validated X")
    ctx = _ctx(k_tile=64)
    c = synth.make_corpus(3000, 600, 20, 1.0, np.float32, seed=9)
    X = _X(c)
    k = 70
    ids = synth.init_ids(c.n, k, 19)
    ivf = ctx.init_centroids(X, k, ids)
    a = torch.zeros(c.n, dtype=torch.int32, device=device())
    own = torch.zeros(c.n, dtype=torch.float32, device=device())
    lam = torch.zeros(k, dtype=torch.uint8, device=device())
    ctx.assign(X, ivf, 1, a, own, lam)
    a_ok = a.clone()
    # an out-of-range column written into the validated X
    p = int(c.row_ptr[1234 + 1] - 1)        # last entry of a row: still ascending
    saved = int(X.col[p])
    X.col[p] = c.d + 7
    a.fill_(3)
    assert _status(lambda: ctx.assign(X, ivf, 1, a, own, lam)) == "SIVF_E_RANGE"
    assert bool((a == 3).all())
    assert _status(lambda: ctx.update(X, a_ok, lam, ivf)) == "SIVF_E_RANGE"
    X.col[p] = saved
    # a duplicate column (unsorted row) written in place
    q = int(np.nonzero(np.diff(c.row_ptr) >= 3)[0][5])
    b0 = int(c.row_ptr[q])
    saved = int(X.col[b0 + 1])
    X.col[b0 + 1] = X.col[b0]
    assert _status(lambda: ctx.assign(X, ivf, 1, a, own, lam)) == "SIVF_E_UNSORTED"
    X.col[b0 + 1] = saved
    # signs flipped in place: the same file (nonnegative centroids) against
    # signed objects must use the absolute bound
    flip = torch.from_numpy(np.random.default_rng(4).random(c.nnz) < 0.35).to(device())
    X.val[flip] = -X.val[flip]
    ctx.assign(X, ivf, 1, a, own, lam)
    signed = synth.Corpus(c.n, c.d, c.row_ptr, c.col, X.val.cpu().numpy())
    ref, _, _ = oracle.assign(signed, oracle.init_centroids(c, ids))
    assert np.array_equal(a.cpu().numpy(), ref)


def test_validation_errors_at_group_edges():
    """The validator reads 64 rows per wave; errors in the first and last row
    of such a group, across a group boundary, and in the last row of X are all
    found and name their row."""
    log("abi: validation at row-group edges")
    ctx = _ctx()
    base = synth.make_corpus(300, 400, 9, 1.0, np.float32, seed=12)
    for row in (0, 63, 64, 127, 128, 299):
        for kind in ("range", "unsorted", "nan"):
            c = synth.Corpus(base.n, base.d, base.row_ptr, base.col.copy(), base.val.copy())
            b, e = int(c.row_ptr[row]), int(c.row_ptr[row + 1])
            assert e - b >= 2
            if kind == "range":
                c.col[e - 1] = c.d
            elif kind == "unsorted":
                c.col[b + 1] = c.col[b]
            else:
                c.val[b] = np.inf
            want = {"range": "SIVF_E_RANGE", "unsorted": "SIVF_E_UNSORTED", "nan": "SIVF_E_NONFINITE"}[kind]
            from paper_2103_16141_amd._native import SivfError
            with pytest.raises(SivfError) as err:
                ctx.validate(_X(c))
            assert err.value.name == want, (row, kind)
            assert ("row %d " % row) in str(err.value), (row, kind, str(err.value))
    # a row whose first column is below the previous row's last column is fine
    ctx.validate(_X(base))
    # row_ptr decreasing inside a group
    c = synth.Corpus(base.n, base.d, base.row_ptr.copy(), base.col, base.val)
    c.row_ptr[70] = c.row_ptr[71] + 1
    assert _status(lambda: ctx.validate(_X(c))) == "SIVF_E_UNSORTED"
