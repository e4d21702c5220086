"""Seeded generator: structure of the rows it writes (sorted unique terms, unit
norms, Poisson row lengths, Zipf rank-frequency, reproducibility)."""
import numpy as np

import synth


def test_rows_sorted_unique_unit_norm():
    c = synth.make_corpus(3000, 2000, 40, 1.0, np.float64, seed=7)
    assert c.row_ptr[0] == 0 and np.all(np.diff(c.row_ptr) >= 1)
    assert c.col.min() >= 0 and c.col.max() < c.d
    starts = c.row_ptr[:-1]
    d = np.diff(c.col.astype(np.int64))
    inner = np.ones(c.nnz, dtype=bool)
    inner[starts] = False
    assert np.all(d[inner[1:]] > 0)  # strictly ascending inside each row
    norms = np.sqrt(np.add.reduceat(c.val ** 2, starts))
    assert np.allclose(norms, 1.0, atol=1e-14)
    assert np.all(c.val > 0)


def test_f32_is_rounded_f64():
    a = synth.make_corpus(500, 1000, 30, 1.1, np.float64, seed=3)
    b = synth.make_corpus(500, 1000, 30, 1.1, np.float32, seed=3)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert np.array_equal(a.val.astype(np.float32), b.val)


def test_reproducible_and_seed_sensitive():
    a = synth.make_corpus(1000, 500, 20, 1.0, np.float32, seed=11)
    b = synth.make_corpus(1000, 500, 20, 1.0, np.float32, seed=11)
    c = synth.make_corpus(1000, 500, 20, 1.0, np.float32, seed=12)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert not (len(a.col) == len(c.col) and np.array_equal(a.col, c.col))


def test_poisson_lengths_and_zipf_slope():
    lam, s = 60.0, 1.1
    c = synth.make_corpus(20000, 50000, lam, s, np.float32, seed=5)
    lens = np.diff(c.row_ptr)
    assert abs(lens.mean() - lam) < 0.5 and abs(lens.var() - lam) < 4.0
    df = np.bincount(c.col, minlength=c.d).astype(np.float64)
    # rank-frequency of the tail (terms 100..1000) follows (t+1)^-s: fit the slope
    t = np.arange(100, 1000)
    slope = np.polyfit(np.log(t + 1.0), np.log(df[t]), 1)[0]
    assert abs(slope + s) < 0.15
    # hot terms are nearly saturated (sampling without repeats inside a row)
    assert df[0] > 0.9 * c.n


def test_clip_to_d_and_min_one():
    c = synth.make_corpus(200, 8, 30, 1.0, np.float64, seed=1)
    lens = np.diff(c.row_ptr)
    assert lens.max() == 8 and lens.min() >= 1


def test_init_ids_distinct():
    ids = synth.init_ids(1000, 100, 5)
    assert len(np.unique(ids)) == 100 and ids.min() >= 0 and ids.max() < 1000
    assert np.array_equal(ids, synth.init_ids(1000, 100, 5))
