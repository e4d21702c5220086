"""Small helpers for tests: corpora from explicit rows, exact rational sums."""
from fractions import Fraction

import numpy as np

from synth import Corpus


def corpus_from_rows(rows, d, values=None, dtype=np.float64):
    """rows: list of term lists (ascending); values: list of value lists or a scalar."""
    ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([t for r in rows for t in r], dtype=np.int32)
    if values is None or np.isscalar(values):
        v = np.full(len(col), 1.0 if values is None else values, dtype=dtype)
    else:
        v = np.array([x for r in values for x in r], dtype=dtype)
    return Corpus(len(rows), d, ptr, col, v)


def corpus_from_dense(x, dtype=np.float64):
    x = np.asarray(x)
    rows, vals = [], []
    for r in x:
        nz = np.nonzero(r)[0]
        rows.append(list(nz))
        vals.append([float(r[t]) for t in nz])
    return corpus_from_rows(rows, x.shape[1], vals, dtype)


def exact_sims(corpus, cents):
    """Exact rational rho_ij = sum_h v_h u_j[t_h] from the stored binary values."""
    dense_c = {}
    for j in range(cents.k):
        dense_c[j] = {int(t): Fraction(float(u)) for t, u in
                      zip(cents.col[cents.ptr[j]:cents.ptr[j + 1]], cents.val[cents.ptr[j]:cents.ptr[j + 1]])}
    out = []
    for i in range(corpus.n):
        terms = corpus.col[corpus.row_ptr[i]:corpus.row_ptr[i + 1]]
        vals = corpus.val[corpus.row_ptr[i]:corpus.row_ptr[i + 1]]
        row = []
        for j in range(cents.k):
            s = Fraction(0)
            for t, v in zip(terms, vals):
                u = dense_c[j].get(int(t))
                if u is not None:
                    s += Fraction(float(v)) * u
            row.append(s)
        out.append(row)
    return out


def gamma(n, u):
    return n * u / (1 - n * u)
