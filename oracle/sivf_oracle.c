/*
 * FP64 CPU oracle for structured inverted-file spherical k-means.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes is the plain definition of the method's result: the
 * structured inverted file and the ICP filter change how the paper traverses
 * the data, not the sums it forms (Section 2.1, ICP; Section 4, Alg. 4), so the
 * assignment is a plain argmax of cosine similarities and the update is a
 * plain mean followed by L2 normalisation (Alg. 1; Alg. 5; spherical k-means,
 * Section 1).  The SIVF bookkeeping (structured inverted file, invariance
 * flags, similarity-calculation counts) is written out as the paper defines it.
 *
 * Arithmetic conventions (the paper states none; these are the readings used):
 *  - all arithmetic in IEEE binary64, round to nearest even, every multiply and
 *    add rounded separately (built with -ffp-contract=off, no fast-math);
 *  - rho_ij = fold over the object's terms h in ascending term order of
 *    acc = acc + v_h * u_j[t_h], starting from +0.0, u_j dense (0 where the
 *    centroid lacks the term);
 *  - argmax keeps the lowest index among equal maxima (strict '>' scanning
 *    ascending j, Alg. 2 / Alg. 4 assignment loop);
 *  - update: w = sum of members in ascending object id (sequential per term),
 *    w /= |C_j|, s = sum_p w_p*w_p ascending p (sequential), n = sqrt(s),
 *    u_p = w_p / n for w_p != 0; an empty cluster keeps its previous centroid.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline double xval(const void* val, int is_f64, int64_t p) {
    return is_f64 ? ((const double*)val)[p] : (double)((const float*)val)[p];
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ *
 * Assignment (Alg. 1 assignment step; Alg. 4 with the ICP reading below).
 *
 * Full mode: a_i = lowest j attaining max_j rho_ij over all k centroids.
 * ICP mode (icp != 0, previous state given, lam_prev[a_prev[i]] == 1): the
 * object's own centroid is unchanged, so its similarity is the cached
 * own_prev[i]; start from best = (own_prev[i], a_prev[i]) and compare only the
 * moving centroids (lam_prev[j] == 0) in ascending j, replacing best when
 * rho_ij > best or (rho_ij == best and j < best_j).  (Reading: the printed
 * Alg. 4 starts the ICP branch from rho_max = 0, which could move an object to
 * a worse centroid; the ICP definition in Section 2.1 and the d_min seed of
 * Alg. 1 fix the start at the own similarity.)
 *
 * rows/n_rows select the objects to process (NULL: all n); outputs are indexed
 * by position in that list.  top2_out (nullable) receives, per processed
 * object, the largest and second largest rho over the candidate set.
 * ------------------------------------------------------------------------ */
int orc_assign(int64_t n, int64_t d, const int64_t* rp, const int32_t* col, const void* val,
               int val_f64, int32_t k, const int64_t* cp, const int32_t* ccol, const double* cval,
               const int64_t* rows, int64_t n_rows, int icp, const uint8_t* lam_prev,
               const int32_t* a_prev, const double* own_prev, int relaxed, int32_t* a_out, double* own_out,
               double* top2_out, uint8_t* branch_out) {
    if (n < 0 || d < 1 || k < 1) return -1;
    int64_t m = rows ? n_rows : n;
    /* dense transposed centroids restricted to the terms the processed rows use */
    int64_t* map = (int64_t*)malloc(sizeof(int64_t) * (size_t)d);
    if (!map) return -2;
    for (int64_t t = 0; t < d; ++t) map[t] = -1;
    int64_t used = 0;
    for (int64_t q = 0; q < m; ++q) {
        int64_t i = rows ? rows[q] : q;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (map[col[p]] < 0) map[col[p]] = used++;
    }
    double* mt = (double*)calloc((size_t)(used > 0 ? used : 1) * (size_t)k, sizeof(double));
    if (!mt) { free(map); return -2; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t j = 0; j < k; ++j)
        for (int64_t p = cp[j]; p < cp[j + 1]; ++p) {
            int64_t r = map[ccol[p]];
            if (r >= 0) mt[r * k + j] = cval[p];
        }
#pragma omp parallel
    {
        double* acc = (double*)malloc(sizeof(double) * (size_t)k);
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < m; ++q) {
            int64_t i = rows ? rows[q] : q;
            for (int32_t j = 0; j < k; ++j) acc[j] = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                double v = xval(val, val_f64, p);
                const double* u = mt + map[col[p]] * k;
                for (int32_t j = 0; j < k; ++j) acc[j] = acc[j] + v * u[j];
            }
            int use_icp = icp && lam_prev && a_prev && own_prev && lam_prev[a_prev[i]];
            /* relaxed ICP (Section 2.1): the own centroid moved, but the object's
             * similarity to it did not decrease, so no invariant centroid can
             * overtake it; only moving centroids are compared, from the own one */
            int use_rel = !use_icp && icp && relaxed && lam_prev && a_prev && own_prev &&
                          acc[a_prev[i]] >= own_prev[i];
            double best, second = -INFINITY;
            int32_t bj;
            if (use_rel) {
                bj = a_prev[i];
                best = acc[bj];
                for (int32_t j = 0; j < k; ++j) {
                    if (lam_prev[j] || j == bj) continue;
                    double r = acc[j];
                    if (r > best || (r == best && j < bj)) {
                        second = best;
                        best = r;
                        bj = j;
                    } else if (r > second) {
                        second = r;
                    }
                }
            } else if (use_icp) {
                best = own_prev[i];
                bj = a_prev[i];
                for (int32_t j = 0; j < k; ++j) {
                    if (lam_prev[j]) continue;
                    double r = acc[j];
                    if (r > best || (r == best && j < bj)) {
                        second = best;
                        best = r;
                        bj = j;
                    } else if (r > second) {
                        second = r;
                    }
                }
            } else {
                best = acc[0];
                bj = 0;
                for (int32_t j = 1; j < k; ++j) {
                    double r = acc[j];
                    if (r > best) {
                        second = best;
                        best = r;
                        bj = j;
                    } else if (r > second) {
                        second = r;
                    }
                }
            }
            a_out[q] = bj;
            if (branch_out) branch_out[q] = (uint8_t)(use_icp ? 1 : use_rel ? 2 : 0);
            if (own_out) own_out[q] = best;
            if (top2_out) { top2_out[2 * q] = best; top2_out[2 * q + 1] = second; }
        }
        free(acc);
    }
    free(mt);
    free(map);
    return 0;
}

/* rho for explicit (object, centroid) pairs, same fold as orc_assign. */
int orc_pair_sims(int64_t d, const int64_t* rp, const int32_t* col, const void* val, int val_f64,
                  const int64_t* cp, const int32_t* ccol, const double* cval, const int64_t* obj,
                  const int32_t* cen, int64_t n_pairs, double* out) {
#pragma omp parallel
    {
        double* u = (double*)calloc((size_t)d, sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < n_pairs; ++q) {
            int32_t j = cen[q];
            int64_t i = obj[q];
            for (int64_t p = cp[j]; p < cp[j + 1]; ++p) u[ccol[p]] = cval[p];
            double acc = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) acc = acc + xval(val, val_f64, p) * u[col[p]];
            out[q] = acc;
            for (int64_t p = cp[j]; p < cp[j + 1]; ++p) u[ccol[p]] = 0.0;
        }
        free(u);
    }
    return 0;
}

/* ------------------------------------------------------------------------ *
 * Update (Alg. 1 update step; Alg. 5 mean computation): centroid j becomes
 * normalise(mean of its members).  Output is a k x d CSR with ascending
 * columns; returns 0, or the required entry count (> 0) if out_cap is too
 * small (outputs then undefined), or < 0 on error.
 * ------------------------------------------------------------------------ */
int64_t orc_update(int64_t n, int64_t d, const int64_t* rp, const int32_t* col, const void* val,
                   int val_f64, int32_t k, const int32_t* a, const int64_t* prev_cp,
                   const int32_t* prev_ccol, const double* prev_cval, int64_t* out_cp,
                   int32_t* out_ccol, double* out_cval, int64_t out_cap, int32_t* counts_out) {
    if (n < 0 || d < 1 || k < 1) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (a[i] < 0 || a[i] >= k) return -1;
    int64_t* cnt = (int64_t*)calloc((size_t)k + 1, sizeof(int64_t));
    int64_t* members = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* nnz = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    int32_t** rc = (int32_t**)calloc((size_t)k, sizeof(int32_t*));
    double** rv = (double**)calloc((size_t)k, sizeof(double*));
    if (!cnt || !members || !nnz || !rc || !rv) return -2;
    for (int64_t i = 0; i < n; ++i) cnt[a[i] + 1]++;
    for (int32_t j = 0; j < k; ++j) cnt[j + 1] += cnt[j];
    {
        int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
        for (int32_t j = 0; j < k; ++j) pos[j] = cnt[j];
        for (int64_t i = 0; i < n; ++i) members[pos[a[i]]++] = i; /* ascending i per cluster */
        free(pos);
    }
    int err = 0;
#pragma omp parallel
    {
        double* w = (double*)calloc((size_t)d, sizeof(double));
        if (!w) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (int32_t j = 0; j < k; ++j) {
            if (!w) continue;
            int64_t size = cnt[j + 1] - cnt[j];
            if (size == 0) {
                /* empty cluster: keep the previous centroid bitwise */
                int64_t m = prev_cp[j + 1] - prev_cp[j];
                nnz[j] = m;
                rc[j] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
                rv[j] = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
                memcpy(rc[j], prev_ccol + prev_cp[j], sizeof(int32_t) * (size_t)m);
                memcpy(rv[j], prev_cval + prev_cp[j], sizeof(double) * (size_t)m);
                continue;
            }
            for (int64_t q = cnt[j]; q < cnt[j + 1]; ++q) {
                int64_t i = members[q];
                for (int64_t p = rp[i]; p < rp[i + 1]; ++p) w[col[p]] = w[col[p]] + xval(val, val_f64, p);
            }
            double sz = (double)size;
            for (int64_t p = 0; p < d; ++p) w[p] = w[p] / sz;
            double s = 0.0;
            for (int64_t p = 0; p < d; ++p) s = s + w[p] * w[p];
            double nr = sqrt(s);
            int64_t m = 0;
            for (int64_t p = 0; p < d; ++p) m += (w[p] != 0.0);
            nnz[j] = m;
            rc[j] = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
            rv[j] = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
            int64_t e = 0;
            for (int64_t p = 0; p < d; ++p) {
                if (w[p] != 0.0) {
                    rc[j][e] = (int32_t)p;
                    rv[j][e] = w[p] / nr;
                    ++e;
                }
                w[p] = 0.0;
            }
        }
        free(w);
    }
    int64_t total = 0;
    for (int32_t j = 0; j < k; ++j) total += nnz[j];
    int64_t ret = 0;
    if (err) {
        ret = err;
    } else if (total > out_cap) {
        ret = total;
    } else {
        out_cp[0] = 0;
        for (int32_t j = 0; j < k; ++j) out_cp[j + 1] = out_cp[j] + nnz[j];
        for (int32_t j = 0; j < k; ++j) {
            memcpy(out_ccol + out_cp[j], rc[j], sizeof(int32_t) * (size_t)nnz[j]);
            memcpy(out_cval + out_cp[j], rv[j], sizeof(double) * (size_t)nnz[j]);
        }
        if (counts_out)
            for (int32_t j = 0; j < k; ++j) counts_out[j] = (int32_t)(cnt[j + 1] - cnt[j]);
    }
    for (int32_t j = 0; j < k; ++j) { free(rc[j]); free(rv[j]); }
    free(rc); free(rv); free(nnz); free(members); free(cnt);
    return ret;
}

/* ------------------------------------------------------------------------ *
 * Structured inverted file (Section 4; Alg. 5 "determine an inverted-file
 * structure" and "make structured inverted-file").  For each term s the list
 * holds (centroid id, value) tuples, moving centroids (lam[j] == 0) first, then
 * invariant ones, each part in ascending centroid id.  split[s] = (mf_[0])_s is
 * the length of the moving part; term_ptr is the CSR-style list start.
 * lam == NULL means every centroid is moving.  Reading: both counting and
 * placement use the same flags (the flags the update receives).
 * ------------------------------------------------------------------------ */
int orc_build_ivf(int32_t k, int64_t d, const int64_t* cp, const int32_t* ccol, const double* cval,
                  const uint8_t* lam, int64_t* term_ptr, int32_t* split, int32_t* cid, double* uval) {
    int64_t* mf0 = (int64_t*)calloc((size_t)d, sizeof(int64_t));
    int64_t* mf1 = (int64_t*)calloc((size_t)d, sizeof(int64_t));
    int64_t* q0 = (int64_t*)malloc(sizeof(int64_t) * (size_t)d);
    int64_t* q1 = (int64_t*)malloc(sizeof(int64_t) * (size_t)d);
    if (!mf0 || !mf1 || !q0 || !q1) return -2;
    for (int32_t j = 0; j < k; ++j) {
        int inv = lam ? (lam[j] != 0) : 0;
        for (int64_t p = cp[j]; p < cp[j + 1]; ++p) {
            if (ccol[p] < 0 || ccol[p] >= d) return -1;
            if (inv) mf1[ccol[p]]++; else mf0[ccol[p]]++;
        }
    }
    term_ptr[0] = 0;
    for (int64_t s = 0; s < d; ++s) {
        term_ptr[s + 1] = term_ptr[s] + mf0[s] + mf1[s];
        split[s] = (int32_t)mf0[s];
        q0[s] = term_ptr[s];
        q1[s] = term_ptr[s] + mf0[s];
    }
    for (int32_t j = 0; j < k; ++j) {
        int inv = lam ? (lam[j] != 0) : 0;
        for (int64_t p = cp[j]; p < cp[j + 1]; ++p) {
            int32_t s = ccol[p];
            int64_t at = inv ? q1[s]++ : q0[s]++;
            cid[at] = j;
            uval[at] = cval[p];
        }
    }
    free(mf0); free(mf1); free(q0); free(q1);
    return 0;
}

/* ------------------------------------------------------------------------ *
 * Similarity-calculation counts (one per posting multiply-add; Section 5.3
 * counts similarity calculations; here the unit is the posting mult-add).
 *   mode 0 (SIVF, Alg. 4): an ICP-mode object reads the moving part of each
 *          of its terms' lists, (mf_[0])_s entries; other objects read (mf)_s.
 *   mode 1 (IVF-CBICP, Alg. 3): an ICP-mode object walks the whole list and
 *          multiplies only where the posting's centroid is moving (per-posting
 *          branch); the count is the number of taken branches.
 *   mode 2 (IVF, Alg. 2): every object reads (mf)_s.
 * ICP mode as in orc_assign (lam_prev NULL: iteration 1, no object in ICP
 * mode).  Uses the structured inverted file from orc_build_ivf.
 * ------------------------------------------------------------------------ */
int orc_multadds(int64_t n, const int64_t* rp, const int32_t* col, const int64_t* term_ptr,
                 const int32_t* split, const int32_t* cid, int icp, const uint8_t* lam_prev,
                 const int32_t* a_prev, int mode, const uint8_t* branch, int64_t* per_row, int64_t* total) {
    int64_t sum = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : sum)
    for (int64_t i = 0; i < n; ++i) {
        /* branch[i] != 0: the object compared moving centroids only (ICP or relaxed ICP) */
        int use_icp = mode != 2 && icp && lam_prev && a_prev &&
                      (branch ? branch[i] != 0 : lam_prev[a_prev[i]] != 0);
        int64_t c = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            int32_t s = col[p];
            if (!use_icp) {
                c += term_ptr[s + 1] - term_ptr[s];
            } else if (mode == 0) {
                c += split[s];
            } else {
                for (int64_t q = term_ptr[s]; q < term_ptr[s + 1]; ++q) c += (lam_prev[cid[q]] == 0);
            }
        }
        if (per_row) per_row[i] = c;
        sum += c;
    }
    *total = sum;
    return 0;
}

/* ------------------------------------------------------------------------ *
 * Soft spherical assignment (the differentiable form):
 *   S = X C^T, lse_i = log sum_j exp(S_ij / tau), L = -sum_i lse_i,
 *   P_ij = exp(S_ij/tau - lse_i), dS = -g P / tau,
 *   dC = dS^T X (dense k x d), dX_it = sum_j dS_ij C_jt on X's nonzeros.
 * C is dense k x d (row major, f64).  S_ij uses the same ascending-term fold
 * as rho_ij above.  lse uses the max-shift: m + log(sum exp(S/tau - m)).
 * ------------------------------------------------------------------------ */
static void soft_row(int64_t i, int64_t d, const int64_t* rp, const int32_t* col, const void* val,
                     int val_f64, int32_t k, const double* C, double* s) {
    for (int32_t j = 0; j < k; ++j) {
        double acc = 0.0;
        const double* c = C + (int64_t)j * d;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) acc = acc + xval(val, val_f64, p) * c[col[p]];
        s[j] = acc;
    }
}

static double row_lse(const double* s, int32_t k, double tau) {
    double m = -INFINITY;
    for (int32_t j = 0; j < k; ++j) if (s[j] / tau > m) m = s[j] / tau;
    double z = 0.0;
    for (int32_t j = 0; j < k; ++j) z = z + exp(s[j] / tau - m);
    return m + log(z);
}

int orc_soft_forward(int64_t d, const int64_t* rp, const int32_t* col, const void* val, int val_f64,
                     int32_t k, const double* C, double tau, const int64_t* rows, int64_t n_rows,
                     double* lse_out) {
#pragma omp parallel
    {
        double* s = (double*)malloc(sizeof(double) * (size_t)k);
#pragma omp for schedule(dynamic, 8)
        for (int64_t q = 0; q < n_rows; ++q) {
            soft_row(rows[q], d, rp, col, val, val_f64, k, C, s);
            lse_out[q] = row_lse(s, k, tau);
        }
        free(s);
    }
    return 0;
}

/* dX on the listed rows (dx_out indexed like X's nonzeros of those rows, i.e.
 * dx_out[p] for p in [rp[i], rp[i+1])), and the contribution of the listed
 * rows to dC (dc_out, k x d, accumulated in ascending row order; NULL to skip).
 * lse is indexed by position in rows. */
int orc_soft_backward(int64_t d, const int64_t* rp, const int32_t* col, const void* val,
                      int val_f64, int32_t k, const double* C, double tau, double g,
                      const int64_t* rows, int64_t n_rows, const double* lse, double* dx_out,
                      double* dc_out) {
    double* ds_all = NULL;
    if (dc_out) {
        ds_all = (double*)malloc(sizeof(double) * (size_t)k * (size_t)(n_rows > 0 ? n_rows : 1));
        if (!ds_all) return -2;
    }
#pragma omp parallel
    {
        double* s = (double*)malloc(sizeof(double) * (size_t)k);
        double* ds = (double*)malloc(sizeof(double) * (size_t)k);
#pragma omp for schedule(dynamic, 8)
        for (int64_t q = 0; q < n_rows; ++q) {
            int64_t i = rows[q];
            soft_row(i, d, rp, col, val, val_f64, k, C, s);
            for (int32_t j = 0; j < k; ++j) ds[j] = -g * exp(s[j] / tau - lse[q]) / tau;
            if (dx_out)
                for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                    double acc = 0.0;
                    for (int32_t j = 0; j < k; ++j) acc = acc + ds[j] * C[(int64_t)j * d + col[p]];
                    dx_out[p] = acc;
                }
            if (ds_all) memcpy(ds_all + q * (int64_t)k, ds, sizeof(double) * (size_t)k);
        }
        free(s);
        free(ds);
    }
    if (dc_out) {
        /* dC_jt = sum over listed rows (ascending position) of dS_ij * x_it */
#pragma omp parallel for schedule(dynamic, 4)
        for (int32_t j = 0; j < k; ++j) {
            double* out = dc_out + (int64_t)j * d;
            for (int64_t q = 0; q < n_rows; ++q) {
                int64_t i = rows[q];
                double dsij = ds_all[q * (int64_t)k + j];
                for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                    out[col[p]] = out[col[p]] + dsij * xval(val, val_f64, p);
            }
        }
        free(ds_all);
    }
    return 0;
}
