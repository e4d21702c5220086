/*
 * Seeded synthetic corpora shaped like the paper's document collections
 * (Section 5.1: L2-normalised tf-idf vectors, tens of nonzeros per row out of
 * ~140k terms, power-law term frequencies).  This file holds input generation
 * only: none of the clustering arithmetic lives here.  Both the oracle and the
 * GPU path consume what it writes.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), used as a counter-based generator: every
 * (seed, row, stream) triple owns an independent sequence, so rows can be
 * generated in parallel and any row can be regenerated alone.
 *
 * Row recipe (row i, given N, D, lambda, s, seed):
 *   n_i   = clip(Poisson(lambda), 1, D)       inversion on one uniform
 *   terms = the first n_i distinct values of an i.i.d. sequence with
 *           P(t) proportional to (t+1)^(-s), t in [0, D)   (inverse CDF),
 *           then sorted ascending
 *   vals  = exp(z), z ~ N(0,1) by Box-Muller, one per term in ascending term
 *           order; divided by the row's f64 L2 norm; stored as f64 or RN f32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s; } sm64;

static inline uint64_t sm64_next(sm64* g) {
    g->s += 0x9E3779B97F4A7C15ULL;
    return mix64(g->s);
}

/* uniform in [0, 1) with 53 random bits */
static inline double sm64_unif(sm64* g) {
    return (double)(sm64_next(g) >> 11) * (1.0 / 9007199254740992.0);
}

/* uniform in (0, 1] */
static inline double sm64_unif_pos(sm64* g) {
    return ((double)(sm64_next(g) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

static inline sm64 stream_for(uint64_t seed, uint64_t row, uint64_t which) {
    sm64 g;
    g.s = mix64(mix64(seed ^ 0xA0761D6478BD642FULL) + row * 0xE7037ED1A0B428DBULL + which);
    return g;
}

/* Poisson by inversion of the CDF, one uniform per draw (fine for lambda up to
 * several hundred: exp(-lambda) stays a normal double). */
static int64_t poisson(sm64* g, double lam) {
    double u = sm64_unif(g);
    double p = exp(-lam);
    double c = p;
    int64_t x = 0;
    while (u >= c && x < 100000) {
        x += 1;
        p *= lam / (double)x;
        c += p;
        if (p == 0.0 && c <= u) break;
    }
    return x;
}

int synth_row_counts(int64_t n, int64_t d, double lam, uint64_t seed, int64_t* counts) {
    if (n < 0 || d < 1 || lam < 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        sm64 g = stream_for(seed, (uint64_t)i, 0);
        int64_t c = poisson(&g, lam);
        if (c < 1) c = 1;
        if (c > d) c = d;
        counts[i] = c;
    }
    return 0;
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* cum[t] = sum_{u <= t} (u+1)^(-s) */
static double* zipf_table(int64_t d, double s) {
    double* cum = (double*)malloc(sizeof(double) * (size_t)d);
    if (!cum) return NULL;
    double acc = 0.0;
    for (int64_t t = 0; t < d; ++t) {
        acc += pow((double)(t + 1), -s);
        cum[t] = acc;
    }
    return cum;
}

static inline int32_t zipf_draw(sm64* g, const double* cum, int64_t d) {
    double target = sm64_unif(g) * cum[d - 1];
    int64_t lo = 0, hi = d - 1; /* smallest t with cum[t] > target */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cum[mid] > target) hi = mid; else lo = mid + 1;
    }
    return (int32_t)lo;
}

/* Fill col/val for rows whose row_ptr is already known.  val_is_f64 selects
 * the stored dtype (1: f64, 0: RN f32). */
int synth_fill(int64_t n, int64_t d, double zipf_s, uint64_t seed, const int64_t* row_ptr,
               int32_t* col, void* val, int val_is_f64) {
    if (n < 0 || d < 1) return -1;
    double* cum = zipf_table(d, zipf_s);
    if (!cum) return -2;
    int err = 0;
#pragma omp parallel
    {
        uint32_t* mark = (uint32_t*)calloc((size_t)d, sizeof(uint32_t));
        double* tmp = NULL;
        int64_t tmp_cap = 0;
        if (!mark) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            if (!mark) continue;
            int64_t b = row_ptr[i], m = row_ptr[i + 1] - b;
            if (m <= 0) continue;
            if (m > tmp_cap) {
                free(tmp);
                tmp_cap = m * 2;
                tmp = (double*)malloc(sizeof(double) * (size_t)tmp_cap);
            }
            const uint32_t stamp = 1u; /* marks are cleared again below */
            sm64 g = stream_for(seed, (uint64_t)i, 1);
            int64_t got = 0;
            int64_t draws = 0, limit = 64 * d + 4096;
            while (got < m && draws < limit) {
                int32_t t = zipf_draw(&g, cum, d);
                ++draws;
                if (mark[t] == stamp) continue;
                mark[t] = stamp;
                col[b + got++] = t;
            }
            /* fallback for rows that ask for nearly every term: smallest unused ids */
            for (int32_t t = 0; got < m && t < d; ++t) {
                if (mark[t] != stamp) { mark[t] = stamp; col[b + got++] = t; }
            }
            for (int64_t h = 0; h < m; ++h) mark[col[b + h]] = 0;
            qsort(col + b, (size_t)m, sizeof(int32_t), cmp_i32);
            sm64 gv = stream_for(seed, (uint64_t)i, 2);
            double ss = 0.0;
            for (int64_t h = 0; h < m; ++h) {
                double u1 = sm64_unif_pos(&gv), u2 = sm64_unif(&gv);
                double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
                double v = exp(z);
                tmp[h] = v;
                ss += v * v;
            }
            double nrm = sqrt(ss);
            for (int64_t h = 0; h < m; ++h) {
                double v = tmp[h] / nrm;
                if (val_is_f64) ((double*)val)[b + h] = v;
                else ((float*)val)[b + h] = (float)v;
            }
        }
        free(mark);
        free(tmp);
    }
    free(cum);
    return err;
}

/* Dense k x d centroid matrix for the soft-assignment workload:
 * C_j = normalise(dense(x_{ids[j]}) + noise * |N(0,1)|), rows f32. */
int synth_dense_centroids(int64_t d, int32_t k, const int64_t* row_ptr, const int32_t* col,
                          const float* val, const int64_t* ids, double noise, uint64_t seed,
                          float* out) {
#pragma omp parallel
    {
        double* row = (double*)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(dynamic, 4)
        for (int32_t j = 0; j < k; ++j) {
            sm64 g = stream_for(seed, (uint64_t)j, 3);
            for (int64_t t = 0; t < d; ++t) {
                double u1 = sm64_unif_pos(&g), u2 = sm64_unif(&g);
                double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
                row[t] = noise * fabs(z);
            }
            int64_t i = ids[j];
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) row[col[p]] += (double)val[p];
            double ss = 0.0;
            for (int64_t t = 0; t < d; ++t) ss += row[t] * row[t];
            double nrm = sqrt(ss);
            for (int64_t t = 0; t < d; ++t) out[(int64_t)j * d + t] = (float)(row[t] / nrm);
        }
        free(row);
    }
    return 0;
}

int synth_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
