/*
 * sivf.h -- C ABI of the MI355X structured inverted-file spherical k-means
 * library (libsivf.so).
 *
 * Method: Aoyama & Saito, "Structured Inverted-File k-Means Clustering for
 * High-Dimensional Sparse Data".  Problem: given N objects x_i (sparse rows,
 * L2-normalised in the paper's use) and k, find clusters maximising the
 * spherical objective sum_i <x_i, mu_a(i)> with unit-norm means (Section 1,
 * spherical k-means; Section 2.1, Eq. (1)); iterate the assignment and update
 * steps of Alg. 1.  The assignment step walks a structured inverted file of the
 * centroids (term -> (centroid id, value) postings, moving centroids in front
 * of invariant ones) and uses the invariant centroid-pair filter (ICP) by
 * ending each list walk at the moving/invariant boundary (Section 4, Alg. 4).
 * The update step forms the means and rebuilds the structured file (Alg. 5).
 *
 * Conventions for every entry point:
 *  - Array pointers are DEVICE pointers (memory of the ctx's device) unless the
 *    parameter name ends in _host.  The caller owns every array it passes; the
 *    library never frees caller memory.  Library-owned objects (sivf_ctx,
 *    sivf_ivf) are released with sivf_destroy / sivf_ivf_free.
 *  - Work is enqueued on the ctx's HIP stream.  Calls return once the work is
 *    enqueued, except that a non-NULL *_host output makes the call wait for the
 *    stream before it returns.
 *  - Every call returns a sivf_status; sivf_last_error(ctx) gives a message.
 *    Arguments and inputs are validated before any output is written, so on a
 *    validation error every output is left untouched.  A SIVF_E_HIP error (a
 *    failed HIP call) can leave outputs partially written.
 *  - One ctx must not be used from two host threads at once.  Calls on one ctx
 *    are ordered by its stream.
 *
 * Exactness: assignments equal those of plain FP64 spherical Lloyd computed
 * with the arithmetic conventions below, bit for bit, in both posting
 * precisions.  A fast FP32 (or BF16-times-FP32) pass certifies each argmax
 * with a rigorous rounding-error bound; objects it cannot certify are
 * re-scored in FP64 on the GPU in the canonical order.  FP64 conventions:
 * rho_ij = fold over x_i's terms in ascending order of acc = acc + v*u (two
 * roundings, from +0.0); lowest index wins ties; centroid = w / ||w||_2 with
 * w = (sum of members in ascending object id) / |C_j|, ||w||^2 summed
 * sequentially in ascending term order; an empty cluster keeps its previous
 * centroid.
 */
#ifndef SIVF_H
#define SIVF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIVF_OK = 0,
    SIVF_E_INVALID = -1,     /* null pointer, bad option or argument */
    SIVF_E_SHAPE = -2,       /* inconsistent sizes (k < 1, k > N, d mismatch, ...) */
    SIVF_E_UNSORTED = -3,    /* a CSR row's columns are not strictly ascending, or row_ptr decreases */
    SIVF_E_RANGE = -4,       /* a column, id or assignment outside its range */
    SIVF_E_NONFINITE = -5,   /* NaN or infinity in a value array */
    SIVF_E_NOMEM = -6,       /* device allocation failed or would exceed workspace_cap_bytes */
    SIVF_E_HIP = -7,         /* a HIP runtime call or kernel launch failed */
    SIVF_E_UNSUPPORTED = -8  /* valid request this library does not support */
} sivf_status;

typedef enum { SIVF_F32 = 0, SIVF_F64 = 1, SIVF_BF16 = 2 } sivf_dtype;

/* Filter used by the assignment step.
 *  SIVF : ICP through the structured file; an object whose own cluster was
 *         invariant reads only the moving (front) part of each list (Alg. 4).
 *  IVF  : no filter; every object reads whole lists (Alg. 2).
 *  CBICP: ICP through a per-posting test of the centroid's flag over whole
 *         lists (Alg. 3); same result and same mult-add count as SIVF.
 *  RELAXED: SIVF, and also an object whose own cluster moved but whose FP64
 *         similarity to its own centroid did not decrease reads only the
 *         moving parts (the relaxed ICP condition of Section 2.1; same
 *         assignments as plain Lloyd).  Needs own64_inout in sivf_assign. */
typedef enum {
    SIVF_MODE_SIVF = 0,
    SIVF_MODE_IVF = 1,
    SIVF_MODE_CBICP = 2,
    SIVF_MODE_RELAXED = 3
} sivf_filter_mode;

/* A sparse matrix in CSR form, all arrays on the device.
 * row_ptr: int64[n_rows + 1], row_ptr[0] = 0, non-decreasing, row_ptr[n_rows] = nnz.
 * col:     int32[nnz], strictly ascending inside each row, 0 <= col < n_cols.
 * val:     nnz values of val_dtype (SIVF_F32 or SIVF_F64), finite.
 * Objects are rows (the paper's standard sparse expression, Fig. 1(a)). */
typedef struct {
    int64_t n_rows;
    int64_t n_cols;
    int64_t nnz;
    const int64_t* row_ptr;
    const int32_t* col;
    const void* val;
    sivf_dtype val_dtype;
} sivf_csr;

typedef struct {
    sivf_dtype posting_dtype;   /* SIVF_F32 (default) or SIVF_BF16 posting values */
    int32_t filter_mode;        /* sivf_filter_mode, default SIVF_MODE_SIVF */
    int32_t k_tile;             /* centroids per LDS similarity tile; 0 = automatic
                                   (k split evenly into tiles of at most 1024,
                                   rounded up to a multiple of 64);
                                   otherwise a multiple of 64 in [64, 4096] */
    int32_t certify;            /* 1 (default): exact assignments (certificate + FP64
                                   re-score).  0: take the fast-pass argmax as is
                                   (diagnostics only; not exact) */
    size_t workspace_cap_bytes; /* 0 = unlimited; else device bytes the ctx and its
                                   files may hold; exceeding it gives SIVF_E_NOMEM */
    float head_density;         /* in [0, 1], or negative (the default, -1) for the
                                   precision's own value: 0.5 with SIVF_F32 postings, 0.3
                                   with SIVF_BF16.  Terms held by at least this
                                   fraction of the k centroids also get a dense row of
                                   posting values (zeros for absent centroids) that the
                                   walk reads instead of the term's lists (objects in
                                   the ICP branch of modes SIVF and RELAXED read only
                                   the moving centroids' part; in CBICP they walk the
                                   lists); 0 disables.  Same results and mult-add counts either
                                   way (a memory layout choice, not the paper's). */
    int32_t tiles_per_launch;   /* centroid tiles the walk covers per kernel launch;
                                   0 (default) = 1: all objects walk tile 0, then
                                   tile 1, ... so one tile's lists stay cache-
                                   resident; a value >= the tile count walks every
                                   tile of an object in one launch.  Same results. */
    int32_t exact_objective;    /* 0 (default) or 1: sivf_assign also computes the
                                   spherical objective of the new assignment against
                                   the centroids it was made with, in FP64 from the
                                   exact similarities (sivf_iter_stats.objective) */
} sivf_options;

/* Per-iteration statistics (host struct). */
typedef struct {
    int32_t iter;                /* r */
    int32_t n_invariant;         /* #{j : lambda_j^[r] = 1} */
    int64_t multadds;            /* posting multiply-adds of the fast pass (one per
                                    (object, posting) pair visited) */
    int64_t moved;               /* #{i : a_i^[r] != a_i^[r-1]}; N at r = 1 */
    int64_t icp_objects;         /* objects that took the ICP branch */
    int64_t rescored_objects;    /* objects re-scored in FP64 from a candidate list */
    int64_t rescored_candidates; /* centroids re-scored over those objects */
    int64_t full_rescored;       /* objects re-scored in FP64 over all eligible centroids */
    double objective_fast;       /* sum_i own_sim_i as written (FP32 values, summed in FP64) */
    float t_walk_ms;             /* fast-pass kernel time (HIP events) */
    float t_assign_ms;           /* whole assignment step (walk + re-score + flags) */
    float t_update_ms;           /* whole update step (means + structured file) */
    int64_t head_rows;           /* dense head rows the walk read (see head_density) */
    int64_t relaxed_objects;     /* objects that took the relaxed ICP branch */
    double objective;            /* exact_objective: F(a^[r], mu^[r-1]) = sum_i rho(x_i,
                                    mu^[r-1]_{a_i^[r]}), each rho the FP64 similarity of the
                                    canonical order, summed in FP64 in a fixed order
                                    (Section 1, the spherical objective); else NaN */
    int64_t walk_bytes;          /* bytes requested by the fast pass's vector loads
                                    (64 lanes x load width per load issued: posting and
                                    head-row batches, segment records, staged terms) */
    int64_t walk_wide_bytes;     /* of which 16-byte-per-lane loads (dense head rows and
                                    segment records; the rest are 4- and 8-byte loads) */
    int32_t walk_launches;       /* fast-pass kernel launches of this step */
    int32_t reserved;
} sivf_iter_stats;

typedef struct sivf_ctx sivf_ctx;  /* device, stream, options, workspace, last error */
typedef struct sivf_ivf sivf_ivf;  /* k centroids (FP64, sparse) + their structured
                                      inverted file + the flags it is structured by */

/* Fill *opt with the defaults listed above. */
sivf_status sivf_default_options(sivf_options* opt);

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  opt may be NULL
 * (defaults).  *out receives the context. */
sivf_status sivf_create(sivf_ctx** out, int device, void* hip_stream, const sivf_options* opt);

/* Release a context and its workspace (waits for its stream).  NULL is a no-op. */
sivf_status sivf_destroy(sivf_ctx* ctx);

/* Message of the last failed call on ctx ("" if none).  Owned by ctx. */
const char* sivf_last_error(const sivf_ctx* ctx);

/* Check X on the device: row_ptr monotone and consistent with nnz, columns in
 * [0, n_cols) and strictly ascending per row, values finite.  Waits for the
 * stream.  Every other entry point that reads X runs the same check on each
 * call (X may have been edited in place since the last one) before any kernel
 * indexes with it; sivf_run_lloyd checks once per run. */
sivf_status sivf_validate_csr(sivf_ctx* ctx, const sivf_csr* X);

/* Initial centroids mu_j^(0) = x_{init_ids_host[j]} as stored (values widened to
 * FP64), j = 0..k-1, all flags 0 (every centroid moving), and their structured
 * inverted file.  The paper leaves initialisation open (Section 1, Alg. 1
 * starts from a given state); ids may repeat.  *out receives a new file. */
sivf_status sivf_init_centroids(sivf_ctx* ctx, const sivf_csr* X, int32_t k,
                                const int32_t* init_ids_host, sivf_ivf** out);

/* Build the structured inverted file of given centroids (Section 4; Alg. 5
 * "determine an inverted-file structure" / "make structured inverted-file").
 * centroids: k x d CSR with SIVF_F64 values (copied; caller keeps ownership).
 * lambda: uint8[k] flags (1 = invariant, goes to the back part), NULL = all 0.
 * *out receives a new file. */
sivf_status sivf_build_centroid_ivf(sivf_ctx* ctx, const sivf_csr* centroids,
                                    const uint8_t* lambda, sivf_ivf** out);

/* Release a file created by this library.  NULL is a no-op. */
sivf_status sivf_ivf_free(sivf_ctx* ctx, sivf_ivf* ivf);

/* Sizes of a file (any pointer may be NULL).  Waits for the stream.
 * postings = number of (centroid, term) pairs = centroid nonzeros. */
sivf_status sivf_ivf_sizes(sivf_ctx* ctx, const sivf_ivf* ivf, int32_t* k_host, int64_t* d_host,
                           int64_t* centroid_nnz_host, int32_t* n_tiles_host, int32_t* k_tile_host);

/* Copy a file out (device buffers, caller-allocated; any may be NULL):
 *   c_ptr int64[k+1], c_col int32[nnz], c_val f64[nnz]   centroids as CSR;
 *   lambda uint8[k]                                       flags of the structure;
 *   term_ptr int64[d+1], split int32[d], p_cid int32[nnz], p_val f64[nnz]
 *       the structured file in the paper's per-term layout: list of term s is
 *       [term_ptr[s], term_ptr[s+1]), moving part first with split[s] entries,
 *       each part in ascending centroid id.
 * The library's own in-memory layout renumbers the centroids (moving ones
 * first, each group in ascending id) and splits each list by tile of that
 * numbering; this export re-joins the tiles and maps back to centroid ids. */
sivf_status sivf_ivf_export(sivf_ctx* ctx, const sivf_ivf* ivf, int64_t* c_ptr, int32_t* c_col,
                            double* c_val, uint8_t* lambda, int64_t* term_ptr, int32_t* split,
                            int32_t* p_cid, double* p_val);

/* Assignment step r = iter (Alg. 4).  ivf holds mu^[r-1] structured by
 * lambda^[r-1] (the flags of the last update, all 0 after init).
 *  assign_inout int32[N]:  in a^[r-1] (ignored when iter == 1), out a^[r].
 *  own_sim_inout f32[N]:   in the values this call wrote at r-1, or those of
 *                          sivf_resume (ignored when iter == 1; read for the
 *                          objects whose cluster is invariant, and trusted: a
 *                          value farther from the exact similarity than the
 *                          certificate's bound can give a wrong argmax); out
 *                          the similarity of each object to its new centroid
 *                          (fast-pass value or FP64 re-score rounded to FP32).
 *  own64_inout f64[N]:     RELAXED mode only (else may be NULL): in the values
 *                          this call wrote at r-1 (ignored when iter == 1);
 *                          out the exact FP64 similarity of each object to its
 *                          new centroid (the oracle's value, bitwise).
 *  lambda_out uint8[k]:    out lambda^[r] (1 iff the cluster's members are the
 *                          same at r-1 and r; all 0 when iter == 1).
 *  stats_host:             optional; non-NULL makes the call wait.
 * ICP branch: iter >= 2, filter mode SIVF/CBICP/RELAXED, and the file's flag
 * of the object's previous cluster is 1.  Relaxed branch (RELAXED): iter >= 2,
 * that flag is 0, and the object's FP64 similarity to its previous centroid
 * now is >= own64_inout. */
sivf_status sivf_assign(sivf_ctx* ctx, const sivf_csr* X, const sivf_ivf* ivf, int32_t iter,
                        int32_t* assign_inout, float* own_sim_inout, double* own64_inout, uint8_t* lambda_out,
                        sivf_iter_stats* stats_host);

/* sivf_assign for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same step with the same arguments, results and errors, but its
 * workspace is a fixed 64 MiB block per device that the library holds from
 * its first use on the device until the process ends; the call makes no
 * device allocation and frees nothing.  The block bounds the sizes it takes:
 * about 330 bytes per object for k above one tile, 50 otherwise (so some
 * 190,000 objects against a multi-tile file); a larger request returns
 * SIVF_E_UNSUPPORTED before anything is written.  Every call on a device
 * shares that device's block and each call initialises what it reads, so
 * consecutive calls are independent; calls that overlap in time on one device
 * (several ctxs or streams) race on the block and must not be issued. */
sivf_status sivf_assign_noalloc(sivf_ctx* ctx, const sivf_csr* X, const sivf_ivf* ivf, int32_t iter,
                                int32_t* assign_inout, float* own_sim_inout, double* own64_inout,
                                uint8_t* lambda_out, sivf_iter_stats* stats_host);

/* Update step r (Alg. 5): replace the file's centroids by mu^[r] computed from
 * X and assign = a^[r] (int32[N], values in [0, k)), and restructure it with
 * lambda = lambda^[r] (uint8[k]).  Clusters with lambda_j = 1 or no members keep
 * their centroid bitwise.  stats_host optional (t_update_ms). */
sivf_status sivf_update(sivf_ctx* ctx, const sivf_csr* X, const int32_t* assign,
                        const uint8_t* lambda, sivf_ivf* ivf_inout, sivf_iter_stats* stats_host);

/* Restart a run between iterations (Alg. 1 from a saved state): the state
 * after the update of iteration r-1 is the centroids mu^[r-1] and the last two
 * assignments.  Builds the file of mu^[r-1] structured by lambda^[r-1], the
 * flags of the clusters whose members are the same in a^[r-2] and a^[r-1]
 * (Alg. 4, invariant clusters; all 0 when a_prev2 is NULL, i.e. r-1 = 1), and
 * the own similarities the next sivf_assign(iter = r) reads.
 *  centroids:     k x d CSR, SIVF_F64 values (copied), e.g. from sivf_ivf_export.
 *  a_prev:        int32[N] a^[r-1]; a_prev2: int32[N] a^[r-2] or NULL.
 *  *out:          receives the new file.
 *  own_sim_out:   f32[N], rho(x_i, mu^[r-1]_{a_i}) in FP64 rounded to FP32.
 *  own64_out:     f64[N] (RELAXED mode only, else may be NULL): that exact value
 *                 where the object's cluster is invariant, +infinity elsewhere,
 *                 so the first resumed step takes no relaxed branch (the
 *                 similarity to the centroid before the last update is not part
 *                 of the state); assignments are unaffected.
 * Continuing with sivf_assign(iter = r, assign_inout = a^[r-1], own_sim_out,
 * own64_out) and sivf_update reproduces the uninterrupted run's assignments,
 * flags, centroids and mult-add counts (RELAXED: counts from step r+1 on).
 * Waits for the stream. */
sivf_status sivf_resume(sivf_ctx* ctx, const sivf_csr* X, const sivf_csr* centroids, const int32_t* a_prev,
                        const int32_t* a_prev2, sivf_ivf** out, float* own_sim_out, double* own64_out);

/* The Lloyd driver (Alg. 1 around Alg. 4 / Alg. 5): init from init_ids_host,
 * then for r = 1..max_iter: assign; stop if r >= 2 and nothing moved; update.
 *  assign_out int32[N], own_sim_out f32[N] (NULL allowed): final a and own sims.
 *  centroids_out: if non-NULL receives the final file (caller frees).
 *  per_iter_host: sivf_iter_stats[max_iter] or NULL.  iters_done_host: or NULL.
 * Waits for the stream before returning. */
sivf_status sivf_run_lloyd(sivf_ctx* ctx, const sivf_csr* X, int32_t k, const int32_t* init_ids_host,
                           int32_t max_iter, int32_t* assign_out, float* own_sim_out,
                           sivf_ivf** centroids_out, sivf_iter_stats* per_iter_host,
                           int32_t* iters_done_host);

/* Soft spherical assignment (the differentiable form of the assignment step):
 *   S = X C^T, lse_i = log sum_j exp(S_ij / tau), loss = -sum_i lse_i.
 * X: N x d CSR (SIVF_F32 values).  C: f32[k * d] row-major dense centroids.
 * lse_out: f32[N].  loss_host: optional (waits); summed in FP64 in a fixed order.
 * Nothing of size N x k is stored. */
sivf_status sivf_soft_assign_fwd(sivf_ctx* ctx, const sivf_csr* X, const float* C, int32_t k,
                                 float tau, float* lse_out, double* loss_host);

/* Backward of sivf_soft_assign_fwd for upstream gradient grad_loss:
 *   P = exp(S/tau - lse), dS = -grad_loss * P / tau (S recomputed, never stored
 *   whole), dC = dS^T X -> dC_out f32[k * d] (overwritten),
 *   dX_it = sum_j dS_ij C_jt on X's nonzeros -> dxval_out f32[nnz] (overwritten).
 * Either output may be NULL.  Deterministic (fixed summation order).
 * Workspace held by the ctx: C^T and dC^T (k * d floats each), X's column
 * copy (8 B per nonzero, built through 4 * d bytes of counts per 1024 rows),
 * dS for one chunk of rows (at most 256 MiB), dX partials (32 B per nonzero
 * of a chunk), and the dC pass's partial rows (k floats per piece of the
 * chunk with the most pieces, counted before the pass: about 130 MB at
 * N = 262,144, D = 100,000, k = 4,096). */
sivf_status sivf_soft_assign_bwd(sivf_ctx* ctx, const sivf_csr* X, const float* C, int32_t k,
                                 float tau, const float* lse, float grad_loss, float* dC_out,
                                 float* dxval_out);

#ifdef __cplusplus
}
#endif

#endif /* SIVF_H */
