// Declarations of the soft-assignment kernels (k_soft.hip) used by the C ABI.
#pragma once

#include "internal.h"

namespace sivf {

hipError_t soft_transpose(const float* in, float* out, int64_t R, int64_t Cn, hipStream_t s);
// pmax, psum: [N * 8] per-row partial max / sum-exp of the 8 column groups
hipError_t soft_forward(int64_t N, const int64_t* rp, const int32_t* col, const float* xv, const float* CT, int32_t k,
                        float tau, float* lse, double* loss_dev, float* pmax, float* psum, int n_cu, hipStream_t s);
// rows [c0, c1) whose nonzeros are [p0, p1); dxp: [(p1 - p0) * 8] per-group dX partials
hipError_t soft_bwd_rows(int64_t c0, int64_t c1, int64_t p0, int64_t p1, const int64_t* rp, const int32_t* col,
                         const float* xv, const float* CT, int32_t k, float tau, float grad, const float* lse, float* dS,
                         float* dxp, float* dxv, int n_cu, hipStream_t s);
hipError_t soft_csc(int64_t N, int64_t d, int64_t nnz, const int64_t* rp, const int32_t* col, const float* xv,
                    int32_t* hist, int64_t* cnt, int64_t* colptr, int64_t* scan_ws, int32_t* xt_row, float* xt_val,
                    hipStream_t s);
// out[j] = rp[min(j * rc, n)] for j in [0, nch]: the nonzero offsets of the row chunks
hipError_t soft_chunk_offsets(const int64_t* rp, int64_t n, int64_t rc, int64_t nch, int64_t* out, hipStream_t s);
// workspace of the dC pass: per-term row ranges of the chunk, pieces of the long ones
struct DctWs {
    int64_t* lo;          // [d] first CSC entry of the chunk's rows
    int64_t* hi;          // [d] one past the last
    int64_t* np;          // [d] pieces of the term's range (0: summed whole)
    int64_t* pstart;      // [d + 1] exclusive scan of np
    int64_t* hflag;       // [d] 1 for a hot term (range longer than hot_min entries)
    int64_t* hscan;       // [d + 1] exclusive scan of hflag
    int32_t* hot;         // [d] the hot terms, ascending
    int64_t* mflag;       // [d] 1 for a mid term (range of piece + 1 .. hot_min entries)
    int64_t* mscan;       // [d + 1] exclusive scan of mflag
    int32_t* mid;         // [d] the mid terms, ascending
    int64_t* scan_ws;     // scan_ws_elems(d)
    int32_t* item;        // [max_pieces] term of each piece
    float* part;          // [max_pieces * k] partial rows
    int64_t max_pieces;   // the most pieces of any chunk (counted by soft_dct_count)
    int64_t piece;        // ranges of at most this many entries are summed whole
    int64_t hot_min;      // entries above which a range is hot
    int64_t blk_rows;     // rows per block of a hot range
    int64_t mid_blk_rows; // rows per block of a mid range
};
// pieces of the chunk [c0, c1) -> *count (device); lo, hi, np, pstart, the
// flags and scans of w are overwritten
hipError_t soft_dct_count(int64_t d, int64_t c0, int64_t c1, const int64_t* colptr, const int32_t* xt_row, DctWs w,
                          int64_t* count, hipStream_t s);
hipError_t soft_dct(int64_t d, int32_t k, int64_t c0, int64_t c1, int first, const int64_t* colptr,
                    const int32_t* xt_row, const float* xt_val, const float* dS, float* dCT, DctWs w, int n_cu,
                    hipStream_t s);


}  // namespace sivf
