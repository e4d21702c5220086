// Structured inverted file of the centroids (Section 4; Alg. 5, "determine an
// inverted-file structure" and "make structured inverted-file").
//
// Device layout (one list per term, split by centroid tile for the LDS-tiled
// walk): postings are ordered by (term, tile, part, position) where part 0
// holds the moving centroids (flag 0) and part 1 the invariant ones.  With a
// single tile this is exactly the paper's per-term [moving | invariant] list.
// Positions renumber the centroids with the moving ones first, each group in
// ascending id (perm[q] = centroid at position q, iperm its inverse), and the
// tiles cover positions: a tile's moving centroids are a prefix of it, so an
// object that compares moving centroids only reads that prefix and skips the
// tiles past the last moving centroid.  Inside each part positions ascend
// with the ids, so per part the order is the paper's.
//   seg[t*T + tile]  start of segment (t, tile); its end is seg[t*T + tile + 1]
//   mid[t*T + tile]  length of the moving part of that segment
//   cid[p]           position minus tile*kt (16 bits)
//   v32/v16[p]       posting value, RN to f32 (or RNE of that to bf16)
//   v64[p]           the FP64 value (exact re-score over whole lists)
//
// Placement is deterministic without ordering atomics: a bitmap bm[w][t] marks
// which centroids hold term t; the rank of centroid j inside its (t, tile,
// part) segment is a popcount of lower bits, so every part comes out in
// ascending centroid id regardless of thread timing (Alg. 5 fills in ascending
// j the same way).
#include <algorithm>

#include "internal.h"
#include "wave.h"

namespace sivf {

int64_t ivf_w64(int32_t k) { return ((int64_t)k + 63) / 64; }

// ---------------------------------------------------------------- positions
__global__ void k_perm_flags(const uint8_t* __restrict__ lam, int32_t k, int64_t* __restrict__ mv) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < k) mv[j] = (lam && lam[j]) ? 0 : 1;
}

// mvpre = exclusive scan of the moving flags; n_moving = mvpre[k]
__global__ void k_perm_fill(const uint8_t* __restrict__ lam, int32_t k, const int64_t* __restrict__ mvpre,
                            int32_t* __restrict__ perm, int32_t* __restrict__ iperm) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= k) return;
    const int64_t nm = mvpre[k];
    const int64_t q = (lam && lam[j]) ? nm + (j - mvpre[j]) : mvpre[j];
    iperm[j] = (int32_t)q;
    perm[q] = (int32_t)j;
}

hipError_t ivf_perm(const uint8_t* lam, int32_t k, int64_t* mv, int64_t* mvpre, int64_t* scan_ws, int32_t* perm,
                    int32_t* iperm, hipStream_t s) {
    const unsigned blocks = (unsigned)(((int64_t)k + 255) / 256);
    hipLaunchKernelGGL(k_perm_flags, dim3(blocks), dim3(256), 0, s, lam, k, mv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan_i64(mv, mvpre, k, scan_ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_perm_fill, dim3(blocks), dim3(256), 0, s, lam, k, mvpre, perm, iperm);
    return hipGetLastError();
}

__global__ void k_ivf_bits(Store st, int32_t k, int64_t d, const int32_t* __restrict__ iperm,
                           unsigned long long* __restrict__ bm) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < k; j += nw) {
        const int64_t b = st.start[j], m = st.nnz[j];
        const int64_t q = iperm[j];
        unsigned long long* row = bm + (q >> 6) * d;
        const unsigned long long bit = 1ull << (q & 63);
        for (int64_t p = lane; p < m; p += 64) {
            const int32_t t = st.term[b + p];
            if (t >= 0 && t < d) atomicOr(&row[t], bit);
        }
    }
}

// invariant bits by position: positions n_moving .. k-1
__global__ void k_lam_bits(int32_t k, int32_t n_moving, unsigned long long* __restrict__ lbits) {
    int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (w >= ((int64_t)k + 63) / 64) return;
    unsigned long long m = 0;
    for (int b = 0; b < 64; ++b) {
        int64_t q = w * 64 + b;
        if (q < k && q >= n_moving) m |= 1ull << b;
    }
    lbits[w] = m;
}

// One thread per (tile, term): per-word prefix counts inside the tile and the
// segment's part sizes.
__global__ void k_ivf_counts(const unsigned long long* __restrict__ bm, const unsigned long long* __restrict__ lbits,
                             int64_t d, int32_t kt, int32_t T, int64_t W64, uint16_t* __restrict__ pre0,
                             uint16_t* __restrict__ pre1, int64_t* __restrict__ cnt) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= d * T) return;
    const int64_t tile = idx / d, t = idx - tile * d;
    const int64_t w0 = tile * (kt / 64);
    int64_t w1 = w0 + kt / 64;
    if (w1 > W64) w1 = W64;
    uint32_t c0 = 0, c1 = 0;
    for (int64_t w = w0; w < w1; ++w) {
        unsigned long long m = bm[w * d + t];
        unsigned long long lb = lbits[w];
        pre0[w * d + t] = (uint16_t)c0;
        pre1[w * d + t] = (uint16_t)c1;
        c0 += __popcll(m & ~lb);
        c1 += __popcll(m & lb);
    }
    cnt[(t * T + tile) * 2 + 0] = c0;
    cnt[(t * T + tile) * 2 + 1] = c1;
}

hipError_t ivf_count(const Store st, int32_t k, int64_t d, int32_t kt, int32_t T, const int32_t* iperm,
                     int32_t n_moving, IvfBuildWs w, hipStream_t s) {
    const int64_t W64 = ivf_w64(k);
    hipError_t e = fill_u64(w.bm, 0ull, W64 * d, s);
    if (e != hipSuccess) return e;
    int64_t blocks = ((int64_t)k * 64 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_ivf_bits, dim3((unsigned)blocks), dim3(256), 0, s, st, k, d, iperm, w.bm);
    hipLaunchKernelGGL(k_lam_bits, dim3((unsigned)((W64 + 255) / 256)), dim3(256), 0, s, k, n_moving, w.lbits);
    int64_t nt = d * T;
    hipLaunchKernelGGL(k_ivf_counts, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, w.bm, w.lbits, d, kt, T,
                       W64, w.pre0, w.pre1, w.cnt);
    return hipGetLastError();
}

__global__ void k_ivf_seg(const int64_t* __restrict__ off, const int64_t* __restrict__ cnt, int64_t d, int32_t T,
                          int64_t* __restrict__ seg, int32_t* __restrict__ mid) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t nt = d * T;
    if (idx < nt) {
        seg[idx] = off[idx * 2];
        mid[idx] = (int32_t)cnt[idx * 2];
    } else if (idx == nt) {
        seg[nt] = off[nt * 2];
    }
}

hipError_t ivf_offsets(int64_t d, int32_t T, IvfBuildWs w, int64_t* seg, int32_t* mid, hipStream_t s) {
    const int64_t n = d * T * 2;
    hipError_t e = exclusive_scan_i64(w.cnt, w.off, n, w.scan_ws, s);
    if (e != hipSuccess) return e;
    int64_t nt = d * T + 1;
    hipLaunchKernelGGL(k_ivf_seg, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, w.off, w.cnt, d, T, seg, mid);
    return hipGetLastError();
}

__global__ void k_ivf_fill(Store st, int32_t k, int64_t d, int32_t kt, int32_t T, const int32_t* __restrict__ iperm,
                           int32_t n_moving,
                           const unsigned long long* __restrict__ bm, const unsigned long long* __restrict__ lbits,
                           const uint16_t* __restrict__ pre0, const uint16_t* __restrict__ pre1,
                           const int64_t* __restrict__ off, uint16_t* __restrict__ cid, float* __restrict__ v32,
                           uint16_t* __restrict__ v16, double* __restrict__ v64) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < k; j += nw) {
        const int64_t q = iperm[j];
        const int part = q >= n_moving ? 1 : 0;
        const int64_t tile = q / kt, w = q >> 6;
        const unsigned long long below = (1ull << (q & 63)) - 1ull;
        const unsigned long long pm = part ? lbits[w] : ~lbits[w];
        const uint16_t* pre = part ? pre1 : pre0;
        const uint16_t local = (uint16_t)(q - tile * kt);
        const int64_t b = st.start[j], m = st.nnz[j];
        for (int64_t p = lane; p < m; p += 64) {
            const int64_t t = st.term[b + p];
            const double u = st.val[b + p];
            const int64_t rank = pre[w * d + t] + __popcll(bm[w * d + t] & pm & below);
            const int64_t pos = off[(t * T + tile) * 2 + part] + rank;
            cid[pos] = local;
            const float f = (float)u;  // round to nearest even
            if (v32) v32[pos] = f;
            if (v16) v16[pos] = f32_to_bf16_rne(f);
            v64[pos] = u;
        }
    }
}

hipError_t ivf_fill(const Store st, int32_t k, int64_t d, int32_t kt, int32_t T, const int32_t* iperm,
                    int32_t n_moving, IvfBuildWs w, uint16_t* cid, float* v32, uint16_t* v16, double* v64,
                    hipStream_t s) {
    int64_t blocks = ((int64_t)k * 64 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_ivf_fill, dim3((unsigned)blocks), dim3(256), 0, s, st, k, d, kt, T, iperm, n_moving, w.bm,
                       w.lbits, w.pre0, w.pre1, w.off, cid, v32, v16, v64);
    return hipGetLastError();
}

// ---------------------------------------------------------------- dense head rows
// A memory layout of this implementation (not the paper's): a term whose
// lists hold at least min_len postings gets a row of kpad = T * ktp values,
// one per centroid id (zero where the centroid lacks the term), rounded to
// the posting dtype exactly as its postings are.  Rows are numbered in term
// order.  Each tile's kt centroids take ktp = kt rounded up to 512 slots.
// FP32 rows hold the tile's centroids in order.  BF16 rows interleave each
// 512-centroid block so that one 16-byte load gives a lane both of its
// 4-centroid groups: slots 8l..8l+3 hold centroids 4l..4l+3 of the block,
// slots 8l+4..8l+7 centroids 256+4l..256+4l+3.
// Slot of position c (0 <= c < ktp) inside a tile's part of a row.
__device__ inline int32_t tile_slot(int32_t c, bool bf16) {
    if (!bf16) return c;
    const int32_t i = c & 511;
    return (c & ~511) + 8 * ((i & 255) >> 2) + 4 * (i >> 8) + (i & 3);
}

__device__ inline int64_t head_slot(int32_t j, int32_t kt, int32_t ktp, bool bf16) {
    const int32_t tile = j / kt, jj = j - tile * kt;
    return (int64_t)tile * ktp + tile_slot(jj, bf16);
}
__global__ void k_head_flags(const int64_t* __restrict__ seg, int64_t d, int32_t T, int64_t min_len,
                             int64_t* __restrict__ flag) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= d) return;
    flag[t] = (seg[(t + 1) * T] - seg[t * T] >= min_len) ? 1 : 0;
}

__global__ void k_head_index(const int64_t* __restrict__ flag, const int64_t* __restrict__ scan, int64_t d,
                             int32_t* __restrict__ head) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= d) return;
    head[t] = flag[t] ? (int32_t)scan[t] : -1;
}

__global__ void k_head_zero(uint32_t* __restrict__ w, int64_t nw) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nw; i += stride) w[i] = 0u;
}

// one wave per centroid: scatter its head-term values into the rows
__global__ void k_head_scatter(Store st, int32_t k, const int32_t* __restrict__ head, const int32_t* __restrict__ iperm,
                               int64_t kpad, int32_t kt, int32_t ktp, float* __restrict__ h32,
                               uint16_t* __restrict__ h16) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < k; j += nw) {
        const int64_t b = st.start[j], m = st.nnz[j];
        for (int64_t p = lane; p < m; p += 64) {
            const int32_t r = head[st.term[b + p]];
            if (r >= 0) {
                const float f = (float)st.val[b + p];  // round to nearest even
                if (h32) h32[r * kpad + head_slot(iperm[j], kt, ktp, false)] = f;
                else h16[r * kpad + head_slot(iperm[j], kt, ktp, true)] = f32_to_bf16_rne(f);
            }
        }
    }
}

// Tile-major copy of the segment bounds for the walk: one 16-byte record per
// (tile, term) holding the segment start, its length and moving length (each
// at most kt <= 4096, so 16 bits apiece) and the term's dense head row (-1:
// none, or head == nullptr).  A launch over one tile then reads a 16*d-byte
// slice with one load per term instead of three scattered over the whole
// term-major table.
__global__ void k_seg_records(const int64_t* __restrict__ seg, const int32_t* __restrict__ mid,
                              const int32_t* __restrict__ head, int64_t d, int32_t T, uint4* __restrict__ rec) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= d * T) return;
    const int64_t tile = idx / d, t = idx - tile * d;
    const int64_t s0 = seg[t * T + tile], len = seg[t * T + tile + 1] - s0;
    const uint32_t mv = (uint32_t)mid[t * T + tile];
    uint4 r;
    r.x = (uint32_t)(uint64_t)s0;
    r.y = (uint32_t)((uint64_t)s0 >> 32);
    r.z = (uint32_t)len | (mv << 16);
    r.w = (uint32_t)(head ? head[t] : -1);
    rec[idx] = r;
}

hipError_t seg_records(const int64_t* seg, const int32_t* mid, const int32_t* head, int64_t d, int32_t T, uint4* rec,
                       hipStream_t s) {
    const int64_t n = d * T;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_records, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seg, mid, head, d, T, rec);
    return hipGetLastError();
}

hipError_t head_flags(const int64_t* seg, int64_t d, int32_t T, int64_t min_len, int64_t* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_head_flags, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, s, seg, d, T, min_len, flag);
    return hipGetLastError();
}

hipError_t head_index(const int64_t* flag, const int64_t* scan, int64_t d, int32_t* head, hipStream_t s) {
    hipLaunchKernelGGL(k_head_index, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, s, flag, scan, d, head);
    return hipGetLastError();
}

hipError_t head_fill(const Store st, int32_t k, const int32_t* head, const int32_t* iperm, int64_t kpad, int32_t kt,
                     int32_t ktp, int64_t H, int pdt_bf16, void* hval, hipStream_t s) {
    const int64_t bytes = H * kpad * (pdt_bf16 ? 2 : 4);
    const int64_t nw = (bytes + 3) / 4;
    if (nw == 0) return hipSuccess;
    int64_t zb = (nw + 255) / 256;
    if (zb > 65536) zb = 65536;
    hipLaunchKernelGGL(k_head_zero, dim3((unsigned)zb), dim3(256), 0, s, (uint32_t*)hval, nw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t blocks = ((int64_t)k * 64 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_head_scatter, dim3((unsigned)blocks), dim3(256), 0, s, st, k, head, iperm, kpad, kt, ktp,
                       pdt_bf16 ? nullptr : (float*)hval, pdt_bf16 ? (uint16_t*)hval : nullptr);
    return hipGetLastError();
}

// ---------------------------------------------------------------- export to the paper's layout
__global__ void k_exp_counts(const int64_t* __restrict__ seg, const int32_t* __restrict__ mid, int64_t d, int32_t T,
                             int64_t* __restrict__ cnt, int32_t* __restrict__ split) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= d) return;
    cnt[t] = seg[(t + 1) * T] - seg[t * T];
    int64_t sp = 0;
    for (int32_t tile = 0; tile < T; ++tile) sp += mid[t * T + tile];
    if (split) split[t] = (int32_t)sp;
}

__global__ void k_exp_fill(const int64_t* __restrict__ seg, const int32_t* __restrict__ mid,
                           const uint16_t* __restrict__ cid, const double* __restrict__ v64, int64_t d, int32_t T,
                           int32_t kt, const int32_t* __restrict__ perm, const int64_t* __restrict__ tptr,
                           int32_t* __restrict__ p_cid,
                           double* __restrict__ p_val) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t t = wave; t < d; t += nw) {
        int64_t o = tptr[t];
        for (int part = 0; part < 2; ++part) {
            for (int32_t tile = 0; tile < T; ++tile) {
                int64_t s0 = seg[t * T + tile], s1 = seg[t * T + tile + 1], sm = s0 + mid[t * T + tile];
                int64_t lo = part ? sm : s0, hi = part ? s1 : sm;
                for (int64_t p = lo + lane; p < hi; p += 64) {
                    if (p_cid) p_cid[o + (p - lo)] = perm[(int32_t)cid[p] + tile * kt];
                    if (p_val) p_val[o + (p - lo)] = v64[p];
                }
                o += hi - lo;
            }
        }
    }
}

hipError_t ivf_export(const sivf_ivf* f, int64_t* term_ptr, int32_t* split, int32_t* p_cid, double* p_val,
                      int64_t* ws_counts, int64_t* scan_ws, hipStream_t s) {
    const int64_t d = f->d;
    hipLaunchKernelGGL(k_exp_counts, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, s, f->seg, f->mid, d, f->T,
                       ws_counts, split);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!term_ptr) return hipSuccess;
    e = exclusive_scan_i64(ws_counts, term_ptr, d, scan_ws, s);
    if (e != hipSuccess) return e;
    if (!p_cid && !p_val) return hipSuccess;
    int64_t blocks = (d * 64 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_exp_fill, dim3((unsigned)blocks), dim3(256), 0, s, f->seg, f->mid, f->cid, f->v64, d, f->T,
                       f->kt, f->perm, term_ptr, p_cid, p_val);
    return hipGetLastError();
}

}  // namespace sivf
