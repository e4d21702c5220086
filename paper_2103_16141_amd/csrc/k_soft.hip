// Soft spherical assignment (the differentiable form of the assignment step):
//   S = X C^T, lse_i = log sum_j exp(S_ij / tau), loss = -sum_i lse_i,
//   backward: P = exp(S/tau - lse), dS = -g P / tau, dC = dS^T X,
//             dX_it = sum_j dS_ij C_jt on X's nonzeros (sampled dense-dense product).
//
// Layout: C arrives k x d row-major; the kernels gather rows of C^T (d x k,
// each a contiguous k-vector) per object nonzero.  The columns are split into
// 8 groups, one per XCD (workgroup b takes group b mod 8), so that each XCD's
// L2 holds its group's slices of the hot terms' rows; a workgroup of 256
// threads owns one (row, group) at a time.  The forward keeps a per-group max
// and sum-exp of S / tau and merges the groups in order.  Nothing of size
// N x k is kept: the backward recomputes S per row and materialises dS only
// for a chunk of rows, from which dC is accumulated term-major over a CSC copy
// of X whose lists are in ascending row order, chunk after chunk.  Every sum
// has a fixed order, so results are run-to-run deterministic.
#include <algorithm>

#include "internal.h"
#include "soft.h"
#include "wave.h"

namespace sivf {

constexpr int kSoftThreads = 256;
constexpr int kSoftTermsInLds = 256;                // forward: row entries staged per pass

// ---------------------------------------------------------------- transpose
// out[c][r] = in[r][c] for an R x Cn row-major matrix; 64x64 tiles via LDS.
__global__ __launch_bounds__(256) void k_transpose_f32(const float* __restrict__ in, float* __restrict__ out, int64_t R,
                                                       int64_t Cn) {
    __shared__ float tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (int y = ty; y < 64; y += 4) {
        const int64_t r = r0 + y, c = c0 + tx;
        tile[y][tx] = (r < R && c < Cn) ? in[r * Cn + c] : 0.0f;
    }
    __syncthreads();
    for (int y = ty; y < 64; y += 4) {
        const int64_t c = c0 + y, r = r0 + tx;
        if (c < Cn && r < R) out[c * R + r] = tile[tx][y];
    }
}

hipError_t soft_transpose(const float* in, float* out, int64_t R, int64_t Cn, hipStream_t s) {
    dim3 grid((unsigned)((Cn + 63) / 64), (unsigned)((R + 63) / 64));
    hipLaunchKernelGGL(k_transpose_f32, grid, dim3(256), 0, s, in, out, R, Cn);
    return hipGetLastError();
}

// ---------------------------------------------------------------- block helpers
__device__ inline float block_max_f32(float v, float* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    float r = sh[0];
    for (int w = 1; w < kSoftThreads / 64; ++w) r = fmaxf(r, sh[w]);
    return r;
}

__device__ inline float block_sum_f32(float v, float* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    float r = 0.0f;
    for (int w = 0; w < kSoftThreads / 64; ++w) r += sh[w];
    return r;
}

// ---------------------------------------------------------------- forward by column groups
// Workgroups are dispatched to the 8 XCDs in turn, so workgroup b runs on XCD
// b mod 8.  Workgroup b takes column group x = b mod 8, columns
// [x kc, (x + 1) kc) with kc = ceil(k / 8) rounded up to a multiple of 4, for
// every row it visits: each XCD then gathers only its group's slice of a
// C^T row (2 KB at k = 4096), so the hot terms' slices stay in its L2.  A
// workgroup sums S for 512 columns at a time (thread (c4, h): columns
// 4 c4 .. 4 c4 + 3, the h-th half of the terms in order; the halves are added
// h = 0 first) and keeps the group's max of S / tau and sum of exp(S / tau -
// max); k_soft_lse_combine merges the 8 groups of a row in group order.
constexpr int kSoftGroups = 8;
constexpr int kFwdCols = 512;   // columns per pass of a workgroup

__host__ __device__ inline int64_t soft_group_width(int64_t k) {
    return ((k + kSoftGroups - 1) / kSoftGroups + 3) & ~(int64_t)3;
}

__global__ __launch_bounds__(kSoftThreads) void k_soft_fwd_part(int64_t N, const int64_t* __restrict__ rp,
                                                                const int32_t* __restrict__ col,
                                                                const float* __restrict__ xv,
                                                                const float* __restrict__ CT, int32_t k, float inv_tau,
                                                                float* __restrict__ pmax, float* __restrict__ psum) {
    __shared__ int32_t s_t[kSoftTermsInLds];
    __shared__ float s_v[kSoftTermsInLds];
    __shared__ float4 half1[kFwdCols / 4];
    __shared__ float sh[kSoftThreads / 64];
    const int x = blockIdx.x % kSoftGroups;
    const int64_t kc = soft_group_width(k);
    const int64_t g0 = min((int64_t)k, x * kc), g1 = min((int64_t)k, g0 + kc);
    const int c4 = threadIdx.x % (kFwdCols / 4), h = threadIdx.x / (kFwdCols / 4);
    const int64_t rstride = gridDim.x / kSoftGroups;
    for (int64_t i = blockIdx.x / kSoftGroups; i < N; i += rstride) {
        const int64_t r0 = rp[i];
        const int n = (int)(rp[i + 1] - r0);
        float m = -INFINITY, z = 0.0f;
        for (int64_t cb = g0; cb < g1; cb += kFwdCols) {
            const int64_t c = cb + 4 * c4;   // this thread's first column
            const bool vec = (k & 3) == 0 && c + 4 <= g1;
            float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            for (int h0 = 0; h0 < n; h0 += kSoftTermsInLds) {
                const int mm = min(kSoftTermsInLds, n - h0);
                __syncthreads();
                for (int e = threadIdx.x; e < mm; e += kSoftThreads) {
                    s_t[e] = col[r0 + h0 + e];
                    s_v[e] = xv[r0 + h0 + e];
                }
                __syncthreads();
                const int half = (mm + 1) / 2;
                const int lo = h == 0 ? 0 : half, hi = h == 0 ? half : mm;
                if (vec) {
                    // four terms' slices in flight, then their products in term order
                    for (int e0 = lo; e0 < hi; e0 += 4) {
                        float4 g[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int e = min(e0 + u, hi - 1);
                            g[u] = *reinterpret_cast<const float4*>(CT + (int64_t)s_t[e] * k + c);
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (e0 + u < hi) {
                                const float v = s_v[e0 + u];
                                acc.x = fmaf(v, g[u].x, acc.x);
                                acc.y = fmaf(v, g[u].y, acc.y);
                                acc.z = fmaf(v, g[u].z, acc.z);
                                acc.w = fmaf(v, g[u].w, acc.w);
                            }
                        }
                    }
                } else if (c < g1) {
                    for (int e = lo; e < hi; ++e) {
                        const float v = s_v[e];
                        const float* row = CT + (int64_t)s_t[e] * k + c;
                        acc.x = fmaf(v, row[0], acc.x);
                        if (c + 1 < g1) acc.y = fmaf(v, row[1], acc.y);
                        if (c + 2 < g1) acc.z = fmaf(v, row[2], acc.z);
                        if (c + 3 < g1) acc.w = fmaf(v, row[3], acc.w);
                    }
                }
            }
            // S = first half + second half
            __syncthreads();
            if (h == 1) half1[c4] = acc;
            __syncthreads();
            float lm = -INFINITY;
            if (h == 0) {
                const float4 o = half1[c4];
                acc.x = acc.x + o.x;
                acc.y = acc.y + o.y;
                acc.z = acc.z + o.z;
                acc.w = acc.w + o.w;
                if (c + 0 < g1) lm = fmaxf(lm, acc.x * inv_tau);
                if (c + 1 < g1) lm = fmaxf(lm, acc.y * inv_tau);
                if (c + 2 < g1) lm = fmaxf(lm, acc.z * inv_tau);
                if (c + 3 < g1) lm = fmaxf(lm, acc.w * inv_tau);
            }
            const float cm = block_max_f32(lm, sh);
            const float nm = fmaxf(m, cm);
            float ls = 0.0f;
            if (h == 0) {
                if (c + 0 < g1) ls += expf(acc.x * inv_tau - nm);
                if (c + 1 < g1) ls += expf(acc.y * inv_tau - nm);
                if (c + 2 < g1) ls += expf(acc.z * inv_tau - nm);
                if (c + 3 < g1) ls += expf(acc.w * inv_tau - nm);
            }
            const float cs = block_sum_f32(ls, sh);
            z = z * expf(m - nm) + cs;
            m = nm;
        }
        if (threadIdx.x == 0) {
            pmax[i * kSoftGroups + x] = m;
            psum[i * kSoftGroups + x] = z;
        }
    }
}

// lse_i = M + log sum_x psum_x exp(pmax_x - M), M = max_x pmax_x, groups in order
// (a group without columns has pmax = -inf, psum = 0)
__global__ void k_soft_lse_combine(int64_t N, const float* __restrict__ pmax, const float* __restrict__ psum,
                                   float* __restrict__ lse) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    float M = -INFINITY;
#pragma unroll
    for (int x = 0; x < kSoftGroups; ++x) M = fmaxf(M, pmax[i * kSoftGroups + x]);
    float z = 0.0f;
#pragma unroll
    for (int x = 0; x < kSoftGroups; ++x) {
        const float px = pmax[i * kSoftGroups + x];
        if (px > -INFINITY) z += psum[i * kSoftGroups + x] * expf(px - M);
    }
    lse[i] = M + logf(z);
}

// loss = -sum_i lse_i in FP64: each thread sums a contiguous range in order,
// then a fixed tree; one workgroup, so the order never changes.
__global__ __launch_bounds__(1024) void k_soft_loss(const float* __restrict__ lse, int64_t N, double* __restrict__ out) {
    __shared__ double sh[1024];
    const int64_t per = (N + 1023) / 1024;
    const int64_t lo = (int64_t)threadIdx.x * per, hi = min(N, lo + per);
    double acc = 0.0;
    for (int64_t i = lo; i < hi; ++i) acc += (double)lse[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = -sh[0];
}

hipError_t soft_forward(int64_t N, const int64_t* rp, const int32_t* col, const float* xv, const float* CT, int32_t k,
                        float tau, float* lse, double* loss_dev, float* pmax, float* psum, int n_cu, hipStream_t s) {
    if (N > 0) {
        // a multiple of the group count, so every workgroup keeps its group
        const int64_t per_group = std::min<int64_t>(N, (int64_t)n_cu * 8 / kSoftGroups);
        hipLaunchKernelGGL(k_soft_fwd_part, dim3((unsigned)(per_group * kSoftGroups)), dim3(kSoftThreads), 0, s, N, rp,
                           col, xv, CT, k, 1.0f / tau, pmax, psum);
        hipLaunchKernelGGL(k_soft_lse_combine, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, pmax, psum, lse);
    }
    hipLaunchKernelGGL(k_soft_loss, dim3(1), dim3(1024), 0, s, lse, N, loss_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------- backward, rows of one chunk
// For rows [c0, c1): recompute S, write dS (row-major, k columns) and dX on the
// row's nonzeros, reading each gathered C^T value once.  Two kernels share the
// rows: those of at most kRegTerms terms go to k_soft_bwd_rows_reg, which
// keeps the gathered slices in registers (further below); the longer ones go
// to k_soft_bwd_rows, which stages them in LDS as follows.
//
// Workgroup b takes column group b mod 8 (the forward's groups: one per XCD)
// of each row it visits and walks the group's columns in blocks of W.  For a
// block it stages the row's C^T slices (W floats per term, kBwTerms terms per
// batch) in LDS, then
//   S:  thread (c, h) sums the h-th of 256 / W contiguous ranges of the terms
//       for column c (in term order), and the ranges' sums are added in order;
//   dS: -g exp(S / tau - lse) / tau, written out and kept in LDS;
//   dX: thread j dots dS with term j's slice (columns in order, four
//       interleaved partial sums added in a fixed order) and adds the block's
//       dot to its running dX_j, blocks in column order; the group's dX_j goes
//       to a partial array, and k_soft_dx_combine adds the 8 groups in order.
// Rows with more than kBwTerms terms stage their terms batch by batch and
// gather each batch a second time for dX.  Rows are W + 4 floats apart, so a
// term's slice and dS are read 16 bytes at a time in the dX pass; the S pass
// reads consecutive columns.  W = 64 and 136 terms keep the LDS of a
// workgroup under 40 KB, four workgroups per CU.
// Workgroup barrier for data exchanged through LDS only: waits for the
// wave's LDS operations, not for its global loads and stores, so gathers for
// the next block and the dS row stores stay in flight across it.
__device__ inline void bw_bar() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kBwTerms = 136;
constexpr int kBwPre = 8;   // float4 gathers per thread in flight

template <int W>
struct BwLds {
    static constexpr int kS = kSoftThreads / W;   // threads per column in the S pass
    static constexpr int kStride = W + 4;          // floats between two terms' slices
    alignas(16) float L[kBwTerms * kStride];
    alignas(16) float P[kS][W];
    alignas(16) float D[W];
    int32_t t[kBwTerms];
    float v[kBwTerms];
};

// term ids and values of entries [t0, t0 + m) of the row
template <int W>
__device__ inline void bw_stage_terms(BwLds<W>& sh, const int32_t* __restrict__ col, const float* __restrict__ xv,
                                      int64_t r0, int t0, int m) {
    for (int e = threadIdx.x; e < m; e += kSoftThreads) {
        sh.t[e] = col[r0 + t0 + e];
        sh.v[e] = xv[r0 + t0 + e];
    }
}

// g[u] = C^T[t_e][cb + 4q .. +3] for slot e = e0 + u * 256 + tid (e = term * W/4 + q).
// The 16-byte path and the element path are separate loops, so the former
// stays one 16-byte load per slot.
template <int W>
__device__ inline void bw_gather(const BwLds<W>& sh, const float* __restrict__ CT, int32_t k, int64_t cb, int64_t lim,
                                 int m, int e0, float4 (&g)[kBwPre]) {
    constexpr int per = W / 4;
    const int tot = m * per;
    if ((k & 3) == 0 && cb + W <= lim) {
        // the slots' term ids first (one LDS wait), then the loads
        int32_t tt[kBwPre];
#pragma unroll
        for (int u = 0; u < kBwPre; ++u) {
            const int e = min(e0 + u * kSoftThreads + (int)threadIdx.x, tot - 1);
            tt[u] = sh.t[e / per];
        }
#pragma unroll
        for (int u = 0; u < kBwPre; ++u) {
            const int e = e0 + u * kSoftThreads + threadIdx.x;
            g[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (e < tot) g[u] = *reinterpret_cast<const float4*>(CT + (int64_t)tt[u] * k + cb + 4 * (e % per));
        }
    } else {
        for (int u = 0; u < kBwPre; ++u) {
            const int e = e0 + u * kSoftThreads + threadIdx.x;
            g[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (e < tot) {
                const float* src = CT + (int64_t)sh.t[e / per] * k + cb + 4 * (e % per);
                const int64_t c = cb + 4 * (e % per);
                g[u].x = c + 0 < lim ? src[0] : 0.0f;
                g[u].y = c + 1 < lim ? src[1] : 0.0f;
                g[u].z = c + 2 < lim ? src[2] : 0.0f;
                g[u].w = c + 3 < lim ? src[3] : 0.0f;
            }
        }
    }
}

template <int W>
__device__ inline void bw_put(BwLds<W>& sh, int m, int e0, const float4 (&g)[kBwPre]) {
    constexpr int per = W / 4;
    const int tot = m * per;
#pragma unroll
    for (int u = 0; u < kBwPre; ++u) {
        const int e = e0 + u * kSoftThreads + threadIdx.x;
        if (e < tot) *reinterpret_cast<float4*>(sh.L + (e / per) * BwLds<W>::kStride + 4 * (e % per)) = g[u];
    }
}

// L[e][c] = C^T[t_e][cb + c] for e < m, c < W (columns >= lim read as 0)
template <int W>
__device__ inline void bw_stage_slices(BwLds<W>& sh, const float* __restrict__ CT, int32_t k, int64_t cb, int64_t lim,
                                       int m) {
    const int tot = m * (W / 4);
    for (int e0 = 0; e0 < tot; e0 += kBwPre * kSoftThreads) {
        float4 g[kBwPre];
        bw_gather<W>(sh, CT, k, cb, lim, m, e0, g);
        bw_put<W>(sh, m, e0, g);
    }
}

// dot of D[0..w) with L row j, four interleaved partial sums in a fixed order
// (D is zero past w and the slice's loaded columns, so whole groups of 4 are
// summed; columns past w in the slice are zero too)
template <int W>
__device__ inline float bw_dot(const BwLds<W>& sh, int j, int w) {
    const float* row = sh.L + j * BwLds<W>::kStride;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    for (int c = 0; c < w; c += 4) {
        const float4 r = *reinterpret_cast<const float4*>(row + c);
        const float4 d = *reinterpret_cast<const float4*>(sh.D + c);
        a0 = fmaf(d.x, r.x, a0);
        a1 = fmaf(d.y, r.y, a1);
        a2 = fmaf(d.z, r.z, a2);
        a3 = fmaf(d.w, r.w, a3);
    }
    return (a0 + a1) + (a2 + a3);
}

// S of the staged terms [0, m) for column c, partial range h, then the block's
// dS (written to dsrow and D); all threads take part
template <int W>
__device__ inline float bw_s_partial(const BwLds<W>& sh, int m, int c, int h) {
    constexpr int kS = BwLds<W>::kS;
    const int q = (m + kS - 1) / kS;
    const int lo = min(m, h * q), hi = min(m, lo + q);
    float s = 0.0f;
    for (int e = lo; e < hi; ++e) s = fmaf(sh.v[e], sh.L[e * BwLds<W>::kStride + c], s);
    return s;
}

template <int W>
__device__ inline void bw_ds(BwLds<W>& sh, float s, int c, int h, int w, float inv_tau, float neg_g_over_tau, float l,
                             float* dsrow, int64_t cb) {
    constexpr int kS = BwLds<W>::kS;
    sh.P[h][c] = s;
    bw_bar();
    if (h == 0) {
        float st = sh.P[0][c];
#pragma unroll
        for (int r = 1; r < kS; ++r) st = st + sh.P[r][c];
        const float ds = c < w ? neg_g_over_tau * expf(st * inv_tau - l) : 0.0f;
        sh.D[c] = ds;
        if (c < w) dsrow[cb + c] = ds;
    }
    bw_bar();
}

// Rows of at most kRegTerms terms (nearly every row of a Poisson(100) corpus)
// go to k_soft_bwd_rows_reg: kRegQ lanes per term slice (4 kRegQ columns per
// block), kRegU register rounds of 256 / kRegQ terms.  Measured at the full
// shape: slices of 8 or 4 lanes (6 and 8 waves per SIMD) are slower, the
// extra shuffle steps and barriers outweighing the occupancy.
constexpr int kRegQ = 16, kRegU = 8;
constexpr int kRegTerms = kRegU * (kSoftThreads / kRegQ);

__device__ inline bool bw_short_row(int n) { return n <= kRegTerms; }

template <int W>
__global__ __launch_bounds__(kSoftThreads) void k_soft_bwd_rows(int64_t c0, int64_t c1, const int64_t* __restrict__ rp,
                                                                const int32_t* __restrict__ col,
                                                                const float* __restrict__ xv,
                                                                const float* __restrict__ CT, int32_t k, float inv_tau,
                                                                float neg_g_over_tau, const float* __restrict__ lse,
                                                                float* __restrict__ dS, float* __restrict__ dxp) {
    __shared__ BwLds<W> sh;
    const int c = threadIdx.x % W, h = threadIdx.x / W;
    const int x = blockIdx.x % kSoftGroups;
    const int64_t kc = soft_group_width(k);
    const int64_t g0 = min((int64_t)k, x * kc), g1 = min((int64_t)k, g0 + kc);
    const int64_t pbase = rp[c0];
    for (int64_t i = c0 + blockIdx.x / kSoftGroups; i < c1; i += gridDim.x / kSoftGroups) {
        const int64_t r0 = rp[i];
        const int n = (int)(rp[i + 1] - r0);
        if (bw_short_row(n)) continue;   // k_soft_bwd_rows_reg takes it
        const int nb = (n + kBwTerms - 1) / kBwTerms;
        const float l = lse[i];
        float* dsrow = dS + (i - c0) * (int64_t)k;
        float* dxrow = dxp + (r0 - pbase) * kSoftGroups + x;   // entry e at dxrow[e * 8]
        bw_bar();
        if (nb == 1) bw_stage_terms<W>(sh, col, xv, r0, 0, n);
        float dxr = 0.0f;   // dX of term threadIdx.x in this group (one batch only)
        for (int64_t cb = g0; cb < g1; cb += W) {
            const int w = (int)min((int64_t)W, g1 - cb);
            float s = 0.0f;
            for (int b = 0; b < nb; ++b) {
                const int t0 = b * kBwTerms, m = min(kBwTerms, n - t0);
                bw_bar();
                if (nb > 1) {
                    bw_stage_terms<W>(sh, col, xv, r0, t0, m);
                    bw_bar();
                }
                bw_stage_slices<W>(sh, CT, k, cb, g1, m);
                bw_bar();
                s += bw_s_partial<W>(sh, m, c, h);
            }
            bw_ds<W>(sh, s, c, h, w, inv_tau, neg_g_over_tau, l, dsrow, cb);
            if (nb == 1) {
                if (threadIdx.x < n) dxr += bw_dot<W>(sh, threadIdx.x, w);
            } else {
                for (int b = 0; b < nb; ++b) {
                    const int t0 = b * kBwTerms, m = min(kBwTerms, n - t0);
                    bw_bar();
                    bw_stage_terms<W>(sh, col, xv, r0, t0, m);
                    bw_bar();
                    bw_stage_slices<W>(sh, CT, k, cb, g1, m);
                    bw_bar();
                    if (threadIdx.x < m) {
                        float* q = dxrow + (int64_t)(t0 + threadIdx.x) * kSoftGroups;
                        *q = (cb == g0 ? 0.0f : *q) + bw_dot<W>(sh, threadIdx.x, w);
                    }
                }
            }
        }
        if (nb == 1) {
            if (threadIdx.x < n) dxrow[(int64_t)threadIdx.x * kSoftGroups] = dxr;
        } else if (g0 >= g1) {
            for (int e = threadIdx.x; e < n; e += kSoftThreads) dxrow[(int64_t)e * kSoftGroups] = 0.0f;
        }
    }
}

// The short rows (bw_short_row), without staging the slices in LDS.  For a
// block of 4Q columns, thread (wave v, lane l) holds in registers, for
// u = 0 .. U-1, the four columns 4q .. 4q+3 (q = l mod Q) of term
// u * (256 / Q) + (64 / Q) v + l / Q of the row: a term's slice lies in Q
// consecutive lanes.  Then
//   S:  each thread sums its terms' products in u order; the 64 / Q lane
//       groups of a wave are added by xor shuffles (distance Q, 2Q, ..., 32),
//       the four waves' sums through LDS in wave order;
//   dS: as in k_soft_bwd_rows, from 4Q threads;
//   dX: each thread dots dS with its slot (4 columns in order), the 16 lanes
//       of the term (one DPP row) are added by row rotations (8, 4, 2, 1;
//       through LDS shuffles instead this pass takes 11% longer), and the
//       block's sum goes to the term's running dX, blocks in column order.
// Every lane of such a tree ends with the same value (each step adds two
// partners' values, and addition commutes), and every step has a fixed
// association, so the result is run-to-run identical.  Each gathered value is
// read from memory once and used twice from registers.
template <int Q, int U>
struct RegLds {
    static constexpr int kTerms = U * (kSoftThreads / Q);
    int32_t t[kTerms];
    float v[kTerms];
    alignas(16) float4 P[2][kSoftThreads / 64][Q];
    alignas(16) float D[2][4 * Q];
};

// sum over the 16 lanes of this lane's DPP row (row_ror 8, 4, 2, 1)
__device__ inline float row16_sum(float p) {
    p = p + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(p), 0x128, 0xf, 0xf, false));
    p = p + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(p), 0x124, 0xf, 0xf, false));
    p = p + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(p), 0x122, 0xf, 0xf, false));
    p = p + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(p), 0x121, 0xf, 0xf, false));
    return p;
}

__device__ inline float4 add4(float4 a, float4 b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

__device__ inline float4 shfl_xor4(float4 a, int o) {
    return make_float4(__shfl_xor(a.x, o, 64), __shfl_xor(a.y, o, 64), __shfl_xor(a.z, o, 64), __shfl_xor(a.w, o, 64));
}

template <int Q, int U>
__global__ __launch_bounds__(kSoftThreads) void k_soft_bwd_rows_reg(int64_t c0, int64_t c1,
                                                                    const int64_t* __restrict__ rp,
                                                                    const int32_t* __restrict__ col,
                                                                    const float* __restrict__ xv,
                                                                    const float* __restrict__ CT, int32_t k,
                                                                    float inv_tau, float neg_g_over_tau,
                                                                    const float* __restrict__ lse,
                                                                    float* __restrict__ dS, float* __restrict__ dxp) {
    static_assert(Q == 16, "a term's slice is one DPP row");
    constexpr int kTpr = kSoftThreads / Q;   // terms per register round
    constexpr int kCols = 4 * Q;             // columns per block
    __shared__ RegLds<Q, U> sh;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q = lane % Q, sub = lane / Q;
    const int x = blockIdx.x % kSoftGroups;
    const int64_t kc = soft_group_width(k);
    const int64_t g0 = min((int64_t)k, x * kc), g1 = min((int64_t)k, g0 + kc);
    const int64_t pbase = rp[c0];
    int par = 0;
    for (int64_t i = c0 + blockIdx.x / kSoftGroups; i < c1; i += gridDim.x / kSoftGroups) {
        const int64_t r0 = rp[i];
        const int n = (int)(rp[i + 1] - r0);
        if (n > RegLds<Q, U>::kTerms) continue;   // k_soft_bwd_rows takes it
        const float l = lse[i];
        float* dsrow = dS + (i - c0) * (int64_t)k;
        float* dxrow = dxp + (r0 - pbase) * kSoftGroups + x;   // entry e at dxrow[e * 8]
        __syncthreads();
        for (int e = threadIdx.x; e < n; e += kSoftThreads) {
            sh.t[e] = col[r0 + e];
            sh.v[e] = xv[r0 + e];
        }
        __syncthreads();
        float xu[U], dxr[U];
        int32_t tu[U];   // term id, -1 past the row's end
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = u * kTpr + (64 / Q) * wv + sub;
            xu[u] = e < n ? sh.v[e] : 0.0f;
            tu[u] = e < n ? sh.t[e] : -1;
            dxr[u] = 0.0f;
        }
        for (int64_t cb = g0; cb < g1; cb += kCols) {
            const int w = (int)min((int64_t)kCols, g1 - cb);
            const int64_t cq = cb + 4 * q;   // this lane's first column
            float4 g[U];
            if ((k & 3) == 0 && cq + 4 <= g1) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    g[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (tu[u] >= 0) g[u] = *reinterpret_cast<const float4*>(CT + (int64_t)tu[u] * k + cq);
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    g[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (tu[u] >= 0) {
                        const float* src = CT + (int64_t)tu[u] * k + cq;
                        if (cq + 0 < g1) g[u].x = src[0];
                        if (cq + 1 < g1) g[u].y = src[1];
                        if (cq + 2 < g1) g[u].z = src[2];
                        if (cq + 3 < g1) g[u].w = src[3];
                    }
                }
            }
            float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                a.x = fmaf(xu[u], g[u].x, a.x);
                a.y = fmaf(xu[u], g[u].y, a.y);
                a.z = fmaf(xu[u], g[u].z, a.z);
                a.w = fmaf(xu[u], g[u].w, a.w);
            }
#pragma unroll
            for (int o = Q; o < 64; o <<= 1) a = add4(a, shfl_xor4(a, o));
            if (sub == 0) sh.P[par][wv][q] = a;
            bw_bar();
            if (threadIdx.x < kCols) {
                const int c = threadIdx.x;
                const float* pc = reinterpret_cast<const float*>(&sh.P[par][0][0]) + c;
                float st = pc[0];
#pragma unroll
                for (int v = 1; v < kSoftThreads / 64; ++v) st = st + pc[v * kCols];
                const float ds = c < w ? neg_g_over_tau * expf(st * inv_tau - l) : 0.0f;
                sh.D[par][c] = ds;
                if (c < w) dsrow[cb + c] = ds;
            }
            bw_bar();
            const float4 d = *reinterpret_cast<const float4*>(&sh.D[par][4 * q]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                float p = d.x * g[u].x;
                p = fmaf(d.y, g[u].y, p);
                p = fmaf(d.z, g[u].z, p);
                p = fmaf(d.w, g[u].w, p);
                dxr[u] += row16_sum(p);
            }
            par ^= 1;
        }
        if (q == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (tu[u] >= 0) dxrow[(int64_t)(u * kTpr + (64 / Q) * wv + sub) * kSoftGroups] = dxr[u];
        }
    }
}

// dxv[p] = sum over the 8 column groups, in group order, of dxp[(p - p0) * 8 + x]
__global__ void k_soft_dx_combine(int64_t p0, int64_t p1, const float* __restrict__ dxp, float* __restrict__ dxv) {
    const int64_t p = p0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= p1) return;
    const float* q = dxp + (p - p0) * kSoftGroups;
    float a = q[0];
#pragma unroll
    for (int x = 1; x < kSoftGroups; ++x) a = a + q[x];
    dxv[p] = a;
}

constexpr int kBwW = 64;   // columns per block of the rows pass

hipError_t soft_bwd_rows(int64_t c0, int64_t c1, int64_t p0, int64_t p1, const int64_t* rp, const int32_t* col,
                         const float* xv, const float* CT, int32_t k, float tau, float grad, const float* lse, float* dS,
                         float* dxp, float* dxv, int n_cu, hipStream_t s) {
    if (c1 <= c0) return hipSuccess;
    const int per_cu = std::max(1, (int)(160 * 1024 / sizeof(BwLds<kBwW>)));
    const int64_t per_group = std::min<int64_t>(c1 - c0, (int64_t)n_cu * per_cu / kSoftGroups);
    // short rows, then the rest (each kernel skips the other's rows)
    {
        const void* fn = (const void*)k_soft_bwd_rows_reg<kRegQ, kRegU>;
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kSoftThreads, 0) != hipSuccess || nb < 1) nb = 1;
        const int64_t pg = std::max<int64_t>(1, std::min<int64_t>(c1 - c0, (int64_t)n_cu * nb / kSoftGroups));
        hipLaunchKernelGGL((k_soft_bwd_rows_reg<kRegQ, kRegU>), dim3((unsigned)(pg * kSoftGroups)), dim3(kSoftThreads),
                           0, s, c0, c1, rp, col, xv, CT, k, 1.0f / tau, -grad / tau, lse, dS, dxp);
    }
    hipLaunchKernelGGL((k_soft_bwd_rows<kBwW>), dim3((unsigned)(per_group * kSoftGroups)), dim3(kSoftThreads), 0, s, c0,
                       c1, rp, col, xv, CT, k, 1.0f / tau, -grad / tau, lse, dS, dxp);
    if (p1 > p0)
        hipLaunchKernelGGL(k_soft_dx_combine, dim3((unsigned)((p1 - p0 + 255) / 256)), dim3(256), 0, s, p0, p1, dxp,
                           dxv);
    return hipGetLastError();
}

// ---------------------------------------------------------------- CSC of X (rows ascending per term)
// hist[b][t] (b = block of kCscRows rows) by integer atomics, column scan over
// blocks, then one wave per block walks its rows in order and places each
// entry at colptr[t] + cursor[b][t]++ (terms inside a row are distinct; the
// fence orders one row's cursor updates before the next row's).
constexpr int kCscRows = 1024;

__global__ void k_csc_hist(int64_t N, const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t d,
                           int32_t* __restrict__ hist) {
    const int64_t b = blockIdx.x;
    const int64_t lo = b * kCscRows, hi = min(N, lo + kCscRows);
    for (int64_t i = lo; i < hi; ++i)
        for (int64_t p = rp[i] + threadIdx.x; p < rp[i + 1]; p += blockDim.x) atomicAdd(&hist[b * d + col[p]], 1);
}

__global__ void k_csc_colscan(int64_t nb, int64_t d, int32_t* __restrict__ hist, int64_t* __restrict__ cnt) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= d) return;
    int64_t run = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t h = hist[b * d + t];
        hist[b * d + t] = (int32_t)run;
        run += h;
    }
    cnt[t] = run;
}

__global__ __launch_bounds__(64) void k_csc_fill(int64_t N, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                 const float* __restrict__ xv, int64_t d, int32_t* __restrict__ hist,
                                                 const int64_t* __restrict__ colptr, int32_t* __restrict__ xt_row,
                                                 float* __restrict__ xt_val) {
    const int64_t b = blockIdx.x;
    const int64_t lo = b * kCscRows, hi = min(N, lo + kCscRows);
    int32_t* cur = hist + b * d;
    for (int64_t i = lo; i < hi; ++i) {
        for (int64_t p = rp[i] + threadIdx.x; p < rp[i + 1]; p += 64) {
            const int32_t t = col[p];
            const int32_t r = cur[t];
            cur[t] = r + 1;
            const int64_t pos = colptr[t] + r;
            xt_row[pos] = (int32_t)i;
            xt_val[pos] = xv[p];
        }
        __threadfence_block();
    }
}

hipError_t soft_csc(int64_t N, int64_t d, int64_t nnz, const int64_t* rp, const int32_t* col, const float* xv,
                    int32_t* hist, int64_t* cnt, int64_t* colptr, int64_t* scan_ws, int32_t* xt_row, float* xt_val,
                    hipStream_t s) {
    const int64_t nb = (N + kCscRows - 1) / kCscRows;
    hipError_t e = hipSuccess;
    e = fill_i32(hist, 0, nb * d, s);
    if (e != hipSuccess) return e;
    if (nb > 0) hipLaunchKernelGGL(k_csc_hist, dim3((unsigned)nb), dim3(256), 0, s, N, rp, col, d, hist);
    hipLaunchKernelGGL(k_csc_colscan, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, s, nb, d, hist, cnt);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan_i64(cnt, colptr, d, scan_ws, s);
    if (e != hipSuccess) return e;
    if (nb > 0)
        hipLaunchKernelGGL(k_csc_fill, dim3((unsigned)nb), dim3(64), 0, s, N, rp, col, xv, d, hist, colptr, xt_row, xt_val);
    (void)nnz;
    return hipGetLastError();
}

// ---------------------------------------------------------------- dC^T, term-major, one chunk of rows
// dCT[t][:] (+)= sum over rows i in [c0, c1) containing t, ascending, of v_it * dS[i - c0][:].
//
// A term's rows inside the chunk are the range [lo_t, hi_t) of its ascending
// CSC list.  Zipf term frequencies make a few ranges as long as the chunk
// (the hottest terms occur in nearly every row) while most hold a handful of
// rows, so one workgroup per term would leave the long ranges to a few
// workgroups.  Three kinds of range:
//   * at most `piece` entries: summed by one workgroup per column group
//     straight into dCT[t] (k_dct_short);
//   * more than hot_min entries (a hot term): cut at the chunk's row blocks
//     of blk_rows rows, one piece per block, and the pieces are run block by
//     block across all hot terms (k_dct_rowblock), so the workgroups of an
//     XCD read the same block of dS rows at the same time and mostly from
//     L2;
//   * the rest (mid terms): the same with blocks of mid_blk_rows rows.
// Each piece is summed into a partial row, and k_dct_combine adds a term's
// partial rows into dCT[t] in piece order.  Every sum has a fixed order, so
// the result is run-to-run identical.  The host counts every chunk's pieces
// first (soft_dct_count) and sizes the partial rows for the largest.

// lo/hi of every term's rows inside [c0, c1); np[t] = pieces of a long range
// (else 0); hflag / mflag mark the hot and the mid terms
__global__ void k_dct_plan(int64_t d, int64_t c0, int64_t c1, int64_t piece, int64_t hot_min, int64_t nblk,
                           int64_t nblk_mid, const int64_t* __restrict__ colptr, const int32_t* __restrict__ xt_row,
                           int64_t* __restrict__ lo_out, int64_t* __restrict__ hi_out, int64_t* __restrict__ np,
                           int64_t* __restrict__ hflag, int64_t* __restrict__ mflag) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= d) return;
    const int64_t b = colptr[t], e = colptr[t + 1];
    int64_t lo = b, len = e - b;
    while (len > 0) {
        const int64_t half = len >> 1;
        if (xt_row[lo + half] < c0) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    int64_t hi = lo;
    len = e - lo;
    while (len > 0) {
        const int64_t half = len >> 1;
        if (xt_row[hi + half] < c1) {
            hi += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    lo_out[t] = lo;
    hi_out[t] = hi;
    const int64_t n = hi - lo;
    const bool is_hot = n > hot_min, is_mid = !is_hot && n > piece;
    hflag[t] = is_hot ? 1 : 0;
    mflag[t] = is_mid ? 1 : 0;
    np[t] = is_hot ? nblk : (is_mid ? nblk_mid : 0);
}

// list[scan[t]] = t for the flagged terms
__global__ void k_dct_list(int64_t d, const int64_t* __restrict__ flag, const int64_t* __restrict__ scan,
                           int32_t* __restrict__ list) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < d && flag[t]) list[scan[t]] = (int32_t)t;
}

__global__ void k_dct_store_count(const int64_t* __restrict__ pstart, int64_t d, int64_t* __restrict__ count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *count = pstart[d];
}

// first entry in [lo, hi) of the ascending xt_row whose row is >= r
__device__ inline int64_t row_lower_bound(const int32_t* __restrict__ xt_row, int64_t lo, int64_t hi, int64_t r) {
    int64_t len = hi - lo;
    while (len > 0) {
        const int64_t half = len >> 1;
        if (xt_row[lo + half] < r) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return lo;
}

// item[pstart[t] + j] = t for the pieces j of each long range
__global__ void k_dct_items(int64_t d, int64_t max_pieces, const int64_t* __restrict__ np,
                            const int64_t* __restrict__ pstart, int32_t* __restrict__ item) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= d) return;
    const int64_t e = min(pstart[t] + np[t], max_pieces);
    for (int64_t q = pstart[t]; q < e; ++q) item[q] = (int32_t)t;
}

__global__ void k_chunk_offsets(const int64_t* __restrict__ rp, int64_t n, int64_t rc, int64_t nch,
                                int64_t* __restrict__ out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j <= nch) out[j] = rp[min(j * rc, n)];
}

hipError_t soft_chunk_offsets(const int64_t* rp, int64_t n, int64_t rc, int64_t nch, int64_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_chunk_offsets, dim3((unsigned)((nch + 256) / 256)), dim3(256), 0, s, rp, n, rc, nch, out);
    return hipGetLastError();
}

// Column groups as in the forward: workgroup b takes column group b mod 8
// (one per XCD), so each XCD's L2 holds only its eighth of every dS row
// (backward 113 -> 107 ms at N = 262,144, k = 4,096 against workgroups
// spanning all k columns).  128 threads, four columns each: 512 columns per
// pass of a group.  Each column is summed over the rows in ascending order,
// one fused multiply-add per row.
constexpr int kDctThreads = 128;
constexpr int kDctRowsG = 8;   // rows whose gathers are in flight together

// acc (+)= sum over CSC entries [p0, p1) (rows ascending) of v * dS[row][cq .. cq+3]
__device__ inline void dct_sum_g(int32_t k, int64_t c0, int64_t cq, int64_t g1, int64_t p0, int64_t p1,
                                 const int32_t* __restrict__ xt_row, const float* __restrict__ xt_val,
                                 const float* __restrict__ dS, float4& acc) {
    if ((k & 3) == 0 && cq + 4 <= g1) {
        for (int64_t q0 = p0; q0 < p1; q0 += kDctRowsG) {
            const int m = (int)min((int64_t)kDctRowsG, p1 - q0);
            int64_t ro[kDctRowsG];
            float vv[kDctRowsG];
#pragma unroll
            for (int u = 0; u < kDctRowsG; ++u) {
                const bool in = u < m;
                ro[u] = (int64_t)(xt_row[in ? q0 + u : q0] - c0) * k + cq;
                vv[u] = in ? xt_val[q0 + u] : 0.0f;
            }
            float4 g[kDctRowsG];
#pragma unroll
            for (int u = 0; u < kDctRowsG; ++u) g[u] = *reinterpret_cast<const float4*>(dS + ro[u]);
#pragma unroll
            for (int u = 0; u < kDctRowsG; ++u) {
                if (u < m) {
                    acc.x = fmaf(vv[u], g[u].x, acc.x);
                    acc.y = fmaf(vv[u], g[u].y, acc.y);
                    acc.z = fmaf(vv[u], g[u].z, acc.z);
                    acc.w = fmaf(vv[u], g[u].w, acc.w);
                }
            }
        }
    } else if (cq < g1) {
        for (int64_t p = p0; p < p1; ++p) {
            const float v = xt_val[p];
            const float* row = dS + (int64_t)(xt_row[p] - c0) * k + cq;
            acc.x = fmaf(v, row[0], acc.x);
            if (cq + 1 < g1) acc.y = fmaf(v, row[1], acc.y);
            if (cq + 2 < g1) acc.z = fmaf(v, row[2], acc.z);
            if (cq + 3 < g1) acc.w = fmaf(v, row[3], acc.w);
        }
    }
}

__device__ inline float4 load4_lim(const float* p, int64_t cq, int64_t g1, bool vec) {
    if (vec) return *reinterpret_cast<const float4*>(p);
    float4 a = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (cq + 0 < g1) a.x = p[0];
    if (cq + 1 < g1) a.y = p[1];
    if (cq + 2 < g1) a.z = p[2];
    if (cq + 3 < g1) a.w = p[3];
    return a;
}

__device__ inline void store4_lim(float* p, float4 a, int64_t cq, int64_t g1, bool vec) {
    if (vec) {
        *reinterpret_cast<float4*>(p) = a;
        return;
    }
    if (cq + 0 < g1) p[0] = a.x;
    if (cq + 1 < g1) p[1] = a.y;
    if (cq + 2 < g1) p[2] = a.z;
    if (cq + 3 < g1) p[3] = a.w;
}

// short ranges: one workgroup per (term, column group), straight into dCT[t]
// (zeroed on the first chunk when the term has no row in it)
__global__ __launch_bounds__(kDctThreads) void k_dct_short(int64_t d, int32_t k, int64_t c0, int first,
                                                           const int64_t* __restrict__ np,
                                                           const int64_t* __restrict__ lo_t,
                                                           const int64_t* __restrict__ hi_t,
                                                           const int32_t* __restrict__ xt_row,
                                                           const float* __restrict__ xt_val,
                                                           const float* __restrict__ dS, float* __restrict__ dCT) {
    const int x = blockIdx.x % kSoftGroups;
    const int64_t kc = soft_group_width(k);
    const int64_t g0 = min((int64_t)k, x * kc), g1 = min((int64_t)k, g0 + kc);
    for (int64_t t = blockIdx.x / kSoftGroups; t < d; t += gridDim.x / kSoftGroups) {
        const int64_t lo = lo_t[t], hi = hi_t[t];
        if (np[t] > 0) continue;   // a long range: summed in pieces
        if (lo == hi && !first) continue;
        for (int64_t cb = g0; cb < g1; cb += 4 * kDctThreads) {
            const int64_t cq = cb + 4 * threadIdx.x;
            if (cq >= g1) continue;
            const bool vec = (k & 3) == 0 && cq + 4 <= g1;
            float* out = dCT + t * (int64_t)k + cq;
            float4 acc = first ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : load4_lim(out, cq, g1, vec);
            dct_sum_g(k, c0, cq, g1, lo, hi, xt_row, xt_val, dS, acc);
            store4_lim(out, acc, cq, g1, vec);
        }
    }
}

// the pieces of a list of terms (the hot or the mid ones), block by block:
// piece o covers row block o / H of term list[o mod H] (H = scan[d] terms), so
// concurrent workgroups read one block of dS rows; one column group per
// workgroup
__global__ __launch_bounds__(kDctThreads) void k_dct_rowblock(int64_t d, int64_t max_pieces, int32_t k, int64_t c0,
                                                              int64_t c1, int64_t blk_rows, int64_t nblk,
                                                              const int32_t* __restrict__ list,
                                                              const int64_t* __restrict__ scan,
                                                              const int64_t* __restrict__ pstart,
                                                              const int64_t* __restrict__ lo_t,
                                                              const int64_t* __restrict__ hi_t,
                                                              const int32_t* __restrict__ xt_row,
                                                              const float* __restrict__ xt_val,
                                                              const float* __restrict__ dS, float* __restrict__ part) {
    const int x = blockIdx.x % kSoftGroups;
    const int64_t kc = soft_group_width(k);
    const int64_t g0 = min((int64_t)k, x * kc), g1 = min((int64_t)k, g0 + kc);
    const int64_t H = scan[d];
    for (int64_t o = blockIdx.x / kSoftGroups; o < H * nblk; o += gridDim.x / kSoftGroups) {
        const int64_t j = o / H;
        const int32_t t = list[o - j * H];
        const int64_t q = pstart[t] + j;
        if (q >= max_pieces) continue;   // cannot happen: the host bound holds
        const int64_t r0 = c0 + j * blk_rows, r1 = min(c1, r0 + blk_rows);
        const int64_t p0 = row_lower_bound(xt_row, lo_t[t], hi_t[t], r0);
        const int64_t p1 = row_lower_bound(xt_row, p0, hi_t[t], r1);
        for (int64_t cb = g0; cb < g1; cb += 4 * kDctThreads) {
            const int64_t cq = cb + 4 * threadIdx.x;
            if (cq >= g1) continue;
            const bool vec = (k & 3) == 0 && cq + 4 <= g1;
            float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            dct_sum_g(k, c0, cq, g1, p0, p1, xt_row, xt_val, dS, acc);
            store4_lim(part + q * (int64_t)k + cq, acc, cq, g1, vec);
        }
    }
}

// dCT[t] = (first ? 0 : dCT[t]) + partial rows of t's pieces, added in piece
// order; one workgroup per (long-range term, column group), found at the
// term's first piece; the loads of kCombineAhead partial rows are issued
// before their adds
constexpr int kCombineAhead = 8;

__global__ __launch_bounds__(kDctThreads) void k_dct_combine(int64_t d, int64_t max_pieces, int32_t k, int first,
                                                             const int32_t* __restrict__ item,
                                                             const int64_t* __restrict__ np,
                                                             const int64_t* __restrict__ pstart,
                                                             const float* __restrict__ part,
                                                             float* __restrict__ dCT) {
    const int x = blockIdx.x % kSoftGroups;
    const int64_t kc = soft_group_width(k);
    const int64_t g0 = min((int64_t)k, x * kc), g1 = min((int64_t)k, g0 + kc);
    const int64_t npieces = min(pstart[d], max_pieces);
    for (int64_t q = blockIdx.x / kSoftGroups; q < npieces; q += gridDim.x / kSoftGroups) {
        const int32_t t = item[q];
        if (pstart[t] != q) continue;   // not the term's first piece
        const int64_t m = np[t];
        if (q + m > max_pieces) continue;   // cannot happen: the host bound holds
        for (int64_t cb = g0; cb < g1; cb += 4 * kDctThreads) {
            const int64_t cq = cb + 4 * threadIdx.x;
            if (cq >= g1) continue;
            const bool vec = (k & 3) == 0 && cq + 4 <= g1;
            float* out = dCT + t * (int64_t)k + cq;
            float4 acc = first ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : load4_lim(out, cq, g1, vec);
            const float* pr = part + q * (int64_t)k + cq;
            for (int64_t j0 = 0; j0 < m; j0 += kCombineAhead) {
                float4 v[kCombineAhead];
#pragma unroll
                for (int u = 0; u < kCombineAhead; ++u)
                    v[u] = j0 + u < m ? load4_lim(pr + (j0 + u) * (int64_t)k, cq, g1, vec)
                                      : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                for (int u = 0; u < kCombineAhead; ++u)
                    if (j0 + u < m) acc = add4(acc, v[u]);
            }
            store4_lim(out, acc, cq, g1, vec);
        }
    }
}

static hipError_t dct_plan(int64_t d, int64_t c0, int64_t c1, const int64_t* colptr, const int32_t* xt_row,
                           const DctWs& w, hipStream_t s) {
    const unsigned tb = (unsigned)((d + 255) / 256);
    const int64_t nblk = (c1 - c0 + w.blk_rows - 1) / w.blk_rows;
    const int64_t nblk_mid = (c1 - c0 + w.mid_blk_rows - 1) / w.mid_blk_rows;
    hipLaunchKernelGGL(k_dct_plan, dim3(tb), dim3(256), 0, s, d, c0, c1, w.piece, w.hot_min, nblk, nblk_mid, colptr,
                       xt_row, w.lo, w.hi, w.np, w.hflag, w.mflag);
    hipError_t e = exclusive_scan_i64(w.np, w.pstart, d, w.scan_ws, s);
    if (e == hipSuccess) e = exclusive_scan_i64(w.hflag, w.hscan, d, w.scan_ws, s);
    if (e == hipSuccess) e = exclusive_scan_i64(w.mflag, w.mscan, d, w.scan_ws, s);
    return e;
}

hipError_t soft_dct_count(int64_t d, int64_t c0, int64_t c1, const int64_t* colptr, const int32_t* xt_row, DctWs w,
                          int64_t* count, hipStream_t s) {
    if (d <= 0) return hipSuccess;
    hipError_t e = dct_plan(d, c0, c1, colptr, xt_row, w, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dct_store_count, dim3(1), dim3(64), 0, s, w.pstart, d, count);
    return hipGetLastError();
}

hipError_t soft_dct(int64_t d, int32_t k, int64_t c0, int64_t c1, int first, const int64_t* colptr,
                    const int32_t* xt_row, const float* xt_val, const float* dS, float* dCT, DctWs w, int n_cu,
                    hipStream_t s) {
    if (d <= 0) return hipSuccess;
    const unsigned tb = (unsigned)((d + 255) / 256);
    hipError_t e = dct_plan(d, c0, c1, colptr, xt_row, w, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dct_items, dim3(tb), dim3(256), 0, s, d, w.max_pieces, w.np, w.pstart, w.item);
    hipLaunchKernelGGL(k_dct_list, dim3(tb), dim3(256), 0, s, d, w.hflag, w.hscan, w.hot);
    hipLaunchKernelGGL(k_dct_list, dim3(tb), dim3(256), 0, s, d, w.mflag, w.mscan, w.mid);
    const int64_t grid = std::min<int64_t>(d, (int64_t)n_cu * 16) * kSoftGroups;
    hipLaunchKernelGGL(k_dct_short, dim3((unsigned)grid), dim3(kDctThreads), 0, s, d, k, c0, first, w.np, w.lo,
                       w.hi, xt_row, xt_val, dS, dCT);
    // pieces: at most max_pieces (the host's count of the largest chunk), the
    // exact count is pstart[d] on the device
    if (w.max_pieces > 0) {
        const int64_t pg = std::min<int64_t>(w.max_pieces, (int64_t)n_cu * 16);
        const int64_t nblk = (c1 - c0 + w.blk_rows - 1) / w.blk_rows;
        const int64_t nblk_mid = (c1 - c0 + w.mid_blk_rows - 1) / w.mid_blk_rows;
        hipLaunchKernelGGL(k_dct_rowblock, dim3((unsigned)(pg * kSoftGroups)), dim3(kDctThreads), 0, s, d,
                           w.max_pieces, k, c0, c1, w.blk_rows, nblk, w.hot, w.hscan, w.pstart, w.lo, w.hi, xt_row,
                           xt_val, dS, w.part);
        hipLaunchKernelGGL(k_dct_rowblock, dim3((unsigned)(pg * kSoftGroups)), dim3(kDctThreads), 0, s, d,
                           w.max_pieces, k, c0, c1, w.mid_blk_rows, nblk_mid, w.mid, w.mscan, w.pstart, w.lo, w.hi,
                           xt_row, xt_val, dS, w.part);
        hipLaunchKernelGGL(k_dct_combine, dim3((unsigned)(pg * kSoftGroups)), dim3(kDctThreads), 0, s, d, w.max_pieces,
                           k, first, w.item, w.np, w.pstart, w.part, dCT);
    }
    return hipGetLastError();
}

}  // namespace sivf
