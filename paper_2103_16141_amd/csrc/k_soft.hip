// Soft spherical assignment (the differentiable form of the assignment step):
//   S = X C^T, lse_i = log sum_j exp(S_ij / tau), loss = -sum_i lse_i,
//   backward: P = exp(S/tau - lse), dS = -g P / tau, dC = dS^T X,
//             dX_it = sum_j dS_ij C_jt on X's nonzeros (sampled dense-dense product).
//
// Layout: C arrives k x d row-major; the kernels gather rows of C^T (d x k,
// each a contiguous k-vector) per object nonzero.  One workgroup of 256
// threads owns one object row at a time; each thread holds 16 columns of the
// row's S in registers (4 float4 groups spaced 1024 apart, so each gather is a
// fully coalesced 4 KB read), column chunks of 4096 are merged with an online
// max / sum-exp.  Nothing of size N x k is kept: the backward recomputes S
// per row and materialises dS only for a chunk of rows, from which dC is
// accumulated term-major over a CSC copy of X whose lists are in ascending
// row order, chunk after chunk: a fixed summation order, so results are
// run-to-run deterministic.
#include <algorithm>

#include "internal.h"
#include "wave.h"

namespace sivf {

constexpr int kSoftThreads = 256;
constexpr int kSoftCols = 16;                       // columns per thread per chunk
constexpr int kSoftChunk = kSoftThreads * kSoftCols;  // 4096 columns per chunk
constexpr int kSoftTermsInLds = 256;                // row entries staged per pass
constexpr int kDctRows = 4;                         // dS rows in flight per dC step

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

// Column index of this thread's q-th value (q = 0..15) inside a 4096 chunk.
__device__ inline int soft_col(int q) { return (q >> 2) * (kSoftThreads * 4) + threadIdx.x * 4 + (q & 3); }

// acc[q] = sum over the row's terms of v * CT[t][ch0 + soft_col(q)] (columns >= k read as 0).
__device__ inline void soft_row_chunk(const int64_t r0, const int n, const int32_t* __restrict__ col,
                                      const float* __restrict__ xv, const float* __restrict__ CT, int32_t k,
                                      int64_t ch0, float acc[kSoftCols], int32_t* s_t, float* s_v) {
#pragma unroll
    for (int q = 0; q < kSoftCols; ++q) acc[q] = 0.0f;
    for (int h0 = 0; h0 < n; h0 += kSoftTermsInLds) {
        const int m = min(kSoftTermsInLds, n - h0);
        __syncthreads();
        for (int h = threadIdx.x; h < m; h += kSoftThreads) {
            s_t[h] = col[r0 + h0 + h];
            s_v[h] = xv[r0 + h0 + h];
        }
        __syncthreads();
        const bool full = ch0 + kSoftChunk <= k && (k & 3) == 0;  // float4 gathers stay 16-byte aligned
        for (int h = 0; h < m; ++h) {
            const float v = s_v[h];
            const float* row = CT + (int64_t)s_t[h] * k + ch0;
            if (full) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const float4 c4 = *reinterpret_cast<const float4*>(row + g * (kSoftThreads * 4) + threadIdx.x * 4);
                    acc[4 * g + 0] = fmaf(v, c4.x, acc[4 * g + 0]);
                    acc[4 * g + 1] = fmaf(v, c4.y, acc[4 * g + 1]);
                    acc[4 * g + 2] = fmaf(v, c4.z, acc[4 * g + 2]);
                    acc[4 * g + 3] = fmaf(v, c4.w, acc[4 * g + 3]);
                }
            } else {
#pragma unroll
                for (int q = 0; q < kSoftCols; ++q) {
                    const int64_t c = ch0 + soft_col(q);
                    if (c < k) acc[q] = fmaf(v, row[soft_col(q)], acc[q]);
                }
            }
        }
    }
}

// lse of one row over all k columns (online merge across 4096-column chunks).
__device__ inline float soft_row_lse(const int64_t r0, const int n, const int32_t* __restrict__ col,
                                     const float* __restrict__ xv, const float* __restrict__ CT, int32_t k,
                                     float inv_tau, int32_t* s_t, float* s_v, float* sh) {
    float m = -INFINITY, z = 0.0f;
    for (int64_t ch0 = 0; ch0 < k; ch0 += kSoftChunk) {
        float acc[kSoftCols];
        soft_row_chunk(r0, n, col, xv, CT, k, ch0, acc, s_t, s_v);
        float lm = -INFINITY;
#pragma unroll
        for (int q = 0; q < kSoftCols; ++q)
            if (ch0 + soft_col(q) < k) lm = fmaxf(lm, acc[q] * inv_tau);
        const float cm = block_max_f32(lm, sh);
        const float nm = fmaxf(m, cm);
        float ls = 0.0f;
#pragma unroll
        for (int q = 0; q < kSoftCols; ++q)
            if (ch0 + soft_col(q) < k) ls += expf(acc[q] * inv_tau - nm);
        const float cs = block_sum_f32(ls, sh);
        z = z * expf(m - nm) + cs;
        m = nm;
    }
    return m + logf(z);
}

__global__ __launch_bounds__(kSoftThreads) void k_soft_fwd(int64_t N, const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col, const float* __restrict__ xv,
                                                           const float* __restrict__ CT, int32_t k, float inv_tau,
                                                           float* __restrict__ lse) {
    __shared__ int32_t s_t[kSoftTermsInLds];
    __shared__ float s_v[kSoftTermsInLds];
    __shared__ float sh[kSoftThreads / 64];
    for (int64_t i = blockIdx.x; i < N; i += gridDim.x) {
        const int64_t r0 = rp[i];
        const int n = (int)(rp[i + 1] - r0);
        const float l = soft_row_lse(r0, n, col, xv, CT, k, inv_tau, s_t, s_v, sh);
        if (threadIdx.x == 0) lse[i] = l;
    }
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
                        float tau, float* lse, double* loss_dev, int n_cu, hipStream_t s) {
    int64_t grid = std::min<int64_t>(N, (int64_t)n_cu * 8);
    if (grid > 0)
        hipLaunchKernelGGL(k_soft_fwd, dim3((unsigned)grid), dim3(kSoftThreads), 0, s, N, rp, col, xv, CT, k, 1.0f / tau,
                           lse);
    hipLaunchKernelGGL(k_soft_loss, dim3(1), dim3(1024), 0, s, lse, N, loss_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------- backward, rows of one chunk
// For rows [c0, c1): recompute S, write dS (row-major, k columns) and dX on the
// row's nonzeros.  dX: 16 terms at a time, each thread forms 16 partial dots
// over its columns, partials go through LDS, 16 lanes per term finish the sum.
__global__ __launch_bounds__(kSoftThreads) void k_soft_bwd_rows(int64_t c0, int64_t c1, const int64_t* __restrict__ rp,
                                                                const int32_t* __restrict__ col,
                                                                const float* __restrict__ xv,
                                                                const float* __restrict__ CT, int32_t k, float inv_tau,
                                                                float neg_g_over_tau, const float* __restrict__ lse,
                                                                float* __restrict__ dS, float* __restrict__ dxv) {
    __shared__ int32_t s_t[kSoftTermsInLds];
    __shared__ float s_v[kSoftTermsInLds];
    __shared__ float part[16][kSoftThreads + 1];
    const int lane = threadIdx.x & 63;
    for (int64_t i = c0 + blockIdx.x; i < c1; i += gridDim.x) {
        const int64_t r0 = rp[i];
        const int n = (int)(rp[i + 1] - r0);
        const float l = lse[i];
        float* dsrow = dS + (i - c0) * (int64_t)k;
        for (int64_t ch0 = 0; ch0 < k; ch0 += kSoftChunk) {
            float acc[kSoftCols];
            soft_row_chunk(r0, n, col, xv, CT, k, ch0, acc, s_t, s_v);
            float ds[kSoftCols];
#pragma unroll
            for (int q = 0; q < kSoftCols; ++q) {
                const int64_t c = ch0 + soft_col(q);
                ds[q] = c < k ? neg_g_over_tau * expf(acc[q] * inv_tau - l) : 0.0f;
                if (c < k) dsrow[c] = ds[q];
            }
            // dX contribution of this column chunk
            const bool full = ch0 + kSoftChunk <= k && (k & 3) == 0;  // float4 gathers stay 16-byte aligned
            for (int h0 = 0; h0 < n; h0 += 16) {
                const int m = min(16, n - h0);
                float pd[16];
                if (full) {
                    // four terms' rows in flight, then their dots in column order
#pragma unroll
                    for (int e0 = 0; e0 < 16; e0 += 4) {
                        float4 g[4][4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int e = e0 + u;
                            const float* row = CT + (int64_t)col[r0 + h0 + (e < m ? e : 0)] * k + ch0;
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                g[u][q] = *reinterpret_cast<const float4*>(row + q * (kSoftThreads * 4) + threadIdx.x * 4);
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            float a = 0.0f;
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                a = fmaf(ds[4 * q + 0], g[u][q].x, a);
                                a = fmaf(ds[4 * q + 1], g[u][q].y, a);
                                a = fmaf(ds[4 * q + 2], g[u][q].z, a);
                                a = fmaf(ds[4 * q + 3], g[u][q].w, a);
                            }
                            pd[e0 + u] = e0 + u < m ? a : 0.0f;
                        }
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        pd[e] = 0.0f;
                        if (e < m) {
                            const float* row = CT + (int64_t)col[r0 + h0 + e] * k + ch0;
#pragma unroll
                            for (int q = 0; q < kSoftCols; ++q)
                                if (ch0 + soft_col(q) < k) pd[e] = fmaf(ds[q], row[soft_col(q)], pd[e]);
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < 16; ++e) part[e][threadIdx.x] = pd[e];
                __syncthreads();
                // thread -> (term e = tid / 16, slice r = tid % 16) sums 16 partials, then 16 lanes reduce
                const int e = threadIdx.x >> 4, r = threadIdx.x & 15;
                float s2 = 0.0f;
#pragma unroll
                for (int q = 0; q < 16; ++q) s2 += part[e][r * 16 + q];
#pragma unroll
                for (int o = 8; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
                if (r == 0 && e < m) {
                    const int64_t p = r0 + h0 + e;
                    dxv[p] = (ch0 == 0 ? 0.0f : dxv[p]) + s2;
                }
                (void)lane;
            }
        }
    }
}

hipError_t soft_bwd_rows(int64_t c0, int64_t c1, const int64_t* rp, const int32_t* col, const float* xv,
                         const float* CT, int32_t k, float tau, float grad, const float* lse, float* dS, float* dxv,
                         int n_cu, hipStream_t s) {
    int64_t grid = std::min<int64_t>(c1 - c0, (int64_t)n_cu * 8);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_soft_bwd_rows, dim3((unsigned)grid), dim3(kSoftThreads), 0, s, c0, c1, rp, col, xv, CT, k,
                       1.0f / tau, -grad / tau, lse, dS, dxv);
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
// dCT[t][:] (+)= sum over rows i in [c0, c1) containing t, ascending, of v_it * dS[i - c0][:]
__global__ __launch_bounds__(kSoftThreads) void k_soft_dct(int64_t d, int32_t k, int64_t c0, int64_t c1, int first,
                                                           const int64_t* __restrict__ colptr,
                                                           const int32_t* __restrict__ xt_row,
                                                           const float* __restrict__ xt_val,
                                                           const float* __restrict__ dS, float* __restrict__ dCT) {
    for (int64_t t = blockIdx.x; t < d; t += gridDim.x) {
        const int64_t b = colptr[t], e = colptr[t + 1];
        // rows of this chunk: [lo, hi) inside the ascending list
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
        if (lo == hi && !first) continue;
        for (int64_t ch0 = 0; ch0 < k; ch0 += kSoftChunk) {
            float acc[kSoftCols];
            float* out = dCT + t * (int64_t)k + ch0;
#pragma unroll
            for (int q = 0; q < kSoftCols; ++q) {
                const int64_t c = ch0 + soft_col(q);
                acc[q] = (first || c >= k) ? 0.0f : out[soft_col(q)];
            }
            const bool full = ch0 + kSoftChunk <= k && (k & 3) == 0;  // float4 gathers stay 16-byte aligned
            if (full) {
                // kDctRows rows per step: their ids, then all their gathers, are
                // issued before the first multiply-add, which still runs in
                // ascending row order
                for (int64_t p0 = lo; p0 < hi; p0 += kDctRows) {
                    const int m = (int)min((int64_t)kDctRows, hi - p0);
                    int64_t ro[kDctRows];
                    float vv[kDctRows];
#pragma unroll
                    for (int u = 0; u < kDctRows; ++u) {
                        const bool in = u < m;
                        ro[u] = (int64_t)(xt_row[in ? p0 + u : p0] - c0) * k + ch0;
                        vv[u] = in ? xt_val[p0 + u] : 0.0f;
                    }
                    float4 g[kDctRows][4];
#pragma unroll
                    for (int u = 0; u < kDctRows; ++u)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            g[u][q] = *reinterpret_cast<const float4*>(dS + ro[u] + q * (kSoftThreads * 4) +
                                                                      threadIdx.x * 4);
#pragma unroll
                    for (int u = 0; u < kDctRows; ++u) {
                        if (u < m) {
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                acc[4 * q + 0] = fmaf(vv[u], g[u][q].x, acc[4 * q + 0]);
                                acc[4 * q + 1] = fmaf(vv[u], g[u][q].y, acc[4 * q + 1]);
                                acc[4 * q + 2] = fmaf(vv[u], g[u][q].z, acc[4 * q + 2]);
                                acc[4 * q + 3] = fmaf(vv[u], g[u][q].w, acc[4 * q + 3]);
                            }
                        }
                    }
                }
            } else {
                for (int64_t p = lo; p < hi; ++p) {
                    const float v = xt_val[p];
                    const float* row = dS + (int64_t)(xt_row[p] - c0) * k + ch0;
#pragma unroll
                    for (int q = 0; q < kSoftCols; ++q)
                        if (ch0 + soft_col(q) < k) acc[q] = fmaf(v, row[soft_col(q)], acc[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < kSoftCols; ++q)
                if (ch0 + soft_col(q) < k) out[soft_col(q)] = acc[q];
        }
    }
}

hipError_t soft_dct(int64_t d, int32_t k, int64_t c0, int64_t c1, int first, const int64_t* colptr,
                    const int32_t* xt_row, const float* xt_val, const float* dS, float* dCT, int n_cu, hipStream_t s) {
    int64_t grid = std::min<int64_t>(d, (int64_t)n_cu * 16);
    hipLaunchKernelGGL(k_soft_dct, dim3((unsigned)grid), dim3(kSoftThreads), 0, s, d, k, c0, c1, first, colptr, xt_row,
                       xt_val, dS, dCT);
    return hipGetLastError();
}

}  // namespace sivf
