// Update step (Alg. 1 update; Alg. 5 mean computation) on CDNA.
//
// 1. Stable sort of object ids by cluster: per 4096-object block, cluster
//    histograms (atomics on integers: order-independent), a column scan over
//    blocks, and an in-block bitonic sort of (cluster, local id) keys that
//    gives each object its rank among same-cluster objects of its block.  The
//    result lists every cluster's members in ascending object id.
// 2. One wave per cluster (persistent waves, each with a private dense FP64
//    row W of length d in HBM): w_t = sum of member values in ascending
//    object id (sequential per term, exactly the reference fold), then in
//    ascending term order q_t = w_t / |C_j|, s = s + q_t*q_t (sequential),
//    support = {t : q_t != 0}; u_t = q_t / sqrt(s).  W is cleared as it is
//    read, so it is zero again for the next cluster.
//    Clusters with no members, or with unchanged members (flag 1), keep their
//    previous centroid bitwise (it would be recomputed to the same bits).
#include "internal.h"
#include "wave.h"

#pragma clang fp contract(off)

namespace sivf {

__global__ __launch_bounds__(256) void k_upd_hist(const int32_t* __restrict__ a, int64_t n, int32_t k,
                                                  const int64_t* __restrict__ rp, int64_t* __restrict__ hist,
                                                  int64_t* __restrict__ memnnz) {
    const int64_t b = blockIdx.x;
    const int64_t lo = b * kObjBlock, hi = min(n, lo + kObjBlock);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const int32_t j = a[i];
        atomicAdd((unsigned long long*)&hist[b * k + j], 1ull);
        atomicAdd((unsigned long long*)&memnnz[j], (unsigned long long)(rp[i + 1] - rp[i]));
    }
}

__global__ void k_upd_colscan(int32_t k, int64_t nblk, int64_t* __restrict__ hist, int64_t* __restrict__ ccount) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= k) return;
    int64_t run = 0;
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t h = hist[b * k + j];
        hist[b * k + j] = run;
        run += h;
    }
    ccount[j] = run;
}

// In-block stable ranks by bitonic sort of unique keys (cluster << 12 | local).
__global__ __launch_bounds__(256) void k_upd_scatter(const int32_t* __restrict__ a, int64_t n, int32_t k,
                                                     const int64_t* __restrict__ hist,
                                                     const int64_t* __restrict__ cstart, int32_t* __restrict__ perm) {
    __shared__ unsigned long long key[kObjBlock];
    const int64_t b = blockIdx.x;
    const int64_t lo = b * kObjBlock;
    for (int l = threadIdx.x; l < kObjBlock; l += blockDim.x) {
        const int64_t i = lo + l;
        key[l] = i < n ? (((unsigned long long)(uint32_t)a[i]) << 12) | (unsigned long long)l : ~0ull;
    }
    __syncthreads();
    for (int size = 2; size <= kObjBlock; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int l = threadIdx.x; l < kObjBlock / 2; l += blockDim.x) {
                const int x = 2 * l - (l & (stride - 1));  // lower index of the pair
                const int y = x + stride;
                const bool up = (x & size) == 0;
                const unsigned long long kx = key[x], ky = key[y];
                if ((kx > ky) == up) {
                    key[x] = ky;
                    key[y] = kx;
                }
            }
            __syncthreads();
        }
    }
    for (int s = threadIdx.x; s < kObjBlock; s += blockDim.x) {
        const unsigned long long kv = key[s];
        if (kv == ~0ull) continue;
        const int32_t j = (int32_t)(kv >> 12);
        const int loc = (int)(kv & 4095ull);
        // first sorted position of cluster j in this block
        int l0 = 0, len = s;
        const unsigned long long target = ((unsigned long long)(uint32_t)j) << 12;
        while (len > 0) {
            const int half = len >> 1;
            if (key[l0 + half] < target) {
                l0 += half + 1;
                len -= half + 1;
            } else {
                len = half;
            }
        }
        const int64_t pos = cstart[j] + hist[b * k + j] + (s - l0);
        perm[pos] = (int32_t)(lo + loc);
    }
}

hipError_t upd_sort(const int32_t* a, int64_t n, int32_t k, const int64_t* rp, UpdateWs w, hipStream_t s) {
    hipError_t e = fill_i64(w.hist, 0, w.nblk * (int64_t)k, s);
    if (e != hipSuccess) return e;
    e = fill_i64(w.memnnz, 0, k, s);
    if (e != hipSuccess) return e;
    if (n > 0) hipLaunchKernelGGL(k_upd_hist, dim3((unsigned)w.nblk), dim3(256), 0, s, a, n, k, rp, w.hist, w.memnnz);
    hipLaunchKernelGGL(k_upd_colscan, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, k, w.nblk, w.hist,
                       w.ccount);
    e = exclusive_scan_i64(w.ccount, w.cstart, k, w.scan_ws, s);
    if (e != hipSuccess) return e;
    if (n > 0) hipLaunchKernelGGL(k_upd_scatter, dim3((unsigned)w.nblk), dim3(256), 0, s, a, n, k, w.hist, w.cstart,
                                  w.perm);
    return hipGetLastError();
}

__global__ void k_upd_bounds(int32_t k, int64_t d, const uint8_t* __restrict__ lam, int allow_copy, Store prev,
                             const int64_t* __restrict__ ccount, const int64_t* __restrict__ memnnz,
                             int64_t* __restrict__ ub) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= k) return;
    const bool copy = ccount[j] == 0 || (allow_copy && lam[j]);
    ub[j] = copy ? prev.nnz[j] : min(d, memnnz[j]);
}

hipError_t upd_bounds(int32_t k, int64_t d, const uint8_t* lam, int allow_copy, const Store prev, UpdateWs w,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_upd_bounds, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, k, d, lam, allow_copy, prev,
                       w.ccount, w.memnnz, w.ub);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return exclusive_scan_i64(w.ub, w.ubscan, k, w.scan_ws, s);
}

__device__ inline double xv64(const void* x, int f64, int64_t p) {
    return f64 ? ((const double*)x)[p] : (double)((const float*)x)[p];
}

// Cluster j's mean direction into next[o .. o + support): sums in ascending
// object id, then the ascending-term pass.
__device__ __noinline__ void sum_normalize(const Csr& X, int64_t j, int64_t cnt, int64_t o, double* __restrict__ W,
                                           Store& next, const UpdateWs& w, int lane) {
    const int64_t d = X.d;
    {  // ---- member sums, ascending object id, one member at a time
        const int64_t q0 = w.cstart[j], q1 = q0 + cnt;
        int64_t i_nx = w.perm[q0];
        int64_t b_nx = X.rp[i_nx], e_nx = X.rp[i_nx + 1];
        for (int64_t q = q0; q < q1; ++q) {
            const int64_t b = b_nx, e = e_nx;
            if (q + 1 < q1) {  // next member's row bounds, independent of W
                i_nx = w.perm[q + 1];
                b_nx = X.rp[i_nx];
                e_nx = X.rp[i_nx + 1];
            }
            for (int64_t p = b + lane; p < e; p += 64) {
                const int32_t t = X.col[p];
                const double v = xv64(X.val, X.f64, p);
                W[t] = W[t] + v;
            }
            // this member's sums must be visible to every lane before the next member
            __threadfence_block();
        }
        // ---- ascending-term pass: divide, fold squares, compact, clear W
        const double dc = (double)cnt;
        double ssq = 0.0;
        int64_t eo = 0;
        for (int64_t p0 = 0; p0 < d; p0 += 64) {
            const int64_t p = p0 + lane;
            double wv = 0.0;
            if (p < d) wv = W[p];
            const double qv = wv / dc;
            const bool nz = qv != 0.0;
            if (wv != 0.0) W[p] = 0.0;
            unsigned long long m = ballot(nz);
            if (!m) continue;
            const double sq = qv * qv;
            const int pos = lanes_below(m);
            if (nz) {
                next.term[o + eo + pos] = (int32_t)p;
                next.val[o + eo + pos] = qv;
            }
            eo += __popcll(m);
            while (m) {
                const int l = __ffsll((long long)m) - 1;
                ssq = ssq + bcast_f64(sq, l);
                m &= m - 1;
            }
        }
        const double nr = sqrt(ssq);
        for (int64_t p = lane; p < eo; p += 64) next.val[o + p] = next.val[o + p] / nr;
        if (lane == 0) {
            next.start[j] = o;
            next.nnz[j] = eo;
        }
        __threadfence_block();
    }
}

__global__ __launch_bounds__(256) void k_upd_segsum(Csr X, int32_t k, const uint8_t* __restrict__ lam, int allow_copy,
                                                    Store prev, Store next, UpdateWs w) {
    const int lane = threadIdx.x & 63;
    const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    if (gw >= w.nslots) return;
    double* __restrict__ W = w.W + gw * X.d;
    for (int64_t j = wave_grab(w.work, 1ull); j < k; j = wave_grab(w.work, 1ull)) {
        const int64_t cnt = w.ccount[j];
        const int64_t o = w.ubscan[j];
        if (cnt == 0 || (allow_copy && lam[j])) {
            const int64_t ps = prev.start[j], m = prev.nnz[j];
            for (int64_t p = lane; p < m; p += 64) {
                next.term[o + p] = prev.term[ps + p];
                next.val[o + p] = prev.val[ps + p];
            }
            if (lane == 0) {
                next.start[j] = o;
                next.nnz[j] = m;
            }
        } else {
            sum_normalize(X, j, cnt, o, W, next, w, lane);
        }
    }
}

hipError_t upd_segsum(const Csr& X, int32_t k, const uint8_t* lam, int allow_copy, const Store prev, Store next,
                      UpdateWs w, hipStream_t s) {
    hipError_t e = fill_u64(w.work, 0ull, 1, s);
    if (e != hipSuccess) return e;
    const int blocks = (w.nslots + 3) / 4;
    hipLaunchKernelGGL(k_upd_segsum, dim3(blocks), dim3(256), 0, s, X, k, lam, allow_copy, prev, next, w);
    return hipGetLastError();
}

}  // namespace sivf
