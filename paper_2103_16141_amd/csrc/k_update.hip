// Update step (Alg. 1 update; Alg. 5 mean computation) on CDNA.
//
// 1. Stable sort of object ids by cluster: per 4096-object block, cluster
//    histograms (atomics on integers: order-independent), a column scan over
//    blocks, and an in-block bitonic sort of (cluster, local id) keys that
//    gives each object its rank among same-cluster objects of its block.  The
//    result lists every cluster's members in ascending object id.
// 2. One wave per cluster (persistent waves, each with private dense FP64
//    sums: term ids below kHotTerms in LDS, the rest in a row W of length d
//    in HBM): w_t = sum of member values in ascending object id (sequential
//    per term, exactly the reference fold), then in ascending term order
//    q_t = w_t / |C_j|, s = s + q_t*q_t (sequential), support
//    = {t : q_t != 0}; u_t = q_t / sqrt(s).  The sums are cleared as they are
//    read, so they are zero again for the next cluster.  The member chain is
//    the cost: each member ends with a wait for its stores, so every load is
//    issued unconditionally and ahead of its use (see member_sums).
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

// Sums of term ids below kHotTerms live in LDS (16 KB per wave), the rest in
// the wave's HBM row: with term ids in decreasing frequency, as in the
// Zipf-shaped corpora, most member nonzeros then update LDS, and the HBM row
// takes only the rest.  (Any other term order gives the same sums.)
constexpr int kHotTerms = 2048;

// Ascending-term pass over a cluster's dense FP64 sums w: q_t = w_t / |C_j|,
// s = s + q_t*q_t sequentially in ascending t, support {t : q_t != 0}
// compacted into next[o ..), then u_t = q_t / sqrt(s).  The sums of four
// 64-term chunks are loaded together; terms below kHotTerms are read from
// the wave's LDS sums, the rest from its HBM row; both are zeroed as read.
__device__ inline void term_pass(double* __restrict__ row, double* hot, int64_t d, int64_t cnt, int64_t o, int64_t j,
                                 Store& next, int lane) {
    const double dc = (double)cnt;
    double ssq = 0.0;
    int64_t eo = 0;
    for (int64_t p0 = 0; p0 < d; p0 += 256) {
        double wq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t p = p0 + u * 64 + lane;
            const double hv = hot[p < kHotTerms ? p : 0];
            const double rv = row[p < d ? p : d - 1];
            wq[u] = p >= d ? 0.0 : p < kHotTerms ? hv : rv;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t p = p0 + u * 64 + lane;
            const double wv = wq[u];
            const double qv = wv / dc;
            const bool nz = qv != 0.0;
            if (wv != 0.0) {
                if (p < kHotTerms) hot[p] = 0.0;
                else row[p] = 0.0;
            }
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
    }
    const double nr = sqrt(ssq);
    for (int64_t p = lane; p < eo; p += 64) next.val[o + p] = next.val[o + p] / nr;
    if (lane == 0) {
        next.start[j] = o;
        next.nnz[j] = eo;
    }
    __threadfence_block();
}

// Row chunks of 64 nonzeros a wave holds in registers per member (rows of up
// to 256 nonzeros; the rest of a longer row is read chunk by chunk).
constexpr int kRowPre = 4;

typedef __attribute__((address_space(1))) double gdouble;   // global memory

template <bool F64>
__device__ inline double xval(const void* x, int64_t p) {
    return F64 ? ((const double*)x)[p] : (double)((const float*)x)[p];
}

// Member sums of cluster j (members q0 .. q1-1 of perm), ascending object id:
// w_t = w_t + v for every nonzero (t, v) of each member row in turn.
//
// The sums are a chain: member q's additions must be visible before member
// q+1's (the same term sits in different lanes of different rows), so each
// member ends with a wait for its stores.  To keep that wait the only one,
// every load is unconditional (clamped indices, masked results; a load
// behind a condition makes the compiler wait for all outstanding loads) and
// runs ahead of its use: the member id three members ahead, the row bounds
// two ahead, the nonzeros one ahead, while member q's accumulators are read
// (all loads before any store: a row's terms are distinct) and written.
template <bool F64>
__device__ inline void member_sums(const Csr& X, int64_t q0, int64_t q1, double* __restrict__ W, double* hot,
                                   const UpdateWs& w, int lane) {
    const int64_t qlast = q1 - 1;
    const int64_t plast = X.nnz - 1;   // >= 0: the caller skips a matrix without nonzeros
    auto perm_at = [&](int64_t q) -> int64_t { return (int64_t)w.perm[q < qlast ? q : qlast]; };
    // stage state: member id of q+2 (bounds next), bounds of q+1 (row next), row of q
    int64_t i2 = perm_at(q0 + 2);
    int64_t b1, e1, b0, e0;
    {
        const int64_t i0 = perm_at(q0), i1 = perm_at(q0 + 1);
        b0 = X.rp[i0];
        e0 = X.rp[i0 + 1];
        b1 = X.rp[i1];
        e1 = X.rp[i1 + 1];
    }
    int32_t tc[kRowPre];
    double vc[kRowPre];
#pragma unroll
    for (int c = 0; c < kRowPre; ++c) {
        const int64_t p = b0 + c * 64 + lane;
        const int64_t pc = p < plast ? p : plast;
        const int32_t t = X.col[pc];
        const double v = xval<F64>(X.val, pc);
        tc[c] = p < e0 ? t : -1;
        vc[c] = v;
    }
    gdouble* Wg = (gdouble*)W;
    for (int64_t q = q0; q < q1; ++q) {
        const bool has1 = q + 1 < q1;
        // member q's accumulators first (the in-order load counter then lets
        // the loads below stay in flight while these are awaited)
        double gv[kRowPre], lv[kRowPre];
#pragma unroll
        for (int c = 0; c < kRowPre; ++c) {
            gv[c] = Wg[tc[c] >= kHotTerms ? tc[c] : 0];
            lv[c] = hot[tc[c] >= 0 && tc[c] < kHotTerms ? tc[c] : 0];
        }
        // member id of q+3, bounds of q+2, nonzeros of q+1
        const int64_t i3 = perm_at(q + 3);
        const int64_t b2 = X.rp[i2], e2 = X.rp[i2 + 1];
        int32_t tn[kRowPre];
        double vn[kRowPre];
#pragma unroll
        for (int c = 0; c < kRowPre; ++c) {
            const int64_t p = b1 + c * 64 + lane;
            const int64_t pc = p < plast ? p : plast;
            const int32_t t = X.col[pc];
            const double v = xval<F64>(X.val, pc);
            tn[c] = has1 && p < e1 ? t : -1;
            vn[c] = v;
        }
        // member q: every accumulator was read before any write (a row's
        // terms are distinct)
#pragma unroll
        for (int c = 0; c < kRowPre; ++c) {
            if (tc[c] >= kHotTerms) Wg[tc[c]] = gv[c] + vc[c];
            else if (tc[c] >= 0) hot[tc[c]] = lv[c] + vc[c];
        }
        for (int64_t p = b0 + kRowPre * 64 + lane; p < e0; p += 64) {   // rows beyond 256 nonzeros
            const int32_t t = X.col[p];
            const double v = xval<F64>(X.val, p);
            if (t >= kHotTerms) Wg[t] = Wg[t] + v;
            else hot[t] = hot[t] + v;
        }
        // this member's sums must be visible to every lane before the next member
        __threadfence_block();
#pragma unroll
        for (int c = 0; c < kRowPre; ++c) {
            tc[c] = tn[c];
            vc[c] = vn[c];
        }
        b0 = b1;
        e0 = e1;
        b1 = b2;
        e1 = e2;
        i2 = i3;
    }
}

// Cluster j's mean direction into next[o .. o + support): member sums, then
// the ascending-term pass.
__device__ inline void sum_normalize(const Csr& X, int64_t j, int64_t cnt, int64_t o, double* __restrict__ W,
                                     double* hot, Store& next, const UpdateWs& w, int lane) {
    const int64_t q0 = w.cstart[j], q1 = q0 + cnt;
    if (X.nnz > 0) {
        if (X.f64) member_sums<true>(X, q0, q1, W, hot, w, lane);
        else member_sums<false>(X, q0, q1, W, hot, w, lane);
    }
    term_pass(W, hot, X.d, cnt, o, j, next, lane);
}

__global__ __launch_bounds__(256) void k_upd_segsum(Csr X, int32_t k, const uint8_t* __restrict__ lam, int allow_copy,
                                                    Store prev, Store next, UpdateWs w) {
    __shared__ double hot_all[4][kHotTerms];   // 64 KB: the four waves' LDS sums
    const int lane = threadIdx.x & 63;
    const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    if (gw >= w.nslots) return;
    double* __restrict__ W = w.W + gw * X.d;
    double* hot = hot_all[threadIdx.x >> 6];
    for (int i = lane; i < kHotTerms; i += 64) hot[i] = 0.0;   // kept zero by the term pass
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
            sum_normalize(X, j, cnt, o, W, hot, next, w, lane);
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
