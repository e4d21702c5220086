// Assignment step (Alg. 4) on CDNA: a wave takes one object, loads its CSR
// row, and for each centroid tile walks the posting lists of the object's
// terms, gather-accumulating v * u into a per-wave similarity tile in LDS.
// Centroid ids are unique inside a list, so the 64 lanes of one instruction
// never collide: the tile is updated with plain LDS read-add-write (a wave's
// LDS operations complete in order), and the accumulation order is fixed:
// term-major, ascending term.  (LDS float atomics are ~25x slower on gfx950.)  An object whose own cluster was invariant (ICP branch)
// stops each list at the moving/invariant boundary of the structured file.
//
// Exactness: the FP32 pass gives rho_hat with |rho_hat - rho_fp64| <= B per
// centroid (rounding of posting values, of object values, of the FP32 fold
// and of the FP64 reference fold; see bound_setup).  The walk keeps the
// largest lower bound theta = max_j (rho_hat_j - B_j) and every centroid whose
// upper bound reaches theta.  One survivor => the argmax is certified.  More
// => the object is re-scored in FP64 over the survivors only (rescore_cand),
// in the reference order; too many => over all eligible centroids through the
// FP64 posting values (rescore_full).
#include "internal.h"
#include "wave.h"

#pragma clang fp contract(off)

namespace sivf {

struct Bound {
    double crel;   // relative coefficient (nonnegative data)
    double cabs;   // eta * ||x|| (signed data; multiplied by cnorm_j)
    double absl;   // flush-to-zero slack
};

__device__ inline double gamma_n(double n, double u) { return n * u / (1.0 - n * u); }

__device__ inline Bound bound_setup(const WalkArgs& A, int n, double xnorm) {
    const double m = (double)n + 1.0;
    double eta = (1.0 + A.eta_x) * (1.0 + A.eta_val) * (1.0 + gamma_n(m, 0x1p-24)) - 1.0 + gamma_n(m, 0x1p-53);
    eta *= (1.0 + 0x1p-20);
    Bound b;
    b.crel = eta / (1.0 - eta) * (1.0 + 0x1p-40);
    b.cabs = eta * xnorm * (1.0 + 0x1p-40);
    b.absl = (2.0 * n + 4.0) * 0x1p-125;
    return b;
}

__device__ inline double bound_of(const WalkArgs& A, const Bound& b, double r, int32_t j) {
    double B = A.nonneg ? b.crel * fabs(r) : b.cabs * A.cnorm[j];
    return B + 0x1p-50 * fabs(r) + b.absl;
}

__device__ inline float load_xval(const void* x, int f64, int64_t p) {
    return f64 ? (float)((const double*)x)[p] : ((const float*)x)[p];
}

__device__ inline double load_xval64(const void* x, int f64, int64_t p) {
    return f64 ? ((const double*)x)[p] : (double)((const float*)x)[p];
}

// max of (v, -j) lexicographically: largest v, lowest j among equals.
__device__ inline void wave_argmax(double& v, int32_t& j) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_xor(v, o, 64);
        int32_t oj = __shfl_xor(j, o, 64);
        if (ov > v || (ov == v && oj < j)) {
            v = ov;
            j = oj;
        }
    }
}

template <bool BF16>
__device__ inline float posting_val(const void* pv, int64_t p) {
    if (BF16) return bf16_to_f32(((const uint16_t*)pv)[p]);
    return ((const float*)pv)[p];
}

// ---------------------------------------------------------------------------
// fast pass
// ---------------------------------------------------------------------------
template <bool BF16>
__global__ __launch_bounds__(256) void k_walk_fast(WalkArgs A, unsigned long long* __restrict__ work) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    float* sim = lds + wid * A.kt;
    int32_t* cj = (int32_t*)(lds + kWalkWaves * A.kt) + wid * kCandCap;
    float* cr = (float*)((int32_t*)(lds + kWalkWaves * A.kt) + kWalkWaves * kCandCap) + wid * kCandCap;

    for (int jj = lane; jj < A.kt; jj += 64) sim[jj] = 0.0f;

    unsigned long long macc = 0, icp_cnt = 0;
    constexpr int kGrab = 8;
    for (int64_t g0 = wave_grab(work, kGrab); g0 < A.n; g0 = wave_grab(work, kGrab)) {
        const int64_t gend = min(g0 + kGrab, A.n);
        for (int64_t i = g0; i < gend; ++i) {
            const int64_t r0 = A.rp[i];
            const int n = (int)(A.rp[i + 1] - r0);
            int32_t a_old = -1;
            bool icp = false;
            float own_old = 0.0f;
            if (A.icp_on) {
                a_old = A.a_prev[i];
                icp = A.lam[a_old] != 0;
                own_old = A.own_prev[i];
            }
            icp_cnt += icp ? 1 : 0;
            double xnorm = 0.0;
            if (!A.nonneg) {
                double ss = 0.0;
                for (int h = lane; h < n; h += 64) {
                    double v = load_xval64(A.xval, A.x_f64, r0 + h);
                    ss = ss + v * v;
                }
                xnorm = sqrt(wave_sum_f64(ss)) * (1.0 + 0x1p-40);
            }
            const Bound bd = bound_setup(A, n, xnorm);

            double theta = -INFINITY;   // largest lower bound so far
            double best_lo = -INFINITY;
            int32_t best_j = 0x7fffffff;
            int ccount = 0;
            bool overflow = false;
            if (icp) {
                double r = (double)own_old;
                theta = r - bound_of(A, bd, r, a_old);
                best_lo = theta;
                best_j = a_old;
                if (lane == 0) {
                    cj[0] = a_old;
                    cr[0] = own_old;
                }
                ccount = 1;
            }
            const bool front_only = icp && !A.cbicp;
            const bool test_flag = icp && A.cbicp;

            for (int tile = 0; tile < A.T; ++tile) {
                const int32_t base = tile * A.kt;
                const int32_t width = min(A.kt, A.k - base);
                // ---- walk the lists of the object's terms for this tile
                for (int c0 = 0; c0 < n; c0 += 64) {
                    const int h = c0 + lane;
                    int64_t s0 = 0, s1 = 0;
                    int32_t mv = 0;
                    float v = 0.0f;
                    if (h < n) {
                        const int64_t t = A.col[r0 + h];
                        v = load_xval(A.xval, A.x_f64, r0 + h);
                        const int64_t sidx = t * A.T + tile;
                        s0 = A.seg[sidx];
                        s1 = A.seg[sidx + 1];
                        mv = A.mid[sidx];
                    }
                    const int64_t e = front_only ? s0 + mv : s1;
                    const int cnt = min(64, n - c0);
                    for (int q = 0; q < cnt; ++q) {
                        const int64_t ps = bcast_i64(s0, q);
                        const int64_t pe = bcast_i64(e, q);
                        const float vq = bcast_f32(v, q);
                        macc += test_flag ? (unsigned long long)bcast_i32(mv, q) : (unsigned long long)(pe - ps);
                        int64_t p = ps + lane;
                        // four postings per lane in flight
                        for (; p + 192 < pe; p += 256) {
                            const uint16_t c_a = A.cid[p], c_b = A.cid[p + 64], c_c = A.cid[p + 128],
                                           c_d = A.cid[p + 192];
                            const float u_a = posting_val<BF16>(A.pval, p), u_b = posting_val<BF16>(A.pval, p + 64),
                                        u_c = posting_val<BF16>(A.pval, p + 128),
                                        u_d = posting_val<BF16>(A.pval, p + 192);
                            // the four postings belong to one list, so their ids are
                            // distinct: read all four, then write all four
                            float pa = vq * u_a, pb = vq * u_b, pc = vq * u_c, pd = vq * u_d;
                            if (test_flag) {
                                if (A.lam[base + c_a]) pa = 0.0f;
                                if (A.lam[base + c_b]) pb = 0.0f;
                                if (A.lam[base + c_c]) pc = 0.0f;
                                if (A.lam[base + c_d]) pd = 0.0f;
                            }
                            const float oa = sim[c_a], ob = sim[c_b], oc = sim[c_c], od = sim[c_d];
                            sim[c_a] = oa + pa;
                            sim[c_b] = ob + pb;
                            sim[c_c] = oc + pc;
                            sim[c_d] = od + pd;
                        }
                        for (; p < pe; p += 64) {
                            const uint16_t c = A.cid[p];
                            const float u = posting_val<BF16>(A.pval, p);
                            if (!test_flag || !A.lam[base + c]) sim[c] = sim[c] + vq * u;
                        }
                    }
                }
                // ---- tile epilogue: bounds, running theta, candidates; clears the tile
                double tmax = -INFINITY;
                int32_t tj = 0x7fffffff;
                for (int jj = lane; jj < width; jj += 64) {
                    const int32_t j = base + jj;
                    const bool elig = !icp || A.lam[j] == 0;
                    if (elig) {
                        const double r = (double)sim[jj];
                        const double lo = r - bound_of(A, bd, r, j);
                        if (lo > tmax) {
                            tmax = lo;
                            tj = j;
                        }
                    }
                }
                wave_argmax(tmax, tj);
                if (tmax > best_lo || (tmax == best_lo && tj < best_j)) {
                    best_lo = tmax;
                    best_j = tj;
                }
                if (tmax > theta) {
                    theta = tmax;
                    // drop earlier candidates that can no longer win
                    bool keep = false;
                    int32_t kj = 0;
                    float kr = 0.0f;
                    if (lane < ccount && lane < kCandCap) {
                        kj = cj[lane];
                        kr = cr[lane];
                        const double r = (double)kr;
                        keep = r + bound_of(A, bd, r, kj) >= theta;
                    }
                    const unsigned long long km = ballot(keep);
                    if (!overflow) {
                        const int pos = lanes_below(km);
                        if (keep) {
                            cj[pos] = kj;
                            cr[pos] = kr;
                        }
                        ccount = __popcll(km);
                    }
                }
                for (int jj0 = 0; jj0 < width; jj0 += 64) {
                    const int jj = jj0 + lane;
                    bool take = false;
                    float r32 = 0.0f;
                    if (jj < width) {
                        const int32_t j = base + jj;
                        r32 = sim[jj];
                        sim[jj] = 0.0f;
                        if (!icp || A.lam[j] == 0) {
                            const double r = (double)r32;
                            take = r + bound_of(A, bd, r, j) >= theta;
                        }
                    }
                    const unsigned long long tm = ballot(take);
                    if (tm && !overflow) {
                        const int pos = ccount + lanes_below(tm);
                        if (take && pos < kCandCap) {
                            cj[pos] = base + jj;
                            cr[pos] = r32;
                        }
                        ccount += __popcll(tm);
                        if (ccount > kCandCap) overflow = true;
                    }
                }
            }
            // ---- decision
            if (!A.certify) {
                if (lane == 0) {
                    A.a_new[i] = best_j;
                    float rb = 0.0f;
                    for (int l = 0; l < min(ccount, kCandCap); ++l)
                        if (cj[l] == best_j) rb = cr[l];
                    A.own_new[i] = rb;
                }
            } else if (!overflow && ccount == 1) {
                if (lane == 0) {
                    A.a_new[i] = cj[0];
                    A.own_new[i] = cr[0];
                }
            } else {
                bool full = overflow;
                int64_t slot = 0;
                if (!full) {
                    if (lane == 0) slot = (int64_t)atomicAdd(&A.counters[1], 1ull);
                    slot = bcast_i64(slot, 0);
                    if (slot >= A.qcap) full = true;
                }
                if (full) {
                    if (lane == 0) {
                        unsigned long long f = atomicAdd(&A.counters[2], 1ull);
                        A.fobj[f] = (int32_t)i;
                    }
                } else {
                    if (lane < ccount) A.qcand[slot * kCandCap + lane] = cj[lane];
                    if (lane == 0) {
                        A.qobj[slot] = (int32_t)i;
                        A.qcnt[slot] = ccount;
                    }
                }
            }
        }
    }
    if (lane == 0) {
        atomicAdd(&A.counters[0], macc);
        atomicAdd(&A.counters[3], icp_cnt);
    }
}

hipError_t walk_fast(const WalkArgs& a, int pdt_bf16, int grid_waves, hipStream_t s) {
    // the work counter lives right after the 8 counters
    unsigned long long* work = a.counters + 8;
    const size_t lds = (size_t)kWalkWaves * a.kt * sizeof(float) + (size_t)kWalkWaves * kCandCap * 8;
    int blocks = (grid_waves + kWalkWaves - 1) / kWalkWaves;
    if (blocks < 1) blocks = 1;
    if (lds > 65536) {
        hipError_t e = pdt_bf16 ? hipFuncSetAttribute((const void*)k_walk_fast<true>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                                : hipFuncSetAttribute((const void*)k_walk_fast<false>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (pdt_bf16)
        hipLaunchKernelGGL(k_walk_fast<true>, dim3(blocks), dim3(64 * kWalkWaves), lds, s, a, work);
    else
        hipLaunchKernelGGL(k_walk_fast<false>, dim3(blocks), dim3(64 * kWalkWaves), lds, s, a, work);
    return hipGetLastError();
}

int walk_blocks_per_cu(int kt, int pdt_bf16) {
    const size_t lds = (size_t)kWalkWaves * kt * sizeof(float) + (size_t)kWalkWaves * kCandCap * 8;
    int nb = 0;
    hipError_t e = pdt_bf16
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk_fast<true>, 64 * kWalkWaves, lds)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk_fast<false>, 64 * kWalkWaves, lds);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

// ---------------------------------------------------------------------------
// FP64 re-score in the reference order
// ---------------------------------------------------------------------------
// rho_ij for one (object, centroid): lanes take the object's terms 64 at a
// time, look each up in the centroid's sorted term list (binary search), and
// the wave then folds the products sequentially in ascending term order.
__device__ double exact_rho(const WalkArgs& A, const Store& st, int64_t r0, int n, int32_t j) {
    const int lane = threadIdx.x & 63;
    const int64_t cs = st.start[j];
    const int64_t cm = st.nnz[j];
    double acc = 0.0;
    for (int c0 = 0; c0 < n; c0 += 64) {
        const int h = c0 + lane;
        bool present = false;
        double prod = 0.0;
        if (h < n) {
            const int32_t t = A.col[r0 + h];
            int64_t lo = 0, len = cm;
            while (len > 0) {
                const int64_t half = len >> 1;
                if (st.term[cs + lo + half] < t) {
                    lo += half + 1;
                    len -= half + 1;
                } else {
                    len = half;
                }
            }
            if (lo < cm && st.term[cs + lo] == t) {
                present = true;
                prod = load_xval64(A.xval, A.x_f64, r0 + h) * st.val[cs + lo];
            }
        }
        unsigned long long m = ballot(present);
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            acc = acc + bcast_f64(prod, l);
            m &= m - 1;
        }
    }
    return acc;
}

__global__ __launch_bounds__(256) void k_rescore_cand(WalkArgs A, Store st) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int64_t nq = (int64_t)A.counters[1];
    if (nq > A.qcap) nq = A.qcap;
    unsigned long long cands = 0;
    for (int64_t slot = wave; slot < nq; slot += nw) {
        const int32_t i = A.qobj[slot];
        const int nc = A.qcnt[slot];
        const int64_t r0 = A.rp[i];
        const int n = (int)(A.rp[i + 1] - r0);
        double best = -INFINITY;
        int32_t bj = 0x7fffffff;
        for (int c = 0; c < nc; ++c) {
            const int32_t j = A.qcand[slot * kCandCap + c];
            const double r = exact_rho(A, st, r0, n, j);
            if (r > best || (r == best && j < bj)) {
                best = r;
                bj = j;
            }
        }
        cands += nc;
        if (lane == 0) {
            A.a_new[i] = bj;
            A.own_new[i] = (float)best;
        }
    }
    if (lane == 0 && cands) atomicAdd(&A.counters[4], cands);
}

hipError_t rescore_candidates(const WalkArgs& a, const Store st, int64_t grid_waves, hipStream_t s) {
    int64_t blocks = (grid_waves + 3) / 4;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_rescore_cand, dim3((unsigned)blocks), dim3(256), 0, s, a, st);
    return hipGetLastError();
}

// Objects whose candidate list overflowed: FP64 walk of the structured file
// (same traversal as the fast pass, FP64 accumulator tile in LDS, plain
// read-modify-write since the lanes of one instruction hold distinct ids),
// exact argmax over every eligible centroid.  In the ICP branch the own
// (invariant) centroid's similarity comes from exact_rho.
__global__ __launch_bounds__(64) void k_rescore_full(WalkArgs A, const double* __restrict__ v64, Store st) {
    extern __shared__ double acc[];
    const int lane = threadIdx.x & 63;
    const int64_t nf = (int64_t)A.counters[2];
    for (int jj = lane; jj < A.kt; jj += 64) acc[jj] = 0.0;
    for (int64_t slot = blockIdx.x; slot < nf; slot += gridDim.x) {
        const int32_t i = A.fobj[slot];
        const int64_t r0 = A.rp[i];
        const int n = (int)(A.rp[i + 1] - r0);
        int32_t a_old = -1;
        bool icp = false;
        if (A.icp_on) {
            a_old = A.a_prev[i];
            icp = A.lam[a_old] != 0;
        }
        double best = -INFINITY;
        int32_t bj = 0x7fffffff;
        if (icp) {
            best = exact_rho(A, st, r0, n, a_old);
            bj = a_old;
        }
        for (int tile = 0; tile < A.T; ++tile) {
            const int32_t base = tile * A.kt;
            const int32_t width = min(A.kt, A.k - base);
            for (int c0 = 0; c0 < n; c0 += 64) {
                const int h = c0 + lane;
                int64_t s0 = 0, s1 = 0;
                int32_t mv = 0;
                double v = 0.0;
                if (h < n) {
                    const int64_t t = A.col[r0 + h];
                    v = load_xval64(A.xval, A.x_f64, r0 + h);
                    const int64_t sidx = t * A.T + tile;
                    s0 = A.seg[sidx];
                    s1 = A.seg[sidx + 1];
                    mv = A.mid[sidx];
                }
                const int64_t e = icp ? s0 + mv : s1;
                const int cnt = min(64, n - c0);
                for (int q = 0; q < cnt; ++q) {
                    const int64_t ps = bcast_i64(s0, q), pe = bcast_i64(e, q);
                    const double vq = bcast_f64(v, q);
                    for (int64_t p = ps + lane; p < pe; p += 64) {
                        const uint16_t c = A.cid[p];
                        acc[c] = acc[c] + vq * v64[p];
                    }
                }
            }
            double tb = -INFINITY;
            int32_t tj = 0x7fffffff;
            for (int jj = lane; jj < width; jj += 64) {
                const int32_t j = base + jj;
                const double r = acc[jj];
                acc[jj] = 0.0;
                if (!icp || A.lam[j] == 0) {
                    if (r > tb || (r == tb && j < tj)) {
                        tb = r;
                        tj = j;
                    }
                }
            }
            wave_argmax(tb, tj);
            if (tb > best || (tb == best && tj < bj)) {
                best = tb;
                bj = tj;
            }
        }
        if (lane == 0) {
            A.a_new[i] = bj;
            A.own_new[i] = (float)best;
        }
    }
}

hipError_t rescore_full(const WalkArgs& a, const double* v64, const Store st, int64_t grid, hipStream_t s) {
    if (grid < 1) grid = 1;
    const size_t lds = (size_t)a.kt * sizeof(double);
    hipLaunchKernelGGL(k_rescore_full, dim3((unsigned)grid), dim3(64), lds, s, a, v64, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// finalisation: copy out, moved count, changed clusters, objective partials
// ---------------------------------------------------------------------------
constexpr int kFinThreads = 256;

__global__ __launch_bounds__(kFinThreads) void k_finalize_assign(int64_t n, int iter, const int32_t* __restrict__ a_new,
                                                                const float* __restrict__ own_new,
                                                                int32_t* __restrict__ a_io, float* __restrict__ own_io,
                                                                uint8_t* __restrict__ changed,
                                                                unsigned long long* __restrict__ counters,
                                                                double* __restrict__ obj_partial) {
    __shared__ double sh[kFinThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = min(n, lo + per);
    double osum = 0.0;
    unsigned long long moved = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kFinThreads) {
        const int32_t an = a_new[i];
        const float on = own_new[i];
        if (iter > 1) {
            const int32_t ao = a_io[i];
            if (ao != an) {
                changed[ao] = 1;
                changed[an] = 1;
                ++moved;
            }
        } else {
            ++moved;
        }
        a_io[i] = an;
        own_io[i] = on;
        osum = osum + (double)on;
    }
    // fixed-shape reduction: deterministic for a given grid
    osum = wave_sum_f64(osum);
    const int64_t mv = wave_sum_i64((int64_t)moved);
    if (lane == 0) sh[wid] = osum;
    if (lane == 0 && mv) atomicAdd(&counters[5], (unsigned long long)mv);
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kFinThreads / 64; ++w) t = t + sh[w];
        obj_partial[blockIdx.x] = t;
    }
}

hipError_t finalize_assign(int64_t n, int iter, const int32_t* a_new, const float* own_new, int32_t* a_io,
                           float* own_io, uint8_t* changed, unsigned long long* counters, double* obj_partial,
                           int nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_assign, dim3(nblk), dim3(kFinThreads), 0, s, n, iter, a_new, own_new, a_io, own_io,
                       changed, counters, obj_partial);
    return hipGetLastError();
}

__global__ void k_finalize_lambda(int32_t k, int iter, const uint8_t* __restrict__ changed, uint8_t* __restrict__ lam,
                                  unsigned long long* __restrict__ counters, const double* __restrict__ obj_partial,
                                  int nblk, double* __restrict__ obj_out) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool inv = false;
    if (j < k) {
        inv = iter > 1 && changed[j] == 0;
        lam[j] = inv ? 1 : 0;
    }
    const int64_t c = wave_sum_i64(inv ? 1 : 0);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&counters[6], (unsigned long long)c);
    if (j == 0) {
        double t = 0.0;
        for (int b = 0; b < nblk; ++b) t = t + obj_partial[b];
        *obj_out = t;
    }
}

hipError_t finalize_lambda(int32_t k, int iter, const uint8_t* changed, uint8_t* lam_out, unsigned long long* counters,
                           const double* obj_partial, int nblk, double* obj_out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_lambda, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, k, iter, changed,
                       lam_out, counters, obj_partial, nblk, obj_out);
    return hipGetLastError();
}

}  // namespace sivf
