// Assignment step (Alg. 4) on CDNA.  One launch per centroid tile covers all
// objects (per-object state carries over between launches); a wave takes one
// object at a time, stages its terms in LDS, reads one 16-byte record per
// (term, tile) -- the segment bounds in the structured file, the length of its
// moving part, the term's dense head row if any -- and gather-accumulates
// v * u into a per-wave similarity tile in LDS:
//   * head terms (held by most centroids) from dense rows of values, 512
//     centroids per batch with 16-byte loads and 16-byte LDS read-add-writes;
//   * other terms from their list segment, 256 postings per batch through a
//     per-list buffer descriptor, the next batch's loads in flight.
// Centroid ids are unique inside a list, so the lanes of one instruction never
// collide: the tile is updated with plain LDS read-add-write (a wave's LDS
// operations complete in order; LDS float atomics are ~25x slower on gfx950).
// Tiles and lists are laid out by position, the moving centroids first (the
// file keeps perm: position -> centroid id).  An object whose own cluster was
// invariant (ICP branch) compares moving centroids only: it stops each list
// at the moving/invariant boundary, reads only the moving prefix of the head
// rows, and skips the tiles past the last moving centroid.  The loads of head
// rows and postings go through the vector memory data path, which is what
// bounds the walk.
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

// Buffer descriptor over `bytes` bytes from `base`: reads past the extent
// return 0 instead of touching memory.  Word 3 is the gfx9 raw-buffer format
// (32-bit data format, no swizzle, no stride).
__device__ inline __amdgpu_buffer_rsrc_t span_rsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// 256 postings of one list: lane l holds postings 4l .. 4l+3, fetched as one
// 8-byte load of their 16-bit ids and one 16-byte (FP32) or 8-byte (BF16)
// load of their values, whole words throughout (the compiler then never
// widens or packs 16-bit values while their loads are in flight).
//   c01, c23 : two 16-bit ids each (low half = the lower posting)
//   u0..u3   : binary32 values (FP32), or two bf16 values in u0 and u1 each
constexpr int kBatch = 256;

struct Batch {
    uint32_t c01, c23, u0, u1, u2, u3;
};

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool BF16>
__device__ inline Batch load_batch(__amdgpu_buffer_rsrc_t dc, __amdgpu_buffer_rsrc_t dv, int off, int lane) {
    Batch b;
    const u32x2 c = __builtin_amdgcn_raw_buffer_load_b64(dc, lane * 8, off * 2, 0);
    b.c01 = c.x;
    b.c23 = c.y;
    if (BF16) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(dv, lane * 8, off * 2, 0);
        b.u0 = v.x;
        b.u1 = v.y;
        b.u2 = 0;
        b.u3 = 0;
    } else {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(dv, lane * 16, off * 4, 0);
        b.u0 = v.x;
        b.u1 = v.y;
        b.u2 = v.z;
        b.u3 = v.w;
    }
    return b;
}

// sim[c] += vq * u for the batch's postings whose position relative to the
// batch start lies in [bs, be).  They belong to one list, so their ids are
// distinct: all four are read first, then written.  In a partial batch the
// lane's postings outside the list use its own spare slot sim[kt + lane]
// instead (no branches).  CB (IVF-CBICP) zeroes the products of invariant
// centroids instead of stopping lists early.
template <bool BF16, bool CB>
__device__ inline void accumulate_batch(const WalkArgs& A, float* sim, const Batch& b, int bs, int be, float vq,
                                        int lane, bool test_flag, int32_t base) {
    uint32_t c[4] = {b.c01 & 0xffffu, b.c01 >> 16, b.c23 & 0xffffu, b.c23 >> 16};
    float u[4];
    if (BF16) {
        u[0] = __uint_as_float(b.u0 << 16);
        u[1] = __uint_as_float(b.u0 & 0xffff0000u);
        u[2] = __uint_as_float(b.u1 << 16);
        u[3] = __uint_as_float(b.u1 & 0xffff0000u);
    } else {
        u[0] = __uint_as_float(b.u0);
        u[1] = __uint_as_float(b.u1);
        u[2] = __uint_as_float(b.u2);
        u[3] = __uint_as_float(b.u3);
    }
    if (!(bs <= 0 && be >= kBatch)) {
        // position of posting i of this lane: 4 * lane + i
        const uint32_t rel = (uint32_t)(4 * lane - bs), n = (uint32_t)(be - bs);
        const uint32_t spare = (uint32_t)(A.kt + lane);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (rel + i >= n) c[i] = spare;
    }
    if (CB && test_flag) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if ((int)c[i] < A.kt && base + (int)c[i] >= A.nmv) u[i] = 0.0f;
    }
    const float o0 = sim[c[0]], o1 = sim[c[1]], o2 = sim[c[2]], o3 = sim[c[3]];
    sim[c[0]] = __builtin_fmaf(vq, u[0], o0);
    sim[c[1]] = __builtin_fmaf(vq, u[1], o1);
    sim[c[2]] = __builtin_fmaf(vq, u[2], o2);
    sim[c[3]] = __builtin_fmaf(vq, u[3], o3);
}

// Dense head rows, accumulated in registers.  The head terms of a chunk are
// taken one row at a time over a 512-centroid group of the tile: lane l holds
// the sums of centroids 4l .. 4l + 3 and 256 + 4l .. 256 + 4l + 3 of the
// group, adds v * row for each head term (one fused multiply-add per
// centroid), and the group's sums enter the LDS tile once per chunk (one
// 16-byte read-add-write per lane and 256 centroids).  FP32 rows hold a
// tile's centroids in order (two 16-byte loads per lane, term and group);
// BF16 rows interleave each 512-centroid block so that one 16-byte load gives
// a lane both of its 4-centroid groups.

constexpr int kHeadGroup = 512;   // centroids of one register-held group

// bytes one wave's vector loads request (64 lanes x width), for the walk's
// load counter: a list batch (8-byte id loads; 16-byte FP32 or 8-byte BF16
// value loads), a segment record (16-byte loads)
constexpr uint32_t kListBatchBytes32 = 512 + 1024;
constexpr uint32_t kListBatchBytes16 = 512 + 512;
constexpr uint32_t kRecordBytes = 64 * 16;

struct HAcc {
    float4 a, b;   // centroids 4l.. and 256 + 4l.. of the group
};

template <bool BF16>
struct HRow {
    u32x4 a, b;    // FP32: the two 4-centroid groups; BF16: a holds both (b unused)
};

// A head row's slots of a tile as a buffer: base = the byte address of the
// tile's first slot in the row (kept per term as two 32-bit halves), `bytes`
// the extent; loads past it read 0 without touching memory.  Offsets stay
// below 16 KiB, so the rows together may span any number of bytes.
__device__ inline __amdgpu_buffer_rsrc_t head_rsrc(uint32_t lo, uint32_t hi, int bytes) {
    const uint64_t base = ((uint64_t)hi << 32) | lo;
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, bytes, 0x00020000);
}

// vo: the lane's byte offset (16 * lane plus the group's start)
template <bool BF16>
__device__ inline HRow<BF16> hrow_load(__amdgpu_buffer_rsrc_t r, int vo) {
    HRow<BF16> h;
    h.a = __builtin_amdgcn_raw_buffer_load_b128(r, vo, 0, 0);
    if (!BF16) h.b = __builtin_amdgcn_raw_buffer_load_b128(r, vo + 1024, 0, 0);
    return h;
}

__device__ inline float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

__device__ inline void fma4(float4& s, float x, float a, float b, float c, float d) {
    s.x = __builtin_fmaf(x, a, s.x);
    s.y = __builtin_fmaf(x, b, s.y);
    s.z = __builtin_fmaf(x, c, s.z);
    s.w = __builtin_fmaf(x, d, s.w);
}

template <bool BF16>
__device__ inline void hrow_fma(HAcc& acc, const HRow<BF16>& h, float x) {
    if (BF16) {
        fma4(acc.a, x, bf_lo(h.a.x), bf_hi(h.a.x), bf_lo(h.a.y), bf_hi(h.a.y));
        fma4(acc.b, x, bf_lo(h.a.z), bf_hi(h.a.z), bf_lo(h.a.w), bf_hi(h.a.w));
    } else {
        fma4(acc.a, x, __uint_as_float(h.a.x), __uint_as_float(h.a.y), __uint_as_float(h.a.z),
             __uint_as_float(h.a.w));
        fma4(acc.b, x, __uint_as_float(h.b.x), __uint_as_float(h.b.y), __uint_as_float(h.b.z),
             __uint_as_float(h.b.w));
    }
}

__device__ inline void add4(float* p, const float4& v) {
    float4* q = (float4*)p;
    float4 o = *q;
    o.x = o.x + v.x;
    o.y = o.y + v.y;
    o.z = o.z + v.z;
    o.w = o.w + v.w;
    *q = o;
}

// The head terms of one chunk (bits of dl: lanes whose term has a head row
// hrow, with object value v) over the tile's slots [0, dl_lim).  First each
// such lane computes the byte address of its row's slice for this tile, and a
// lane permutation moves the i-th head term (ascending term order) to lane i,
// so the loop below walks terms by a counter and takes each term's address
// and value with lane reads, with no per-term address arithmetic.  Then per
// group of 512 centroids, every term's row is loaded (the next term's loads in
// flight while the current one is added) and summed in registers, and the
// sums are merged into the tile below kt.  Returns the 4-byte words fetched.
template <bool BF16>
__device__ inline uint32_t head_terms(const WalkArgs& A, float* sim, unsigned long long dl, int32_t hrow, float v,
                                      int tile, int ktp, int dl_lim, int lane) {
    const int nt = __popcll(dl);
    const bool mine = (dl >> lane) & 1ull;
    const uint64_t esz = BF16 ? 2 : 4;
    const uint64_t addr = (uint64_t)A.hval +
                          ((uint64_t)(uint32_t)(mine ? hrow : 0) * (uint64_t)A.kpad + (uint64_t)tile * ktp) * esz;
    // destination lane: rank among the head lanes, the others after them
    const int rank = mine ? lanes_below(dl) : nt + lanes_below(~dl);
    const uint32_t plo = (uint32_t)__builtin_amdgcn_ds_permute(rank * 4, (int)(uint32_t)addr);
    const uint32_t phi = (uint32_t)__builtin_amdgcn_ds_permute(rank * 4, (int)(uint32_t)(addr >> 32));
    const float pv = __int_as_float(__builtin_amdgcn_ds_permute(rank * 4, __float_as_int(v)));
    uint32_t words = 0;
    for (int at = 0; at < dl_lim; at += kHeadGroup) {
        const int rem = min(dl_lim - at, kHeadGroup);
        // slots the loads may read: whole 256-centroid groups (FP32) or the
        // 512-centroid interleaved block (BF16)
        const int lim = BF16 ? kHeadGroup : (rem + 255) & ~255;
        const int bytes = lim * (int)esz;
        const int end = (at + lim) * (int)esz;   // extent of the buffer from the tile's first slot
        const int vo = 16 * lane + at * (int)esz;
        words += (uint32_t)nt * (uint32_t)bytes / 4u;
        HAcc acc;
        acc.a = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        acc.b = acc.a;
        auto term = [&](int i, float& x) -> HRow<BF16> {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)plo, i);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)phi, i);
            x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pv), i));
            return hrow_load<BF16>(head_rsrc(lo, hi, end), vo);
        };
        // two terms per trip, one loop exit, so the sums stay in the same
        // registers (no copies between the two halves)
        float xa, xb;
        HRow<BF16> RA = term(0, xa), RB;
        int i = 1;
        while (i + 1 < nt) {
            RB = term(i, xb);
            hrow_fma<BF16>(acc, RA, xa);
            RA = term(i + 1, xa);
            hrow_fma<BF16>(acc, RB, xb);
            i += 2;
        }
        if (i < nt) {
            RB = term(i, xb);
            hrow_fma<BF16>(acc, RA, xa);
            hrow_fma<BF16>(acc, RB, xb);
        } else {
            hrow_fma<BF16>(acc, RA, xa);
        }
        const int c0 = at + 4 * lane, c1 = c0 + 256;
        if (c0 < A.kt) add4(sim + c0, acc.a);
        if (256 < lim && c1 < A.kt) add4(sim + c1, acc.b);
    }
    return words;
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

// ---------------------------------------------------------------------------
// fast pass
// ---------------------------------------------------------------------------
// BF16 instantiations ask for 6 waves per SIMD (80 VGPRs): measured 6% faster
// at N=8M, k=10k; the FP32 ones stay at the compiler's choice (5 waves),
// where the cap's spills cost more than the extra wave gains.
template <bool BF16, bool CB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BF16 ? 6 : 5))) void k_walk_fast(WalkArgs A, unsigned long long* __restrict__ work, int tb,
                                                   int te) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int kts = A.kt + 64;   // tile plus one spare slot per lane
    const int ktp = (A.kt + 511) & ~511;   // a tile's slots in a head row
    float* sim = lds + wid * kts;
    int32_t* cj = (int32_t*)(lds + kWalkWaves * kts) + wid * kCandCap;
    float* cr = (float*)((int32_t*)(lds + kWalkWaves * kts) + kWalkWaves * kCandCap) + wid * kCandCap;
    int32_t* tt = (int32_t*)(lds + kWalkWaves * (kts + 2 * kCandCap)) + wid * kTermCap;
    float* tv = lds + kWalkWaves * (kts + 2 * kCandCap + kTermCap) + wid * kTermCap;
    for (int jj = lane; jj < A.kt; jj += 64) sim[jj] = 0.0f;

    unsigned long long macc = 0, icp_cnt = 0, rel_cnt = 0;
    uint32_t lwords = 0;   // 4-byte words requested by this wave's vector loads (flushed at 2^31)
    uint32_t hwords = 0;   // of which words of 16-byte-per-lane loads (head rows, records)
    const uint32_t xb = 4u + (A.x_f64 ? 8u : 4u);   // one staged term: column + value
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
            if (tb == 0) icp_cnt += icp ? 1 : 0;
            // relaxed ICP: own cluster moved, but the exact similarity to the
            // own centroid did not decrease -> moving centroids only
            bool rel = false;
            if (A.relaxed && A.icp_on && !icp) {
                if (tb == 0) {
                    const double rn = exact_rho(A, A.st, r0, n, a_old);
                    rel = rn >= A.own64_prev[i];
                    if (lane == 0) {
                        A.own64_cur[i] = rn;
                        if (te < A.T) A.st_rel[i] = rel ? 1 : 0;
                    }
                    rel_cnt += rel ? 1 : 0;
                } else {
                    rel = A.st_rel[i] != 0;
                }
            }
            const bool filt = icp || rel;   // compare moving centroids only
            const bool front_only = filt && !CB;
            const bool test_flag = icp && CB;
            // front_only objects stop at the tile holding the last moving
            // position; in a launch wholly past it their state stays as is
            const int tmv = (A.nmv + A.kt - 1) / A.kt;
            const int te_obj = front_only ? max(tb, min(te, tmv)) : te;
            if (te_obj == tb && tb > 0 && te < A.T) continue;
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
            int ccount = 0;             // > kCandCap once the list has overflowed
            if (tb > 0) {
                // resume after the tiles of earlier launches
                theta = A.st_theta[i];
                best_lo = A.st_best[i];
                best_j = A.st_bj[i];
                ccount = A.st_cnt[i];
                if (lane < min(ccount, kCandCap)) {
                    cj[lane] = A.st_cj[i * kCandCap + lane];
                    cr[lane] = A.st_cr[i * kCandCap + lane];
                }
            } else if (icp) {
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
            bool overflow = ccount > kCandCap;

            // Stage the object's first kTermCap terms and values in LDS once
            // (each lane later reads only the entries it wrote itself).
            for (int h = lane; h < min(n, kTermCap); h += 64) {
                const int32_t t = A.col[r0 + h];
                tt[h] = t;
                tv[h] = load_xval(A.xval, A.x_f64, r0 + h);
            }
            lwords += (uint32_t)min(n, kTermCap) * (xb / 4);
            if (lwords >= 0x80000000u) {   // wave-uniform; far below any one object's share
                if (lane == 0) {
                    atomicAdd(&A.counters[10], 4ull * lwords);
        atomicAdd(&A.counters[11], 4ull * hwords);
                    atomicAdd(&A.counters[11], 4ull * hwords);
                }
                lwords = 0;
                hwords = 0;
            }
            // Work is a sequence of (tile, term chunk) pairs, tile-major; an
            // empty row still has one pair per tile so every tile is closed.
            const int nch = max(1, (n + 63) >> 6);
            const int npairs = (te_obj - tb) * nch;
            // segment record and object value of pair pi, issued one pair ahead
            // of their use and decoded only there: every lane loads (terms past
            // the row read term 0's record), so no condition makes the compiler
            // wait for the load right away
            uint4 nrec = {0u, 0u, 0u, 0u};
            bool nin = false;
            float nv = 0.0f;
            auto seg_load = [&](int pi) {
                const int rel = pi / nch;   // tile index within this launch
                const int tl = tb + rel;
                const int hb = (pi - rel * nch) * 64;
                const int h = hb + lane;
                nin = h < n;
                int32_t t;
                float xv;
                if (hb < kTermCap) {   // staged terms (hb + lane < kTermCap)
                    t = tt[hb + lane];
                    xv = tv[hb + lane];
                } else {               // rows longer than kTermCap: n > hb
                    const int64_t hc = r0 + min(h, n - 1);
                    t = A.col[hc];
                    xv = load_xval(A.xval, A.x_f64, hc);
                }
                nrec = A.rec[(int64_t)tl * A.d + (nin ? t : 0)];
                nv = nin ? xv : 0.0f;
                lwords += (kRecordBytes + (hb < kTermCap ? 0u : 64u * xb)) / 4;
                hwords += kRecordBytes / 4;
            };
            seg_load(0);
            for (int pi = 0; pi < npairs; ++pi) {
                const int tile = tb + pi / nch;
                const int ch = pi - (tile - tb) * nch;
                const int32_t base = tile * A.kt;
                const int32_t width = min(A.kt, A.k - base);
                // eligible prefix of the tile (moving positions for filt objects)
                const int32_t elim = filt ? min(width, max(0, A.nmv - base)) : width;
                // dense batches cover [0, dlim); the tile range the walk may
                // have touched, and the epilogue clears, is [0, ew)
                const int32_t dlim = front_only ? elim : A.kt;
                const int32_t ew = front_only ? min(width, (elim + 511) & ~511) : width;
                const uint4 rr = nrec;
                const bool in = nin;
                const float v = nv;
                if (pi + 1 < npairs) seg_load(pi + 1);
                const int64_t s0 = in ? (int64_t)(((uint64_t)rr.y << 32) | rr.x) : 0;
                const int32_t mv = in ? (int32_t)(rr.z >> 16) : 0;
                const int64_t e = s0 + (in ? (front_only ? mv : (int32_t)(rr.z & 0xffffu)) : 0);
                const int32_t hr = in ? (int32_t)rr.w : -1;
                const int h = ch * 64 + lane;
                if (in) macc += test_flag ? (unsigned long long)mv : (unsigned long long)(e - s0);
                // ---- walk the non-empty lists of this chunk in ascending term
                // order, kBatch postings per batch (a batch never spans two
                // lists); the next batch's loads are in flight while the
                // current one is accumulated.  Postings are read through
                // buffer descriptors made per list: the lane offset is a
                // constant, the batch offset is scalar, and lanes past the
                // list's end read 0 from the hardware range check.
                // ---- head terms: dense rows (in the ICP branch their moving
                // prefix only), in ascending term order, whole rows of a
                // 1024-centroid group summed in registers, one merge into
                // the tile per chunk
                int hrow = -1;
                const bool use_head = A.head && !(filt && CB);
                if (use_head && h < n) hrow = hr;
                const unsigned long long dl = ballot(hrow >= 0);
                if (dl) {
                    const uint32_t w = head_terms<BF16>(A, sim, dl, hrow, v, tile, ktp, dlim, lane);
                    lwords += w;
                    hwords += w;
                }
                // ---- other terms: structured lists
                unsigned long long live = ballot(h < n && e > s0 && hrow < 0);
                if (live) {
                    // current list seen from a base aligned to 8 postings:
                    // positions [lo, hi) relative to the base are the list's
                    int lo = 0, hi = 0, off = 0;
                    float lv = 0.0f;
                    __amdgpu_buffer_rsrc_t dc, dv;
                    auto next_list = [&]() -> bool {
                        if (!live) return false;
                        const int q = __builtin_ctzll(live);
                        live &= live - 1;
                        const int64_t ls = bcast_i64(s0, q);
                        const int64_t b0 = ls & ~(int64_t)7;
                        lo = (int)(ls - b0);
                        hi = (int)(bcast_i64(e, q) - b0);
                        {
                            const uint32_t nbt = (uint32_t)((hi + kBatch - 1) / kBatch);
                            lwords += nbt * ((BF16 ? kListBatchBytes16 : kListBatchBytes32) / 4);
                            if (!BF16) hwords += nbt * (1024 / 4);   // the values' 16-byte loads
                        }
                        lv = bcast_f32(v, q);
                        off = 0;
                        // extent rounded up to whole groups of 8 (the arrays keep
                        // 8 spare entries past the last posting)
                        const int64_t span = (hi + 7) & ~7;
                        dc = span_rsrc(A.cid + b0, span * 2);
                        dv = BF16 ? span_rsrc((const uint16_t*)A.pval + b0, span * 2)
                                  : span_rsrc((const float*)A.pval + b0, span * 4);
                        return true;
                    };
                    next_list();
                    Batch X = load_batch<BF16>(dc, dv, off, lane), Y;
                    int xs = lo - off, xe = hi - off, ys = 0, ye = 0;
                    float xv = lv, yv = 0.0f;
                    off += kBatch;
                    for (;;) {
                        if (off >= hi && !next_list()) {
                            accumulate_batch<BF16, CB>(A, sim, X, xs, xe, xv, lane, test_flag, base);
                            break;
                        }
                        Y = load_batch<BF16>(dc, dv, off, lane);
                            ys = lo - off;
                        ye = hi - off;
                        yv = lv;
                        off += kBatch;
                        accumulate_batch<BF16, CB>(A, sim, X, xs, xe, xv, lane, test_flag, base);
                        if (off >= hi && !next_list()) {
                            accumulate_batch<BF16, CB>(A, sim, Y, ys, ye, yv, lane, test_flag, base);
                            break;
                        }
                        X = load_batch<BF16>(dc, dv, off, lane);
                            xs = lo - off;
                        xe = hi - off;
                        xv = lv;
                        off += kBatch;
                        accumulate_batch<BF16, CB>(A, sim, Y, ys, ye, yv, lane, test_flag, base);
                    }
                }
                if (ch == nch - 1) {
                    // ---- tile epilogue: bounds, running theta, candidates; clears the tile
                    double tmax = -INFINITY;
                    int32_t tj = 0x7fffffff;
                    if (A.nonneg) {
                        // lower and upper bounds are non-decreasing in r (the bound is
                        // a fixed multiple of |r| plus a constant): the tile's largest
                        // lower bound is that of its largest eligible r
                        float rmax = -INFINITY;
                        int32_t rj = 0x7fffffff;
                        for (int jj = lane; jj < elim; jj += 64) {
                            const float r = sim[jj];
                            if (r > rmax) {
                                rmax = r;
                                rj = base + jj;
                            }
                        }
                        double rm = (double)rmax;
                        wave_argmax(rm, rj);   // a position; the centroid id below
                        if (rj != 0x7fffffff) rj = A.perm[rj];
                        if (rj != 0x7fffffff) {
                            tmax = rm - bound_of(A, bd, rm, rj);
                            tj = rj;
                        }
                    } else {
                        for (int jj = lane; jj < elim; jj += 64) {
                            const int32_t j = A.perm[base + jj];
                            const double r = (double)sim[jj];
                            const double lo = r - bound_of(A, bd, r, j);
                            if (lo > tmax || (lo == tmax && j < tj)) {
                                tmax = lo;
                                tj = j;
                            }
                        }
                        wave_argmax(tmax, tj);
                    }
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
                    // nonnegative data: r below rlow cannot reach theta (the upper
                    // bound r + B(r) is below theta there, with margin for the
                    // rounding of this test), so only the others take the FP64 test
                    float rlow = -INFINITY;
                    if (A.nonneg && theta > -INFINITY) {
                        const double t = (theta - bd.absl * (1.0 + 0x1p-50)) /
                                         ((1.0 + bd.crel + 0x1p-50) * (1.0 + 0x1p-50)) * (1.0 - 0x1p-45);
                        rlow = __double2float_rd(t);
                    }
                    for (int jj0 = 0; jj0 < ew; jj0 += 64) {
                        const int jj = jj0 + lane;
                        bool take = false;
                        float r32 = 0.0f;
                        int32_t jc = 0;   // the centroid id, once needed
                        if (jj < ew) {
                            r32 = sim[jj];
                            sim[jj] = 0.0f;
                            if (r32 >= rlow && jj < elim) {
                                jc = A.perm[base + jj];
                                const double r = (double)r32;
                                take = r + bound_of(A, bd, r, jc) >= theta;
                            }
                        }
                        const unsigned long long tm = ballot(take);
                        if (tm && !overflow) {
                            const int pos = ccount + lanes_below(tm);
                            if (take && pos < kCandCap) {
                                cj[pos] = jc;
                                cr[pos] = r32;
                            }
                            ccount += __popcll(tm);
                            if (ccount > kCandCap) overflow = true;
                        }
                    }
                }
            }
            if (te < A.T) {
                // later tiles follow in another launch: keep the running state
                if (lane == 0) {
                    A.st_theta[i] = theta;
                    A.st_best[i] = best_lo;
                    A.st_bj[i] = best_j;
                    A.st_cnt[i] = ccount;
                }
                if (lane < min(ccount, kCandCap)) {
                    A.st_cj[i * kCandCap + lane] = cj[lane];
                    A.st_cr[i * kCandCap + lane] = cr[lane];
                }
            } else if (!A.certify) {
                // ---- decision
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
    macc = (unsigned long long)wave_sum_i64((int64_t)macc);
    if (lane == 0) {
        atomicAdd(&A.counters[0], macc);
        atomicAdd(&A.counters[10], 4ull * lwords);
        atomicAdd(&A.counters[11], 4ull * hwords);
        atomicAdd(&A.counters[3], icp_cnt);
        if (rel_cnt) atomicAdd(&A.counters[7], rel_cnt);
    }
}

// per wave: the similarity tile and its 64 spare slots, the candidate list
// (ids, values) and the staged terms (id, value)
static size_t walk_lds_bytes(int kt) {
    return (size_t)kWalkWaves * ((size_t)kt + 64 + 2 * kCandCap + 2 * kTermCap) * sizeof(float);
}

// The four instantiations: posting precision x (SIVF | IVF-CBICP filter).
static const void* walk_kernel(int bf16, int cb) {
    return bf16 ? (cb ? (const void*)k_walk_fast<true, true> : (const void*)k_walk_fast<true, false>)
                : (cb ? (const void*)k_walk_fast<false, true> : (const void*)k_walk_fast<false, false>);
}

hipError_t walk_fast(const WalkArgs& a, int pdt_bf16, int grid_waves, int tb, int te, unsigned long long* work,
                     hipStream_t s) {
    const size_t lds = walk_lds_bytes(a.kt);
    int blocks = (grid_waves + kWalkWaves - 1) / kWalkWaves;
    if (blocks < 1) blocks = 1;
    const void* fn = walk_kernel(pdt_bf16, a.cbicp);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    WalkArgs args = a;
    void* params[] = {&args, &work, &tb, &te};
    return hipLaunchKernel(fn, dim3(blocks), dim3(64 * kWalkWaves), params, lds, s);
}

int walk_blocks_per_cu(int kt, int pdt_bf16, int cbicp) {
    const size_t lds = walk_lds_bytes(kt);
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_kernel(pdt_bf16, cbicp), 64 * kWalkWaves, lds);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
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
                const double r = acc[jj];
                acc[jj] = 0.0;
                if (!icp || base + jj < A.nmv) {
                    const int32_t j = A.perm[base + jj];
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

// ---------------------------------------------------------------------------
// Exact own similarities for the next relaxed ICP decision: the FP64 rho of
// each object to its new centroid.  An object that kept its centroid reuses
// the value from this step (moving centroid: computed by the walk) or from
// the previous one (invariant centroid: unchanged); the others are queued and
// re-scored with exact_rho.
// ---------------------------------------------------------------------------
__global__ void k_own64_known(WalkArgs A, double* __restrict__ own64, int32_t* __restrict__ queue) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int32_t an = A.a_new[i];
    bool known = false;
    if (A.icp_on && A.a_prev[i] == an) {
        known = true;
        if (!A.lam[an]) own64[i] = A.own64_cur[i];   // else: unchanged centroid, value stays
    }
    if (!known) {
        const unsigned long long slot = atomicAdd(&A.counters[9], 1ull);
        queue[slot] = (int32_t)i;
    }
}

__global__ __launch_bounds__(256) void k_own64_exact(WalkArgs A, double* __restrict__ own64,
                                                      const int32_t* __restrict__ queue) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nq = (int64_t)A.counters[9];
    for (int64_t q = wave; q < nq; q += nw) {
        const int32_t i = queue[q];
        const int64_t r0 = A.rp[i];
        const double r = exact_rho(A, A.st, r0, (int)(A.rp[i + 1] - r0), A.a_new[i]);
        if (lane == 0) own64[i] = r;
    }
}

hipError_t own64_update(const WalkArgs& a, double* own64, int32_t* queue, int64_t grid_waves, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_own64_known, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, own64, queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t blocks = (grid_waves + 3) / 4;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_own64_exact, dim3((unsigned)blocks), dim3(256), 0, s, a, own64, queue);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact FP64 objective F(a, mu) = sum_i rho(x_i, mu_{a_i}) (the spherical
// k-means objective of Section 1): each rho is exact_rho's fold (the
// reference order), summed in a fixed order -- every wave adds its objects in
// ascending id, the workgroup adds its waves in order, one thread adds the
// workgroups in order -- so the value is run-to-run identical for a fixed grid.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_objective64(WalkArgs A, Store st, const int32_t* __restrict__ assign,
                                                     double* __restrict__ partial) {
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    double acc = 0.0;
    for (int64_t i = wave; i < A.n; i += nw) {
        const int64_t r0 = A.rp[i];
        const double r = exact_rho(A, st, r0, (int)(A.rp[i + 1] - r0), assign[i]);
        acc = acc + r;
    }
    if (lane == 0) sh[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ void k_sum_partials(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t = t + partial[b];
    *out = t;
}

hipError_t objective64(const WalkArgs& a, const Store st, const int32_t* assign, double* partial, int nblk,
                       double* out, hipStream_t s) {
    if (a.n > 0) {
        hipLaunchKernelGGL(k_objective64, dim3((unsigned)nblk), dim3(256), 0, s, a, st, assign, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    } else {
        nblk = 0;
    }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, partial, nblk, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Restart helpers: the clusters whose membership changed between two
// assignments (Alg. 4, marking invariant clusters), and the exact own
// similarities a restarted assignment step starts the ICP branch from.
// ---------------------------------------------------------------------------
__global__ void k_mark_changed(int64_t n, const int32_t* __restrict__ a_old, const int32_t* __restrict__ a_new,
                               uint8_t* __restrict__ changed) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t ao = a_old[i], an = a_new[i];
        if (ao != an) {
            changed[ao] = 1;
            changed[an] = 1;
        }
    }
}

hipError_t mark_changed(int64_t n, const int32_t* a_old, const int32_t* a_new, uint8_t* changed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_mark_changed, dim3((unsigned)blocks), dim3(256), 0, s, n, a_old, a_new, changed);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_resume_own(WalkArgs A, Store st, const int32_t* __restrict__ assign,
                                                    const uint8_t* __restrict__ lam, float* __restrict__ own32,
                                                    double* __restrict__ own64) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < A.n; i += nw) {
        const int64_t r0 = A.rp[i];
        const int32_t j = assign[i];
        const double r = exact_rho(A, st, r0, (int)(A.rp[i + 1] - r0), j);
        if (lane == 0) {
            own32[i] = (float)r;
            if (own64) own64[i] = lam[j] ? r : INFINITY;
        }
    }
}

hipError_t resume_own(const WalkArgs& a, const Store st, const int32_t* assign, const uint8_t* lam, float* own32,
                      double* own64, int64_t grid_waves, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    int64_t blocks = (grid_waves + 3) / 4;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_resume_own, dim3((unsigned)blocks), dim3(256), 0, s, a, st, assign, lam, own32, own64);
    return hipGetLastError();
}

}  // namespace sivf
