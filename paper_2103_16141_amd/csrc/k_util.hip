// Utility kernels: device-wide exclusive scan, fills, CSR validation, and the
// centroid-store helpers (gather of initial rows, import from CSR, export,
// per-centroid norm bounds).
#include "internal.h"
#include "wave.h"

#pragma clang fp contract(off)

namespace sivf {

// ---------------------------------------------------------------- fills
template <typename T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
static hipError_t fill_any(T* p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) { return fill_any(p, v, n, s); }
hipError_t fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s) { return fill_any(p, v, n, s); }
hipError_t fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) { return fill_any(p, v, n, s); }
hipError_t fill_f64(double* p, double v, int64_t n, hipStream_t s) { return fill_any(p, v, n, s); }
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) { return fill_any(p, v, n, s); }

// ---------------------------------------------------------------- scan
// out[i] = sum_{j < i} in[j] for i in [0, n], three phases: per-chunk totals,
// scan of the totals (one workgroup), per-chunk local scan plus carry-in.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanChunk = kScanThreads * kScanPer;

int64_t scan_ws_elems(int64_t n) { return (n + kScanChunk - 1) / kScanChunk + 1; }

__device__ inline int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t* total) {
    // sh: kScanThreads/64 entries
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan_i64(v);
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    int64_t off = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        int64_t x = sh[w];
        if (w < wid) off += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void k_scan_totals(const int64_t* __restrict__ in, int64_t n, int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int64_t acc = 0;
    for (int q = 0; q < kScanPer; ++q) {
        int64_t i = base + q;
        if (i < n) acc += in[i];
    }
    int64_t tot;
    block_excl_scan(acc, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_bsum(int64_t* __restrict__ bsum, int64_t nb) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        int64_t i = b0 + threadIdx.x;
        int64_t v = i < nb ? bsum[i] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan(v, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void k_scan_apply(const int64_t* __restrict__ in, int64_t n, const int64_t* __restrict__ bsum,
                             int64_t nb, int64_t* __restrict__ out) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int64_t loc[kScanPer];
    int64_t acc = 0;
    for (int q = 0; q < kScanPer; ++q) {
        int64_t i = base + q;
        loc[q] = i < n ? in[i] : 0;
        acc += loc[q];
    }
    int64_t tot;
    int64_t ex = block_excl_scan(acc, sh, &tot) + bsum[blockIdx.x];
    for (int q = 0; q < kScanPer; ++q) {
        int64_t i = base + q;
        if (i < n) out[i] = ex;
        ex += loc[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* bsum, hipStream_t s) {
    if (n <= 0) {
        hipLaunchKernelGGL(k_fill<int64_t>, dim3(1), dim3(64), 0, s, out, (int64_t)0, (int64_t)1);
        return hipGetLastError();
    }
    int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(kScanThreads), 0, s, bsum, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, bsum, nb, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- validation
// flags[0]: bit0 unsorted/row_ptr decreasing, bit1 column out of range,
//           bit2 non-finite value, bit3 row_ptr inconsistent with nnz
// flags[1]: smallest offending row (initialised to ~0 by the host)
// flags[2]: 1 if some value is negative
//
// One wave per group of 64 consecutive rows: lane l holds the bounds of row
// g*64 + l, and the wave reads the group's nonzeros as one contiguous range,
// 64 at a time (coalesced).  For each such window the lanes OR together the
// bits of the row starts that fall in it, so a lane knows whether its element
// opens a row; otherwise its column must exceed its left neighbour's (taken
// by a shuffle, lane 0 from the previous window).  Row bounds that are out of
// order are reported as such and their group's elements are not inspected.
__device__ inline unsigned long long wave_or_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(256) void k_validate(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const void* __restrict__ val, int f64, int64_t n, int64_t d,
                                                  int64_t nnz, unsigned long long* flags) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t ngroups = (n + 63) / 64;
    for (int64_t g = wave; g < ngroups; g += nw) {
        const int64_t i = g * 64 + lane;
        const bool row = i < n;
        int64_t b = 0, e = 0;
        unsigned long long bad = 0;
        if (row) {
            b = rp[i];
            e = rp[i + 1];
            if (i == 0 && b != 0) bad |= 8;
            if (i == n - 1 && e != nnz) bad |= 8;
            if (e < b || b < 0 || e > nnz) bad |= 1;
        }
        int64_t first_bad_row = bad ? i : INT64_MAX;
        const bool bounds_ok = ballot(bad != 0) == 0ull;
        unsigned long long ebad = 0;
        int neg = 0;
        if (bounds_ok) {
            // the group's nonzeros: [rp[g*64], rp[min(g*64+64, n)])
            const int64_t lo = bcast_i64(b, 0);
            const int last_lane = (int)min<int64_t>(63, n - 1 - g * 64);
            const int64_t hi = bcast_i64(e, last_lane);
            int32_t prev_last = -1;
            for (int64_t q = lo; q < hi; q += 64) {
                // rows (non-empty) starting inside [q, q + 64)
                const unsigned long long sb =
                    (row && b < e && b >= q && b < q + 64) ? (1ull << (int)(b - q)) : 0ull;
                const unsigned long long starts = wave_or_u64(sb);
                const int64_t p = q + lane;
                const bool in = p < hi;
                int32_t c = in ? col[p] : 0;
                int32_t left = __shfl_up(c, 1, 64);
                if (lane == 0) left = prev_last;
                unsigned long long eb = 0;
                if (in) {
                    if (c < 0 || c >= d) eb |= 2;
                    if (!((starts >> lane) & 1ull) && c <= left) eb |= 1;
                    const double v = f64 ? ((const double*)val)[p] : (double)((const float*)val)[p];
                    if (!isfinite(v)) eb |= 4;
                    if (v < 0) neg = 1;
                }
                prev_last = __shfl(c, 63, 64);
                if (ballot(eb != 0)) {
                    // error path: the row of each offending element (the last
                    // row of the group starting at or before it)
                    int64_t rbad = INT64_MAX;
                    for (int l = 0; l < 64 && g * 64 + l < n; ++l) {
                        const int64_t bl = bcast_i64(b, l), el = bcast_i64(e, l);
                        if (eb && p >= bl && p < el) rbad = g * 64 + l;
                    }
                    first_bad_row = min(first_bad_row, rbad);
                    ebad |= eb;
                }
            }
        }
        bad |= ebad;
        if (bad) {
            atomicOr(&flags[0], bad);
            atomicMin(&flags[1], (unsigned long long)first_bad_row);
        }
        if (ballot(neg != 0) && lane == 0) atomicOr(&flags[2], 1ull);
    }
}

hipError_t validate_csr(const int64_t* rp, const int32_t* col, const void* val, int f64, int64_t n, int64_t d,
                        int64_t nnz, unsigned long long* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = ((n + 63) / 64 + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, s, rp, col, val, f64, n, d, nnz, flags);
    return hipGetLastError();
}

// flags[0] = 1 if some a[i] is outside [0, k)
__global__ void k_range_i32(const int32_t* __restrict__ a, int64_t n, int32_t k, unsigned long long* flags) {
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= (a[i] < 0 || a[i] >= k);
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&flags[0], 1ull);
}

hipError_t range_check_i32(const int32_t* a, int64_t n, int32_t k, unsigned long long* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_range_i32, dim3((unsigned)blocks), dim3(256), 0, s, a, n, k, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- centroid store helpers
// phase 0: lens_out[j] = nnz of row ids[j]; phase 1: copy the rows (values
// widened to FP64) to st.start[j] and set st.nnz[j].  One wave per centroid.
__global__ void k_gather_rows(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                              const void* __restrict__ val, int f64, const int32_t* __restrict__ ids, int32_t k,
                              Store st, int64_t* lens_out, int phase) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < k; j += nw) {
        int64_t i = ids[j];
        int64_t b = rp[i], e = rp[i + 1];
        if (phase == 0) {
            if (lane == 0) lens_out[j] = e - b;
            continue;
        }
        int64_t o = st.start[j];
        for (int64_t p = b + lane; p < e; p += 64) {
            st.term[o + (p - b)] = col[p];
            st.val[o + (p - b)] = f64 ? ((const double*)val)[p] : (double)((const float*)val)[p];
        }
        if (lane == 0) st.nnz[j] = e - b;
    }
}

hipError_t gather_rows(const Csr& X, const int32_t* ids, int32_t k, Store st, int64_t* lens_out, hipStream_t s,
                       int phase) {
    int64_t blocks = ((int64_t)k * 64 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)blocks), dim3(256), 0, s, X.rp, X.col, X.val, X.f64, ids, k,
                       st, lens_out, phase);
    return hipGetLastError();
}

__global__ void k_csr_to_store(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                               const double* __restrict__ val, int32_t k, Store st) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < k; j += nw) {
        int64_t b = ptr[j], e = ptr[j + 1];
        for (int64_t p = b + lane; p < e; p += 64) {
            st.term[p] = col[p];
            st.val[p] = val[p];
        }
        if (lane == 0) {
            st.start[j] = b;
            st.nnz[j] = e - b;
        }
    }
}

hipError_t csr_to_store(const int64_t* ptr, const int32_t* col, const double* val, int32_t k, Store st,
                        hipStream_t s) {
    int64_t blocks = ((int64_t)k * 64 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_csr_to_store, dim3((unsigned)blocks), dim3(256), 0, s, ptr, col, val, k, st);
    return hipGetLastError();
}

__global__ void k_store_export(Store st, int32_t k, const int64_t* __restrict__ c_ptr, int32_t* c_col,
                               double* c_val) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < k; j += nw) {
        int64_t b = st.start[j], m = st.nnz[j], o = c_ptr[j];
        for (int64_t p = lane; p < m; p += 64) {
            if (c_col) c_col[o + p] = st.term[b + p];
            if (c_val) c_val[o + p] = st.val[b + p];
        }
    }
}

hipError_t store_export(const Store st, int32_t k, const int64_t* c_ptr, int32_t* c_col, double* c_val,
                        hipStream_t s) {
    int64_t blocks = ((int64_t)k * 64 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_store_export, dim3((unsigned)blocks), dim3(256), 0, s, st, k, c_ptr, c_col, c_val);
    return hipGetLastError();
}

// cnorm[j] >= ||mu_j||_2: FP64 sum of squares (relative error <= nnz * 2^-53),
// square root, then a 2^-30 relative margin.
__global__ void k_centroid_norms(Store st, int32_t k, double* __restrict__ cnorm) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < k; j += nw) {
        int64_t b = st.start[j], m = st.nnz[j];
        double acc = 0.0;
        for (int64_t p = lane; p < m; p += 64) {
            double v = st.val[b + p];
            acc = acc + v * v;
        }
        acc = wave_sum_f64(acc);
        if (lane == 0) cnorm[j] = sqrt(acc) * (1.0 + 0x1p-30) + 0x1p-1000;
    }
}

hipError_t centroid_norms(const Store st, int32_t k, double* cnorm, hipStream_t s) {
    int64_t blocks = ((int64_t)k * 64 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_centroid_norms, dim3((unsigned)blocks), dim3(256), 0, s, st, k, cnorm);
    return hipGetLastError();
}

}  // namespace sivf
