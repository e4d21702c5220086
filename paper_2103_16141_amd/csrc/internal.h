// Internal declarations shared by the C-ABI host code and the HIP kernels of
// libsivf.so.  Nothing here is part of the public ABI (include/sivf.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>

#include "../../include/sivf.h"

namespace sivf {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kCandCap = 32;       // candidate-list capacity per object in the fast pass
constexpr int kTermCap = 128;      // object terms staged in LDS per wave by the fast pass (the rest read from X)
static_assert(kTermCap % 64 == 0, "the walk reads staged terms a whole 64-term chunk at a time");
constexpr int64_t kHeadMaxBytes = 1LL << 36;      // largest dense head-row buffer a file may request
constexpr int kWalkWaves = 4;      // waves per workgroup in the walk kernels
constexpr int kMaxTile = 4096;     // largest similarity tile (centroids) per wave

// A device CSR that passed validation.
struct Csr {
    int64_t n = 0, d = 0, nnz = 0;
    const int64_t* rp = nullptr;
    const int32_t* col = nullptr;
    const void* val = nullptr;
    int f64 = 0;      // values are double (else float)
    int nonneg = 0;   // every value >= 0
};

// FP64 centroid store in "padded CSR" form: centroid j's sorted (term, value)
// entries live at [start[j], start[j] + nnz[j]) of term/val.
struct Store {
    int64_t* start = nullptr;
    int64_t* nnz = nullptr;
    int32_t* term = nullptr;
    double* val = nullptr;
    int64_t cap = 0;    // capacity of term/val
};

// Everything one launch of the fast walk needs (passed by value).
struct WalkArgs {
    int64_t n;
    const int64_t* rp;
    const int32_t* col;
    const void* xval;
    int x_f64;
    int32_t k, kt, T;
    const int64_t* seg;     // [d*T + 1] segment starts, segment (t, tile) = t*T + tile
    const int32_t* mid;     // [d*T] moving-part length of each segment
    const uint4* rec;       // [T*d] record of segment (t, tile) at tile*d + t: start (lo, hi),
                            // length | moving length << 16, dense head row or -1
    int64_t d;
    const uint16_t* cid;    // tile-local positions
    const int32_t* perm;    // [k] centroid id at each position
    int32_t nmv;            // moving centroids: positions [0, nmv)
    const void* pval;       // f32 or bf16 posting values
    const uint8_t* lam;     // flags the file is structured by (lambda^[r-1])
    const double* cnorm;    // ||mu_j|| upper bounds (signed-data bound)
    const int32_t* a_prev;  // a^[r-1]
    const float* own_prev;  // own similarity written at r-1
    int icp_on;             // iter >= 2 and filter mode uses ICP
    int cbicp;              // ICP by per-posting test over whole lists
    int nonneg;             // relative bound (X and centroids nonnegative)
    int certify;
    double eta_val;         // relative rounding of posting values
    double eta_x;           // relative rounding of object values (f64 X -> f32)
    // outputs
    int32_t* a_new;
    float* own_new;
    int32_t* qobj;          // candidate re-score queue: object ids
    int32_t* qcand;         // kCandCap candidates per queue slot
    int32_t* qcnt;          // candidates per slot
    int32_t* fobj;          // full re-score queue: object ids
    unsigned long long* counters;  // [0] multadds [1] queue len [2] full len [3] icp objects
                                   // [4] re-scored candidates [5] moved [6] invariant
                                   // [7] relaxed-ICP objects [9] own64 queue length
                                   // [10] bytes requested by the walk's vector loads
                                   // [11] of which 16-byte-per-lane loads
                                   // [16 + launch] walk work counters
    int64_t qcap;           // capacity of the candidate queue
    // dense head rows (nullptr head: none)
    const int32_t* head;    // [d] row of each term, -1 if none
    const void* hval;       // [H * kpad] values in the posting dtype
    int64_t kpad;           // row length: T * head_ktp(kt) (each tile padded to 512 slots)
    // relaxed ICP (filter mode RELAXED)
    Store st;                  // the current centroids (FP64 CSR) for exact similarities
    int relaxed;
    const double* own64_prev;  // [n] exact rho to the previous centroid under the previous centroids
    double* own64_cur;         // [n] exact rho to the previous centroid under the current centroids
    uint8_t* st_rel;           // [n] relaxed branch taken (kept between tile launches)
    // per-object running state between launches over successive tile ranges
    double* st_theta;       // [n] largest lower bound so far
    double* st_best;        // [n] best lower bound (diagnostic argmax)
    int32_t* st_bj;         // [n] its centroid
    int32_t* st_cnt;        // [n] candidates (> kCandCap: overflowed)
    int32_t* st_cj;         // [n * kCandCap] candidate ids
    float* st_cr;           // [n * kCandCap] their fast-pass similarities
};

}  // namespace sivf

struct sivf_ivf {
    int32_t k = 0;
    int64_t d = 0;
    int32_t kt = 0, T = 0;
    sivf_dtype pdt = SIVF_F32;
    sivf::Store cur, nxt;           // current centroids, and the buffer the next update writes
    int64_t* seg = nullptr;         // [d*T + 1]
    int32_t* mid = nullptr;         // [d*T]
    uint4* rec = nullptr;           // [T*d] tile-major segment records read by the walk
    int32_t* perm = nullptr;        // [k] centroid id at each position (moving first)
    int32_t* iperm = nullptr;       // [k] position of each centroid
    int32_t nmv = 0;                // moving centroids in the current structure
    uint16_t* cid = nullptr;        // [pcap] position minus tile*kt
    float* v32 = nullptr;           // [pcap] (posting dtype f32)
    uint16_t* v16 = nullptr;        // [pcap] (posting dtype bf16)
    double* v64 = nullptr;          // [pcap] FP64 values (exact re-score over whole lists)
    int64_t P = 0, pcap = 0;
    int32_t* head = nullptr;        // [d] dense head row of each term, -1 if none
    void* hval = nullptr;           // [hcap * kpad] dense head rows, posting dtype
    int64_t H = 0, hcap = 0;        // head rows in use / allocated
    uint8_t* lam = nullptr;         // [k]
    double* cnorm = nullptr;        // [k]
    int nonneg = 1;
    size_t bytes = 0;               // device bytes held (counted against the ctx cap)
};

struct sivf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    sivf_options opt{};
    std::string err;
    int n_cu = 256;
    size_t bytes_held = 0;
    std::map<std::string, std::pair<void*, size_t>> ws;  // grow-only named workspace
    hipEvent_t ev[8] = {};
};

namespace sivf {

// ---- launchers (all enqueue on `s`) ----
// generic
hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* bsum_ws, hipStream_t s);
int64_t scan_ws_elems(int64_t n);
hipError_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
hipError_t fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s);
hipError_t fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s);
hipError_t fill_f64(double* p, double v, int64_t n, hipStream_t s);
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

// validation: flags[0] |= error bits, flags[1] = min bad row, flags[2] = any negative
hipError_t validate_csr(const int64_t* rp, const int32_t* col, const void* val, int f64, int64_t n,
                        int64_t d, int64_t nnz, unsigned long long* flags, hipStream_t s);

// flags[0] |= 1 if some a[i] is outside [0, k)
hipError_t range_check_i32(const int32_t* a, int64_t n, int32_t k, unsigned long long* flags, hipStream_t s);

// centroid init: gather rows ids[j] of X into store (start must be exclusive scan of lengths)
hipError_t gather_rows(const Csr& X, const int32_t* ids, int32_t k, Store st, int64_t* lens_out,
                       hipStream_t s, int phase);
hipError_t centroid_norms(const Store st, int32_t k, double* cnorm, hipStream_t s);
hipError_t csr_to_store(const int64_t* ptr, const int32_t* col, const double* val, int32_t k,
                        Store st, hipStream_t s);

// structured inverted file
struct IvfBuildWs {
    unsigned long long* bm;     // [d * W64] centroid-presence bitmap per term
    unsigned long long* lbits;  // [W64] flag bits
    uint16_t* pre0;             // [d * W64] moving-bit prefix within tile
    uint16_t* pre1;             // [d * W64] invariant-bit prefix within tile
    int64_t* cnt;               // [d * T * 2] (term, tile, part) counts
    int64_t* off;               // [d * T * 2 + 1] exclusive scan of cnt
    int64_t* scan_ws;
};
int64_t ivf_w64(int32_t k);
// positions: moving centroids (flag 0) first, each group in ascending id;
// mvpre[k] = number of moving centroids
hipError_t ivf_perm(const uint8_t* lam, int32_t k, int64_t* mv, int64_t* mvpre, int64_t* scan_ws, int32_t* perm,
                    int32_t* iperm, hipStream_t s);
hipError_t ivf_count(const Store st, int32_t k, int64_t d, int32_t kt, int32_t T, const int32_t* iperm,
                     int32_t n_moving, IvfBuildWs w, hipStream_t s);
hipError_t ivf_offsets(int64_t d, int32_t T, IvfBuildWs w, int64_t* seg, int32_t* mid, hipStream_t s);
hipError_t ivf_fill(const Store st, int32_t k, int64_t d, int32_t kt, int32_t T, const int32_t* iperm,
                    int32_t n_moving, IvfBuildWs w, uint16_t* cid, float* v32, uint16_t* v16, double* v64,
                    hipStream_t s);
// dense head rows: flag[t] = 1 if term t's lists hold >= min_len postings
hipError_t head_flags(const int64_t* seg, int64_t d, int32_t T, int64_t min_len, int64_t* flag, hipStream_t s);
hipError_t seg_records(const int64_t* seg, const int32_t* mid, const int32_t* head, int64_t d, int32_t T, uint4* rec,
                       hipStream_t s);
hipError_t head_index(const int64_t* flag, const int64_t* scan, int64_t d, int32_t* head, hipStream_t s);
// head-row slots per tile: kt rounded up to whole 512-centroid batches
inline int32_t head_ktp(int32_t kt) { return (kt + 511) & ~511; }
hipError_t head_fill(const Store st, int32_t k, const int32_t* head, const int32_t* iperm, int64_t kpad, int32_t kt,
                     int32_t ktp, int64_t H, int pdt_bf16, void* hval, hipStream_t s);
hipError_t ivf_export(const sivf_ivf* f, int64_t* term_ptr, int32_t* split, int32_t* p_cid, double* p_val,
                      int64_t* ws_counts, int64_t* scan_ws, hipStream_t s);
hipError_t store_export(const Store st, int32_t k, const int64_t* c_ptr, int32_t* c_col, double* c_val,
                        hipStream_t s);

// assignment
// walks tiles [tb, te) for every object; `work` is a zeroed grab counter
hipError_t walk_fast(const WalkArgs& a, int pdt_bf16, int grid_waves, int tb, int te, unsigned long long* work,
                     hipStream_t s);
int walk_blocks_per_cu(int kt, int pdt_bf16, int cbicp);
hipError_t rescore_candidates(const WalkArgs& a, const Store st, int64_t grid_waves, hipStream_t s);
// exact FP64 similarity of every object to its new centroid (relaxed ICP state)
hipError_t own64_update(const WalkArgs& a, double* own64, int32_t* queue, int64_t grid_waves, hipStream_t s);
hipError_t rescore_full(const WalkArgs& a, const double* v64, const Store st, int64_t grid, hipStream_t s);
hipError_t finalize_assign(int64_t n, int iter, const int32_t* a_new, const float* own_new, int32_t* a_io,
                           float* own_io, uint8_t* changed, unsigned long long* counters,
                           double* obj_partial, int nblk, hipStream_t s);
hipError_t finalize_lambda(int32_t k, int iter, const uint8_t* changed, uint8_t* lam_out,
                           unsigned long long* counters, const double* obj_partial, int nblk,
                           double* obj_out, hipStream_t s);
// exact FP64 objective sum_i rho(x_i, mu_{a_i}) over the centroids in st, in a
// fixed order (partial: nblk doubles of workspace)
hipError_t objective64(const WalkArgs& a, const Store st, const int32_t* assign, double* partial, int nblk,
                       double* out, hipStream_t s);
// changed[a_old[i]] = changed[a_new[i]] = 1 where they differ
hipError_t mark_changed(int64_t n, const int32_t* a_old, const int32_t* a_new, uint8_t* changed, hipStream_t s);
// restart state: exact FP64 rho of each object to its centroid assign[i] in
// st; own32 gets it rounded to FP32, own64 (nullable) gets it where the
// centroid is invariant (lam = 1) and +infinity elsewhere
hipError_t resume_own(const WalkArgs& a, const Store st, const int32_t* assign, const uint8_t* lam, float* own32,
                      double* own64, int64_t grid_waves, hipStream_t s);

// update
struct UpdateWs {
    int64_t* hist;      // [nblk * k] per object-block cluster counts -> offsets
    int64_t* ccount;    // [k] cluster sizes
    int64_t* cstart;    // [k + 1] exclusive scan of sizes
    int32_t* perm;      // [n] objects sorted by cluster (ascending id inside)
    int64_t* memnnz;    // [k] sum of member row lengths
    int64_t* ub;        // [k] entry bound per cluster
    int64_t* ubscan;    // [k + 1] exclusive scan of ub
    double* W;          // [nslots * d] dense FP64 accumulators, kept zero between uses
    int64_t* scan_ws;
    unsigned long long* work; // [1] work counter for seg_sum
    int nslots;
    int64_t nblk;
};
constexpr int kObjBlock = 4096;
hipError_t upd_sort(const int32_t* a, int64_t n, int32_t k, const int64_t* rp, UpdateWs w, hipStream_t s);
hipError_t upd_bounds(int32_t k, int64_t d, const uint8_t* lam, int allow_copy, const Store prev, UpdateWs w,
                      hipStream_t s);
hipError_t upd_segsum(const Csr& X, int32_t k, const uint8_t* lam, int allow_copy, const Store prev,
                      Store next, UpdateWs w, hipStream_t s);

}  // namespace sivf
