// Host side of the C ABI (include/sivf.h): context and workspace management,
// input validation, and the sequencing of the assignment step (Alg. 4),
// update step (Alg. 5) and Lloyd driver (Alg. 1) on one HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"
#include "soft.h"

using namespace sivf;

namespace {

sivf_status fail(sivf_ctx* ctx, sivf_status st, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((ctx), SIVF_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                       \
    } while (0)

#define STCHK(expr)                      \
    do {                                 \
        sivf_status s_ = (expr);         \
        if (s_ != SIVF_OK) return s_;    \
    } while (0)

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool cap_ok(sivf_ctx* ctx, size_t more) {
    return ctx->opt.workspace_cap_bytes == 0 || ctx->bytes_held + more <= ctx->opt.workspace_cap_bytes;
}

sivf_status dev_alloc(sivf_ctx* ctx, void** p, size_t bytes, size_t* account) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    if (!cap_ok(ctx, bytes))
        return fail(ctx, SIVF_E_NOMEM, "workspace cap of %zu bytes exceeded (%zu held, %zu requested)",
                    ctx->opt.workspace_cap_bytes, ctx->bytes_held, bytes);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(ctx, SIVF_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    ctx->bytes_held += bytes;
    if (account) *account += bytes;
    return SIVF_OK;
}

void dev_free(sivf_ctx* ctx, void* p, size_t bytes, size_t* account) {
    if (!p) return;
    if (bytes == 0) bytes = 8;
    (void)hipFree(p);
    ctx->bytes_held -= std::min(ctx->bytes_held, bytes);
    if (account) *account -= std::min(*account, bytes);
}

// Grow-only named workspace buffer owned by the ctx.
template <typename T>
sivf_status ws(sivf_ctx* ctx, const char* name, int64_t elems, T** out) {
    size_t bytes = (size_t)std::max<int64_t>(elems, 1) * sizeof(T);
    auto it = ctx->ws.find(name);
    if (it != ctx->ws.end() && it->second.second >= bytes) {
        *out = (T*)it->second.first;
        return SIVF_OK;
    }
    if (it != ctx->ws.end()) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        dev_free(ctx, it->second.first, it->second.second, nullptr);
        ctx->ws.erase(it);
    }
    size_t grow = bytes + bytes / 8;
    void* p = nullptr;
    STCHK(dev_alloc(ctx, &p, grow, nullptr));
    ctx->ws[name] = {p, grow};
    *out = (T*)p;
    return SIVF_OK;
}

// Workspace of one call, handed out buffer by buffer: the ctx's grow-only
// named buffers (kCtx), consecutive 256-byte aligned pieces of a fixed device
// block that is never allocated or freed here (kFixed), or no memory at all,
// only the byte count such a block needs for the same requests (kMeasure).
struct Work {
    enum Mode { kCtx, kFixed, kMeasure };
    sivf_ctx* ctx;
    Mode mode = kCtx;
    char* base = nullptr;
    size_t cap = 0, used = 0;

    template <typename T>
    sivf_status get(const char* name, int64_t elems, T** out) {
        if (mode == kCtx) return ws(ctx, name, elems, out);
        const size_t bytes = (size_t)std::max<int64_t>(elems, 1) * sizeof(T);
        const size_t at = (used + 255) & ~(size_t)255;
        if (mode == kFixed && at + bytes > cap)
            return fail(ctx, SIVF_E_UNSUPPORTED, "workspace '%s' does not fit the %zu-byte scratch block", name, cap);
        *out = (T*)(base + at);   // kMeasure: an offset, never dereferenced
        used = at + bytes;
        return SIVF_OK;
    }
};

// ------------------------------------------------------------ fixed scratch
// The workspace of sivf_assign_noalloc: one block per device, part of the
// library's device code, so the loader provides it when the library is first
// used on a device and it stays until the process ends.  Host code never
// names the array itself (that is a host-side stand-in, not a device
// address): it uses the address hipGetSymbolAddress reports for each device,
// taken once per device with that device current, when a ctx is created.
constexpr size_t kScratchBytes = 64ull << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device must be current
hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void* scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

sivf_status check_csr_args(sivf_ctx* ctx, const sivf_csr* X, const char* what) {
    if (!X) return fail(ctx, SIVF_E_INVALID, "%s is NULL", what);
    if (X->n_rows < 0 || X->n_cols < 1 || X->nnz < 0)
        return fail(ctx, SIVF_E_SHAPE, "%s: bad sizes n_rows=%lld n_cols=%lld nnz=%lld", what, (long long)X->n_rows,
                    (long long)X->n_cols, (long long)X->nnz);
    if (X->n_cols > INT32_MAX) return fail(ctx, SIVF_E_SHAPE, "%s: n_cols exceeds int32", what);
    if (!X->row_ptr || (X->nnz > 0 && (!X->col || !X->val)))
        return fail(ctx, SIVF_E_INVALID, "%s: NULL array", what);
    if (X->val_dtype != SIVF_F32 && X->val_dtype != SIVF_F64)
        return fail(ctx, SIVF_E_INVALID, "%s: values must be SIVF_F32 or SIVF_F64", what);
    return SIVF_OK;
}

// Validate X on the device on every call that reads it.  Nothing is cached:
// X may be edited in place between calls (same pointers, new contents), and
// both the column range (used as an index by the walk) and the sign of the
// values (which selects the certificate's error bound) must hold for the
// contents the kernels will read.  One coalesced pass over the nonzeros.
sivf_status validate(sivf_ctx* ctx, const sivf_csr* X, Csr* out, Work& w) {
    STCHK(check_csr_args(ctx, X, "X"));
    const int f64 = X->val_dtype == SIVF_F64;
    unsigned long long* flags = nullptr;
    STCHK(w.get("vflags", 4, &flags));
    unsigned long long init[3] = {0ull, ~0ull, 0ull};
    HIPCHK(ctx, hipMemcpyAsync(flags, init, sizeof(init), hipMemcpyHostToDevice, ctx->stream));
    if (X->n_rows > 0)
        HIPCHK(ctx, validate_csr(X->row_ptr, X->col, X->val, f64, X->n_rows, X->n_cols, X->nnz, flags, ctx->stream));
    unsigned long long h[3];
    HIPCHK(ctx, hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (X->n_rows == 0) {
        int64_t rp0 = 0;
        HIPCHK(ctx, hipMemcpy(&rp0, X->row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost));
        if (rp0 != 0 || X->nnz != 0) return fail(ctx, SIVF_E_UNSORTED, "X: empty matrix with row_ptr[0] != 0 or nnz != 0");
    }
    if (h[0] & 1ull) return fail(ctx, SIVF_E_UNSORTED, "X: row %llu has unsorted/duplicate columns or a decreasing row_ptr", h[1]);
    if (h[0] & 8ull) return fail(ctx, SIVF_E_UNSORTED, "X: row_ptr[0] != 0 or row_ptr[n] != nnz");
    if (h[0] & 2ull) return fail(ctx, SIVF_E_RANGE, "X: row %llu has a column outside [0, %lld)", h[1], (long long)X->n_cols);
    if (h[0] & 4ull) return fail(ctx, SIVF_E_NONFINITE, "X: row %llu has a non-finite value", h[1]);
    out->n = X->n_rows;
    out->d = X->n_cols;
    out->nnz = X->nnz;
    out->rp = X->row_ptr;
    out->col = X->col;
    out->val = X->val;
    out->f64 = f64;
    out->nonneg = h[2] ? 0 : 1;
    return SIVF_OK;
}

sivf_status validate(sivf_ctx* ctx, const sivf_csr* X, Csr* out) {
    Work w{ctx};
    return validate(ctx, X, out, w);
}

// Every a[i] must lie in [0, k) before it is used as an index on the device.
sivf_status check_assign(sivf_ctx* ctx, const int32_t* a, int64_t n, int32_t k, const char* what, Work& w) {
    unsigned long long* flags = nullptr;
    STCHK(w.get("aflags", 2, &flags));
    if (n <= 0) return SIVF_OK;
    HIPCHK(ctx, fill_u64(flags, 0ull, 1, ctx->stream));
    HIPCHK(ctx, range_check_i32(a, n, k, flags, ctx->stream));
    unsigned long long h = 0;
    HIPCHK(ctx, hipMemcpyAsync(&h, flags, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (h) return fail(ctx, SIVF_E_RANGE, "%s has a value outside [0, %d)", what, k);
    return SIVF_OK;
}

sivf_status check_assign(sivf_ctx* ctx, const int32_t* a, int64_t n, int32_t k, const char* what) {
    Work w{ctx};
    return check_assign(ctx, a, n, k, what, w);
}

void choose_tiles(const sivf_ctx* ctx, int32_t k, int32_t* kt, int32_t* T) {
    int32_t want = ctx->opt.k_tile;
    if (want <= 0) {
        // widest tile measured fastest at N = 8M, k = 10k (tile-major walk, both dtypes)
        const int32_t kmax = 1024;
        int32_t t = (k + kmax - 1) / kmax;
        int32_t w = (k + t - 1) / t;
        want = ((w + 63) / 64) * 64;
    }
    *kt = want;
    *T = (k + want - 1) / want;
}

// ---------------------------------------------------------------- file storage
sivf_status store_reserve(sivf_ctx* ctx, sivf_ivf* f, Store* st, int64_t cap) {
    if (st->cap >= cap && st->term) return SIVF_OK;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    dev_free(ctx, st->term, (size_t)st->cap * sizeof(int32_t), &f->bytes);
    dev_free(ctx, st->val, (size_t)st->cap * sizeof(double), &f->bytes);
    st->term = nullptr;
    st->val = nullptr;
    st->cap = 0;
    int64_t c = std::max<int64_t>(cap + cap / 8, 64);
    STCHK(dev_alloc(ctx, (void**)&st->term, (size_t)c * sizeof(int32_t), &f->bytes));
    STCHK(dev_alloc(ctx, (void**)&st->val, (size_t)c * sizeof(double), &f->bytes));
    st->cap = c;
    return SIVF_OK;
}

sivf_status postings_reserve(sivf_ctx* ctx, sivf_ivf* f, int64_t P) {
    // spare entries: the walk reads postings in aligned groups of 8, which
    // may reach up to 7 entries past the last one
    if (f->pcap >= P + 8 && f->cid) return SIVF_OK;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    dev_free(ctx, f->cid, (size_t)f->pcap * 2, &f->bytes);
    dev_free(ctx, f->v32, (size_t)f->pcap * 4, &f->bytes);
    dev_free(ctx, f->v16, (size_t)f->pcap * 2, &f->bytes);
    dev_free(ctx, f->v64, (size_t)f->pcap * 8, &f->bytes);
    f->cid = nullptr;
    f->v32 = nullptr;
    f->v16 = nullptr;
    f->v64 = nullptr;
    f->pcap = 0;
    int64_t c = std::max<int64_t>(P + P / 8 + 8, 64);
    STCHK(dev_alloc(ctx, (void**)&f->cid, (size_t)c * 2, &f->bytes));
    if (f->pdt == SIVF_BF16) {
        STCHK(dev_alloc(ctx, (void**)&f->v16, (size_t)c * 2, &f->bytes));
    } else {
        STCHK(dev_alloc(ctx, (void**)&f->v32, (size_t)c * 4, &f->bytes));
    }
    STCHK(dev_alloc(ctx, (void**)&f->v64, (size_t)c * 8, &f->bytes));
    f->pcap = c;
    return SIVF_OK;
}

void free_file(sivf_ctx* ctx, sivf_ivf* f) {
    if (!f) return;
    (void)hipStreamSynchronize(ctx->stream);
    Store* sts[2] = {&f->cur, &f->nxt};
    for (Store* st : sts) {
        dev_free(ctx, st->start, (size_t)f->k * 8, &f->bytes);
        dev_free(ctx, st->nnz, (size_t)f->k * 8, &f->bytes);
        dev_free(ctx, st->term, (size_t)st->cap * 4, &f->bytes);
        dev_free(ctx, st->val, (size_t)st->cap * 8, &f->bytes);
    }
    dev_free(ctx, f->seg, (size_t)(f->d * f->T + 1) * 8, &f->bytes);
    dev_free(ctx, f->mid, (size_t)(f->d * f->T) * 4, &f->bytes);
    dev_free(ctx, f->rec, (size_t)(f->d * f->T) * 16, &f->bytes);
    dev_free(ctx, f->perm, (size_t)f->k * 4, &f->bytes);
    dev_free(ctx, f->iperm, (size_t)f->k * 4, &f->bytes);
    dev_free(ctx, f->cid, (size_t)f->pcap * 2, &f->bytes);
    dev_free(ctx, f->v32, (size_t)f->pcap * 4, &f->bytes);
    dev_free(ctx, f->v16, (size_t)f->pcap * 2, &f->bytes);
    dev_free(ctx, f->v64, (size_t)f->pcap * 8, &f->bytes);
    dev_free(ctx, f->lam, (size_t)f->k, &f->bytes);
    dev_free(ctx, f->cnorm, (size_t)f->k * 8, &f->bytes);
    dev_free(ctx, f->head, (size_t)f->d * 4, &f->bytes);
    dev_free(ctx, f->hval, (size_t)f->hcap * f->T * head_ktp(f->kt) * (f->pdt == SIVF_BF16 ? 2 : 4), &f->bytes);
    delete f;
}

sivf_status new_file(sivf_ctx* ctx, int32_t k, int64_t d, sivf_ivf** out) {
    sivf_ivf* f = new (std::nothrow) sivf_ivf();
    if (!f) return fail(ctx, SIVF_E_NOMEM, "host allocation failed");
    f->k = k;
    f->d = d;
    f->pdt = ctx->opt.posting_dtype;
    choose_tiles(ctx, k, &f->kt, &f->T);
    sivf_status st = SIVF_OK;
    for (Store* s : {&f->cur, &f->nxt}) {
        if (st == SIVF_OK) st = dev_alloc(ctx, (void**)&s->start, (size_t)k * 8, &f->bytes);
        if (st == SIVF_OK) st = dev_alloc(ctx, (void**)&s->nnz, (size_t)k * 8, &f->bytes);
    }
    if (st == SIVF_OK) st = dev_alloc(ctx, (void**)&f->seg, (size_t)(d * f->T + 1) * 8, &f->bytes);
    if (st == SIVF_OK) st = dev_alloc(ctx, (void**)&f->mid, (size_t)(d * f->T) * 4, &f->bytes);
    if (st == SIVF_OK) st = dev_alloc(ctx, (void**)&f->rec, (size_t)(d * f->T) * 16, &f->bytes);
    if (st == SIVF_OK) st = dev_alloc(ctx, (void**)&f->perm, (size_t)k * 4, &f->bytes);
    if (st == SIVF_OK) st = dev_alloc(ctx, (void**)&f->iperm, (size_t)k * 4, &f->bytes);
    if (st == SIVF_OK) st = dev_alloc(ctx, (void**)&f->lam, (size_t)k, &f->bytes);
    if (st == SIVF_OK) st = dev_alloc(ctx, (void**)&f->cnorm, (size_t)k * 8, &f->bytes);
    if (st == SIVF_OK && ctx->opt.head_density > 0.0f) st = dev_alloc(ctx, (void**)&f->head, (size_t)d * 4, &f->bytes);
    if (st != SIVF_OK) {
        free_file(ctx, f);
        return st;
    }
    *out = f;
    return SIVF_OK;
}

// Structure f's current centroids by the flags in f->lam (Alg. 5 second half):
// positions put the moving centroids first, then the file is built by position.
sivf_status restructure(sivf_ctx* ctx, sivf_ivf* f) {
    const int64_t W64 = ivf_w64(f->k);
    const int64_t nseg2 = f->d * f->T * 2;
    IvfBuildWs w{};
    STCHK(ws(ctx, "ivf_bm", W64 * f->d, &w.bm));
    STCHK(ws(ctx, "ivf_lbits", W64, &w.lbits));
    STCHK(ws(ctx, "ivf_pre0", W64 * f->d, &w.pre0));
    STCHK(ws(ctx, "ivf_pre1", W64 * f->d, &w.pre1));
    STCHK(ws(ctx, "ivf_cnt", nseg2, &w.cnt));
    STCHK(ws(ctx, "ivf_off", nseg2 + 1, &w.off));
    STCHK(ws(ctx, "scan_ws", scan_ws_elems(std::max<int64_t>(nseg2, f->k + 1)) + 8,
             &w.scan_ws));
    int64_t* pmv = nullptr;
    int64_t* pmvpre = nullptr;
    STCHK(ws(ctx, "ivf_mv", (int64_t)f->k, &pmv));
    STCHK(ws(ctx, "ivf_mvpre", (int64_t)f->k + 1, &pmvpre));
    HIPCHK(ctx, ivf_perm(f->lam, f->k, pmv, pmvpre, w.scan_ws, f->perm, f->iperm, ctx->stream));
    int64_t nmv = 0;
    HIPCHK(ctx, hipMemcpyAsync(&nmv, pmvpre + f->k, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    f->nmv = (int32_t)nmv;
    HIPCHK(ctx, ivf_count(f->cur, f->k, f->d, f->kt, f->T, f->iperm, f->nmv, w, ctx->stream));
    HIPCHK(ctx, ivf_offsets(f->d, f->T, w, f->seg, f->mid, ctx->stream));
    // dense head rows: terms whose lists hold >= ceil(head_density * k) postings
    int64_t* hflag = nullptr;
    int64_t* hscan = nullptr;
    int64_t H = 0;
    if (f->head) {
        const int64_t min_len = std::max<int64_t>(1, (int64_t)std::ceil((double)ctx->opt.head_density * f->k));
        STCHK(ws(ctx, "head_flag", f->d + 1, &hflag));
        STCHK(ws(ctx, "head_scan", f->d + 1, &hscan));
        HIPCHK(ctx, head_flags(f->seg, f->d, f->T, min_len, hflag, ctx->stream));
        HIPCHK(ctx, exclusive_scan_i64(hflag, hscan, f->d, w.scan_ws, ctx->stream));
        HIPCHK(ctx, head_index(hflag, hscan, f->d, f->head, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(&H, hscan + f->d, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    }
    int64_t P = 0, total = 0;
    int64_t* cscan = nullptr;
    STCHK(ws(ctx, "ivf_cscan", (int64_t)f->k + 1, &cscan));
    HIPCHK(ctx, exclusive_scan_i64(f->cur.nnz, cscan, f->k, w.scan_ws, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(&total, cscan + f->k, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(&P, f->seg + f->d * f->T, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (P != total)
        return fail(ctx, SIVF_E_HIP, "internal: %lld postings for %lld centroid entries", (long long)P, (long long)total);
    STCHK(postings_reserve(ctx, f, P));
    f->P = P;
    HIPCHK(ctx, ivf_fill(f->cur, f->k, f->d, f->kt, f->T, f->iperm, f->nmv, w, f->cid, f->v32, f->v16, f->v64,
                         ctx->stream));
    f->H = 0;
    if (f->head && H > 0) {
        const int64_t kpad = (int64_t)f->T * head_ktp(f->kt), esz = f->pdt == SIVF_BF16 ? 2 : 4;
        // every row is addressed through a descriptor of its own, so the rows
        // together may exceed 4 GiB; kHeadMaxBytes only bounds the request
        if (H * kpad * esz > kHeadMaxBytes)
            return fail(ctx, SIVF_E_UNSUPPORTED,
                        "dense head rows would take %lld bytes (%lld rows), above %lld; raise head_density",
                        (long long)(H * kpad * esz), (long long)H, (long long)kHeadMaxBytes);
        if (H > f->hcap) {
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            dev_free(ctx, f->hval, (size_t)(f->hcap * kpad * esz), &f->bytes);
            f->hval = nullptr;
            f->hcap = 0;
            const int64_t c = std::min<int64_t>(H + H / 8 + 16, std::min<int64_t>(f->d, kHeadMaxBytes / (kpad * esz)));
            STCHK(dev_alloc(ctx, &f->hval, (size_t)(c * kpad * esz), &f->bytes));
            f->hcap = c;
        }
        HIPCHK(ctx, head_fill(f->cur, f->k, f->head, f->iperm, kpad, f->kt, head_ktp(f->kt), H, f->pdt == SIVF_BF16,
                              f->hval, ctx->stream));
        f->H = H;
    }
    HIPCHK(ctx, seg_records(f->seg, f->mid, f->H > 0 ? f->head : nullptr, f->d, f->T, f->rec, ctx->stream));
    // norm bounds for the signed-data certificate: needed whenever the X of a
    // later call has a negative value, whatever the centroids' signs
    HIPCHK(ctx, centroid_norms(f->cur, f->k, f->cnorm, ctx->stream));
    return SIVF_OK;
}

// ------------------------------------------------------------ step bodies
// The ABI entry points validate their arguments (X on every call) and then
// run these; the Lloyd driver validates X once and calls them directly.

sivf_status init_impl(sivf_ctx* ctx, const Csr& Xc, int32_t k, const int32_t* init_ids_host, sivf_ivf** out) {
    if (k < 1 || k > Xc.n) return fail(ctx, SIVF_E_SHAPE, "need 1 <= k <= N (k=%d, N=%lld)", k, (long long)Xc.n);
    for (int32_t j = 0; j < k; ++j)
        if (init_ids_host[j] < 0 || init_ids_host[j] >= Xc.n)
            return fail(ctx, SIVF_E_RANGE, "init id %d at position %d outside [0, N)", init_ids_host[j], j);
    sivf_ivf* f = nullptr;
    STCHK(new_file(ctx, k, Xc.d, &f));
    f->nonneg = Xc.nonneg;
    sivf_status st = SIVF_OK;
    int32_t* ids = nullptr;
    int64_t *lens = nullptr, *scan = nullptr, *sws = nullptr;
    if (st == SIVF_OK) st = ws(ctx, "init_ids", k, &ids);
    if (st == SIVF_OK) st = ws(ctx, "init_lens", k, &lens);
    if (st == SIVF_OK) st = ws(ctx, "init_scan", k + 1, &scan);
    if (st == SIVF_OK) st = ws(ctx, "scan_ws", scan_ws_elems(k + 1) + 8, &sws);
    int64_t total = 0;
    auto H = [&](hipError_t e) {
        if (st == SIVF_OK && e != hipSuccess) st = fail(ctx, SIVF_E_HIP, "HIP error: %s", hipGetErrorString(e));
    };
    if (st == SIVF_OK) {
        H(hipMemcpyAsync(ids, init_ids_host, (size_t)k * 4, hipMemcpyHostToDevice, ctx->stream));
        H(gather_rows(Xc, ids, k, f->cur, lens, ctx->stream, 0));
        H(exclusive_scan_i64(lens, scan, k, sws, ctx->stream));
        H(hipMemcpyAsync(&total, scan + k, 8, hipMemcpyDeviceToHost, ctx->stream));
        H(hipStreamSynchronize(ctx->stream));
    }
    if (st == SIVF_OK) st = store_reserve(ctx, f, &f->cur, total);
    if (st == SIVF_OK) {
        H(hipMemcpyAsync(f->cur.start, scan, (size_t)k * 8, hipMemcpyDeviceToDevice, ctx->stream));
        H(gather_rows(Xc, ids, k, f->cur, lens, ctx->stream, 1));
        H(fill_u8(f->lam, 0, k, ctx->stream));
    }
    if (st == SIVF_OK) st = restructure(ctx, f);
    if (st == SIVF_OK) H(hipStreamSynchronize(ctx->stream));
    if (st != SIVF_OK) {
        free_file(ctx, f);
        return st;
    }
    *out = f;
    return SIVF_OK;
}

// lambda: device flags (NULL = all moving), copied into the file
sivf_status build_impl(sivf_ctx* ctx, const sivf_csr* C, const uint8_t* lambda, sivf_ivf** out) {
    STCHK(check_csr_args(ctx, C, "centroids"));
    if (C->val_dtype != SIVF_F64) return fail(ctx, SIVF_E_INVALID, "centroid values must be SIVF_F64");
    if (C->n_rows < 1 || C->n_rows > INT32_MAX) return fail(ctx, SIVF_E_SHAPE, "need 1 <= k <= 2^31-1");
    unsigned long long* flags = nullptr;
    STCHK(ws(ctx, "vflags", 4, &flags));
    unsigned long long init[3] = {0ull, ~0ull, 0ull};
    HIPCHK(ctx, hipMemcpyAsync(flags, init, sizeof(init), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, validate_csr(C->row_ptr, C->col, C->val, 1, C->n_rows, C->n_cols, C->nnz, flags, ctx->stream));
    unsigned long long h[3];
    HIPCHK(ctx, hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (h[0] & 9ull) return fail(ctx, SIVF_E_UNSORTED, "centroids: row %llu unsorted or bad row_ptr", h[1]);
    if (h[0] & 2ull) return fail(ctx, SIVF_E_RANGE, "centroids: column out of range in row %llu", h[1]);
    if (h[0] & 4ull) return fail(ctx, SIVF_E_NONFINITE, "centroids: non-finite value in row %llu", h[1]);
    const int32_t k = (int32_t)C->n_rows;
    sivf_ivf* f = nullptr;
    STCHK(new_file(ctx, k, C->n_cols, &f));
    f->nonneg = h[2] ? 0 : 1;
    sivf_status st = store_reserve(ctx, f, &f->cur, C->nnz);
    if (st == SIVF_OK) {
        hipError_t e = csr_to_store(C->row_ptr, C->col, (const double*)C->val, k, f->cur, ctx->stream);
        if (e == hipSuccess)
            e = lambda ? hipMemcpyAsync(f->lam, lambda, (size_t)k, hipMemcpyDeviceToDevice, ctx->stream)
                       : fill_u8(f->lam, 0, k, ctx->stream);
        if (e != hipSuccess) st = fail(ctx, SIVF_E_HIP, "HIP error: %s", hipGetErrorString(e));
    }
    if (st == SIVF_OK) st = restructure(ctx, f);
    if (st == SIVF_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(ctx, SIVF_E_HIP, "sync failed");
    if (st != SIVF_OK) {
        free_file(ctx, f);
        return st;
    }
    *out = f;
    return SIVF_OK;
}

// The assignment step's workspace (everything it reads or writes besides
// its inputs, outputs and the file).
struct AssignBufs {
    unsigned long long* counters = nullptr;
    int32_t *a_new = nullptr, *qobj = nullptr, *qcand = nullptr, *qcnt = nullptr, *fobj = nullptr;
    float* own_new = nullptr;
    uint8_t* changed = nullptr;
    double *obj_partial = nullptr, *obj = nullptr, *obj64_partial = nullptr;
    double *st_theta = nullptr, *st_best = nullptr, *own64_cur = nullptr;
    int32_t *st_bj = nullptr, *st_cnt = nullptr, *st_cj = nullptr, *own64_queue = nullptr;
    float* st_cr = nullptr;
    uint8_t* st_rel = nullptr;
    int64_t qcap = 0;
    int nfin = 0, launches = 0, tpl = 0, nobj = 0;
};

sivf_status assign_buffers(sivf_ctx* ctx, Work& w, int64_t n, int32_t k, int32_t T, AssignBufs* b) {
    const int relaxed = ctx->opt.filter_mode == SIVF_MODE_RELAXED;
    b->qcap = std::max<int64_t>(1024, n / 4);
    b->nfin = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 4095) / 4096));
    b->tpl = std::min<int>(T, std::max<int>(1, ctx->opt.tiles_per_launch));
    b->launches = (T + b->tpl - 1) / b->tpl;
    b->nobj = ctx->n_cu * 16;   // workgroups of the exact objective (fixed: a fixed summation order)
    STCHK(w.get("counters", 16 + b->launches, &b->counters));
    STCHK(w.get("a_new", n, &b->a_new));
    STCHK(w.get("own_new", n, &b->own_new));
    STCHK(w.get("qobj", b->qcap, &b->qobj));
    STCHK(w.get("qcand", b->qcap * kCandCap, &b->qcand));
    STCHK(w.get("qcnt", b->qcap, &b->qcnt));
    STCHK(w.get("fobj", std::max<int64_t>(n, 1), &b->fobj));
    STCHK(w.get("changed", k, &b->changed));
    STCHK(w.get("obj_partial", b->nfin + 1, &b->obj_partial));
    STCHK(w.get("objective", 2, &b->obj));
    if (ctx->opt.exact_objective) STCHK(w.get("obj64_partial", b->nobj, &b->obj64_partial));
    const int64_t m = std::max<int64_t>(n, 1);
    if (b->launches > 1) {
        STCHK(w.get("st_theta", m, &b->st_theta));
        STCHK(w.get("st_best", m, &b->st_best));
        STCHK(w.get("st_bj", m, &b->st_bj));
        STCHK(w.get("st_cnt", m, &b->st_cnt));
        STCHK(w.get("st_cj", m * kCandCap, &b->st_cj));
        STCHK(w.get("st_cr", m * kCandCap, &b->st_cr));
    }
    if (relaxed) {
        STCHK(w.get("own64_cur", m, &b->own64_cur));
        STCHK(w.get("own64_queue", m, &b->own64_queue));
        if (b->launches > 1) STCHK(w.get("st_rel", m, &b->st_rel));
    }
    return SIVF_OK;
}

// Assignment step r = iter (Alg. 4) of X against the file f.
sivf_status assign_impl(sivf_ctx* ctx, Work& w, const Csr& Xc, const sivf_ivf* f, int32_t iter, int32_t* assign_inout,
                        float* own_sim_inout, double* own64_inout, uint8_t* lambda_out, sivf_iter_stats* stats_host) {
    if (Xc.d != f->d) return fail(ctx, SIVF_E_SHAPE, "X has %lld columns, centroids %lld", (long long)Xc.d, (long long)f->d);
    const int64_t n = Xc.n;
    const int32_t k = f->k;
    const int relaxed = ctx->opt.filter_mode == SIVF_MODE_RELAXED;
    const int icp_on = iter >= 2 && ctx->opt.filter_mode != SIVF_MODE_IVF;
    if (iter >= 2) STCHK(check_assign(ctx, assign_inout, n, k, "assign_inout (a^[r-1])", w));
    AssignBufs B;
    STCHK(assign_buffers(ctx, w, n, k, f->T, &B));
    const int64_t qcap = B.qcap;
    unsigned long long* counters = B.counters;
    int32_t *a_new = B.a_new, *qobj = B.qobj, *qcand = B.qcand, *qcnt = B.qcnt, *fobj = B.fobj;
    float* own_new = B.own_new;
    uint8_t* changed = B.changed;
    double *obj_partial = B.obj_partial, *obj = B.obj;
    const int nfin = B.nfin, tpl = B.tpl, launches = B.launches, nobj = B.nobj;
    double* obj64_partial = B.obj64_partial;

    WalkArgs A{};
    A.n = n;
    A.rp = Xc.rp;
    A.col = Xc.col;
    A.xval = Xc.val;
    A.x_f64 = Xc.f64;
    A.k = k;
    A.kt = f->kt;
    A.T = f->T;
    A.seg = f->seg;
    A.mid = f->mid;
    A.rec = f->rec;
    A.d = f->d;
    A.perm = f->perm;
    A.nmv = f->nmv;
    A.cid = f->cid;
    A.pval = f->pdt == SIVF_BF16 ? (const void*)f->v16 : (const void*)f->v32;
    A.lam = f->lam;
    A.cnorm = f->cnorm;
    A.a_prev = assign_inout;
    A.own_prev = own_sim_inout;
    A.icp_on = icp_on;
    A.cbicp = ctx->opt.filter_mode == SIVF_MODE_CBICP;
    A.nonneg = Xc.nonneg && f->nonneg;
    A.certify = ctx->opt.certify;
    A.eta_val = f->pdt == SIVF_BF16 ? (0x1p-8 + 0x1p-24 + 0x1p-32) : 0x1p-24;
    A.eta_x = Xc.f64 ? 0x1p-24 : 0.0;
    A.a_new = a_new;
    A.own_new = own_new;
    A.qobj = qobj;
    A.qcand = qcand;
    A.qcnt = qcnt;
    A.fobj = fobj;
    A.counters = counters;
    A.qcap = qcap;
    A.st_theta = B.st_theta;
    A.st_best = B.st_best;
    A.st_bj = B.st_bj;
    A.st_cnt = B.st_cnt;
    A.st_cj = B.st_cj;
    A.st_cr = B.st_cr;
    A.st = f->cur;
    A.relaxed = relaxed;
    A.own64_prev = own64_inout;
    A.own64_cur = B.own64_cur;
    A.st_rel = B.st_rel;
    int32_t* own64_queue = B.own64_queue;
    A.head = f->H > 0 ? f->head : nullptr;
    A.hval = f->hval;
    A.kpad = (int64_t)f->T * head_ktp(f->kt);

    hipStream_t s = ctx->stream;
    HIPCHK(ctx, fill_u64(counters, 0ull, 16 + launches, s));
    HIPCHK(ctx, fill_u8(changed, 0, k, s));
    HIPCHK(ctx, hipEventRecord(ctx->ev[0], s));
    if (n > 0) {
        const int bpc = walk_blocks_per_cu(f->kt, f->pdt == SIVF_BF16, A.cbicp);
        for (int l = 0; l < launches; ++l)
            HIPCHK(ctx, walk_fast(A, f->pdt == SIVF_BF16, ctx->n_cu * bpc * kWalkWaves, l * tpl,
                                  std::min(f->T, (l + 1) * tpl), counters + 16 + l, s));
    }
    HIPCHK(ctx, hipEventRecord(ctx->ev[1], s));
    if (n > 0) {
        HIPCHK(ctx, rescore_candidates(A, f->cur, (int64_t)ctx->n_cu * 16, s));
        HIPCHK(ctx, rescore_full(A, f->v64, f->cur, (int64_t)ctx->n_cu * 4, s));
        if (relaxed) HIPCHK(ctx, own64_update(A, own64_inout, own64_queue, (int64_t)ctx->n_cu * 16, s));
        HIPCHK(ctx, finalize_assign(n, iter, a_new, own_new, assign_inout, own_sim_inout, changed, counters,
                                    obj_partial, nfin, s));
    }
    HIPCHK(ctx, finalize_lambda(k, iter, changed, lambda_out, counters, obj_partial, n > 0 ? nfin : 0, obj, s));
    HIPCHK(ctx, hipEventRecord(ctx->ev[2], s));
    // the FP64 objective of the new assignment against the centroids it was
    // made with, F(a^[r], mu^[r-1]) (opt-in; outside the step's timing)
    if (ctx->opt.exact_objective)
        HIPCHK(ctx, objective64(A, f->cur, assign_inout, obj64_partial, nobj, obj + 1, s));
    if (stats_host) {
        unsigned long long c[12];
        double o[2] = {0.0, 0.0};
        HIPCHK(ctx, hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipMemcpyAsync(o, obj, sizeof(o), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        memset(stats_host, 0, sizeof(*stats_host));
        stats_host->iter = iter;
        stats_host->multadds = (int64_t)c[0];
        stats_host->rescored_objects = (int64_t)std::min<unsigned long long>(c[1], (unsigned long long)qcap);
        stats_host->full_rescored = (int64_t)c[2];
        stats_host->icp_objects = (int64_t)c[3];
        stats_host->rescored_candidates = (int64_t)c[4];
        stats_host->moved = (int64_t)c[5];
        stats_host->n_invariant = (int32_t)c[6];
        stats_host->objective_fast = o[0];
        stats_host->objective = ctx->opt.exact_objective ? o[1] : NAN;
        stats_host->head_rows = f->H;
        stats_host->relaxed_objects = (int64_t)c[7];
        stats_host->walk_bytes = (int64_t)c[10];
        stats_host->walk_wide_bytes = (int64_t)c[11];
        stats_host->walk_launches = launches;
        float t = 0.0f;
        HIPCHK(ctx, hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
        stats_host->t_walk_ms = t;
        HIPCHK(ctx, hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[2]));
        stats_host->t_assign_ms = t;
    }
    return SIVF_OK;
}

// Update step (Alg. 5): centroids from assign, file restructured by lambda.
sivf_status update_impl(sivf_ctx* ctx, const Csr& Xc, const int32_t* assign, const uint8_t* lambda, sivf_ivf* f,
                        sivf_iter_stats* stats_host) {
    if (Xc.d != f->d) return fail(ctx, SIVF_E_SHAPE, "X has %lld columns, centroids %lld", (long long)Xc.d, (long long)f->d);
    const int64_t n = Xc.n;
    const int32_t k = f->k;
    hipStream_t s = ctx->stream;
    UpdateWs w{};
    w.nblk = std::max<int64_t>(1, (n + kObjBlock - 1) / kObjBlock);
    w.nslots = ctx->n_cu * 8;
    STCHK(ws(ctx, "u_hist", w.nblk * (int64_t)k, &w.hist));
    STCHK(ws(ctx, "u_ccount", k, &w.ccount));
    STCHK(ws(ctx, "u_cstart", k + 1, &w.cstart));
    STCHK(ws(ctx, "u_perm", std::max<int64_t>(n, 1), &w.perm));
    STCHK(ws(ctx, "u_memnnz", k, &w.memnnz));
    STCHK(ws(ctx, "u_ub", k, &w.ub));
    STCHK(ws(ctx, "u_ubscan", k + 1, &w.ubscan));
    STCHK(ws(ctx, "u_work", 1, &w.work));
    STCHK(ws(ctx, "scan_ws", scan_ws_elems(std::max<int64_t>(std::max<int64_t>(k, f->d * f->T * 2) + 1, n + 1)) + 8,
             &w.scan_ws));
    {
        // the dense accumulators must start zeroed; the kernel keeps them zero
        auto it = ctx->ws.find("u_W");
        const size_t need = (size_t)w.nslots * (size_t)Xc.d * sizeof(double);
        bool fresh = it == ctx->ws.end() || it->second.second < need;
        STCHK(ws(ctx, "u_W", (int64_t)w.nslots * Xc.d, &w.W));
        if (fresh) HIPCHK(ctx, fill_f64(w.W, 0.0, (int64_t)w.nslots * Xc.d, s));
    }
    STCHK(check_assign(ctx, assign, n, k, "assign"));
    HIPCHK(ctx, hipEventRecord(ctx->ev[3], s));
    HIPCHK(ctx, upd_sort(assign, n, k, Xc.rp, w, s));
    HIPCHK(ctx, upd_bounds(k, Xc.d, lambda, 1, f->cur, w, s));
    int64_t total = 0;
    HIPCHK(ctx, hipMemcpyAsync(&total, w.ubscan + k, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    STCHK(store_reserve(ctx, f, &f->nxt, total));
    HIPCHK(ctx, upd_segsum(Xc, k, lambda, 1, f->cur, f->nxt, w, s));
    std::swap(f->cur, f->nxt);
    HIPCHK(ctx, hipMemcpyAsync(f->lam, lambda, (size_t)k, hipMemcpyDeviceToDevice, s));
    f->nonneg = f->nonneg && Xc.nonneg;
    STCHK(restructure(ctx, f));
    HIPCHK(ctx, hipEventRecord(ctx->ev[4], s));
    if (stats_host) {
        HIPCHK(ctx, hipStreamSynchronize(s));
        float t = 0.0f;
        HIPCHK(ctx, hipEventElapsedTime(&t, ctx->ev[3], ctx->ev[4]));
        stats_host->t_update_ms = t;
    }
    return SIVF_OK;
}

}  // namespace

// =========================================================================== ABI
extern "C" {

sivf_status sivf_default_options(sivf_options* opt) {
    if (!opt) return SIVF_E_INVALID;
    opt->posting_dtype = SIVF_F32;
    opt->filter_mode = SIVF_MODE_SIVF;
    opt->k_tile = 0;
    opt->certify = 1;
    opt->workspace_cap_bytes = 0;
    opt->head_density = -1.0f;
    opt->tiles_per_launch = 0;
    opt->exact_objective = 0;
    return SIVF_OK;
}

sivf_status sivf_create(sivf_ctx** out, int device, void* hip_stream, const sivf_options* opt) {
    if (!out) return SIVF_E_INVALID;
    *out = nullptr;
    sivf_options o;
    sivf_default_options(&o);
    if (opt) o = *opt;
    if (o.posting_dtype != SIVF_F32 && o.posting_dtype != SIVF_BF16) return SIVF_E_INVALID;
    if (o.filter_mode < 0 || o.filter_mode > 3) return SIVF_E_INVALID;
    if (o.k_tile != 0 && (o.k_tile < 64 || o.k_tile > kMaxTile || o.k_tile % 64 != 0)) return SIVF_E_INVALID;
    if (!(o.head_density <= 1.0f)) return SIVF_E_INVALID;   // NaN fails too
    // negative: the precision's own density (dense rows cost half the bytes
    // in BF16, so more terms pay for one there)
    if (o.head_density < 0.0f) o.head_density = o.posting_dtype == SIVF_BF16 ? 0.3f : 0.5f;
    if (o.tiles_per_launch < 0) return SIVF_E_INVALID;
    if (o.exact_objective != 0 && o.exact_objective != 1) return SIVF_E_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SIVF_E_HIP;
    sivf_ctx* ctx = new (std::nothrow) sivf_ctx();
    if (!ctx) return SIVF_E_NOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->opt = o;
    DevGuard g(device);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        ctx->n_cu = ncu;
    if (scratch_setup(device) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return SIVF_E_HIP;
    }
    for (auto& e : ctx->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            delete ctx;
            return SIVF_E_HIP;
        }
    }
    *out = ctx;
    return SIVF_OK;
}

sivf_status sivf_destroy(sivf_ctx* ctx) {
    if (!ctx) return SIVF_OK;
    DevGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->ws) (void)hipFree(kv.second.first);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
    return SIVF_OK;
}

const char* sivf_last_error(const sivf_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

sivf_status sivf_validate_csr(sivf_ctx* ctx, const sivf_csr* X) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    Csr c;
    return validate(ctx, X, &c);
}

sivf_status sivf_init_centroids(sivf_ctx* ctx, const sivf_csr* X, int32_t k, const int32_t* init_ids_host,
                                sivf_ivf** out) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if (!out || !init_ids_host) return fail(ctx, SIVF_E_INVALID, "NULL argument");
    Csr Xc;
    STCHK(validate(ctx, X, &Xc));
    return init_impl(ctx, Xc, k, init_ids_host, out);
}

sivf_status sivf_build_centroid_ivf(sivf_ctx* ctx, const sivf_csr* C, const uint8_t* lambda, sivf_ivf** out) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if (!out) return fail(ctx, SIVF_E_INVALID, "NULL out");
    return build_impl(ctx, C, lambda, out);
}

sivf_status sivf_ivf_free(sivf_ctx* ctx, sivf_ivf* ivf) {
    if (!ivf) return SIVF_OK;
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    free_file(ctx, ivf);
    return SIVF_OK;
}

sivf_status sivf_ivf_sizes(sivf_ctx* ctx, const sivf_ivf* f, int32_t* k_host, int64_t* d_host, int64_t* nnz_host,
                           int32_t* n_tiles_host, int32_t* k_tile_host) {
    if (!ctx || !f) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (k_host) *k_host = f->k;
    if (d_host) *d_host = f->d;
    if (nnz_host) *nnz_host = f->P;
    if (n_tiles_host) *n_tiles_host = f->T;
    if (k_tile_host) *k_tile_host = f->kt;
    return SIVF_OK;
}

sivf_status sivf_ivf_export(sivf_ctx* ctx, const sivf_ivf* f, int64_t* c_ptr, int32_t* c_col, double* c_val,
                            uint8_t* lambda, int64_t* term_ptr, int32_t* split, int32_t* p_cid, double* p_val) {
    if (!ctx || !f) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if ((c_col || c_val) && !c_ptr) return fail(ctx, SIVF_E_INVALID, "c_col/c_val need c_ptr");
    if ((p_cid || p_val) && !term_ptr) return fail(ctx, SIVF_E_INVALID, "p_cid/p_val need term_ptr");
    int64_t* sws = nullptr;
    STCHK(ws(ctx, "scan_ws", scan_ws_elems(std::max<int64_t>(f->k, f->d) + 1) + 8, &sws));
    if (c_ptr) {
        HIPCHK(ctx, exclusive_scan_i64(f->cur.nnz, c_ptr, f->k, sws, ctx->stream));
        if (c_col || c_val) HIPCHK(ctx, store_export(f->cur, f->k, c_ptr, c_col, c_val, ctx->stream));
    }
    if (lambda) HIPCHK(ctx, hipMemcpyAsync(lambda, f->lam, (size_t)f->k, hipMemcpyDeviceToDevice, ctx->stream));
    if (term_ptr || split) {
        int64_t* cnt = nullptr;
        STCHK(ws(ctx, "exp_cnt", f->d, &cnt));
        HIPCHK(ctx, ivf_export(f, term_ptr, split, p_cid, p_val, cnt, sws, ctx->stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SIVF_OK;
}

sivf_status sivf_assign(sivf_ctx* ctx, const sivf_csr* X, const sivf_ivf* f, int32_t iter, int32_t* assign_inout,
                        float* own_sim_inout, double* own64_inout, uint8_t* lambda_out, sivf_iter_stats* stats_host) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if (!f || !assign_inout || !own_sim_inout || !lambda_out) return fail(ctx, SIVF_E_INVALID, "NULL argument");
    if (ctx->opt.filter_mode == SIVF_MODE_RELAXED && !own64_inout)
        return fail(ctx, SIVF_E_INVALID, "the RELAXED filter needs own64_inout");
    if (iter < 1) return fail(ctx, SIVF_E_INVALID, "iter must be >= 1");
    Csr Xc;
    STCHK(validate(ctx, X, &Xc));
    Work w{ctx};
    return assign_impl(ctx, w, Xc, f, iter, assign_inout, own_sim_inout, own64_inout, lambda_out, stats_host);
}

sivf_status sivf_assign_noalloc(sivf_ctx* ctx, const sivf_csr* X, const sivf_ivf* f, int32_t iter,
                                int32_t* assign_inout, float* own_sim_inout, double* own64_inout,
                                uint8_t* lambda_out, sivf_iter_stats* stats_host) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if (!f || !assign_inout || !own_sim_inout || !lambda_out) return fail(ctx, SIVF_E_INVALID, "NULL argument");
    if (ctx->opt.filter_mode == SIVF_MODE_RELAXED && !own64_inout)
        return fail(ctx, SIVF_E_INVALID, "the RELAXED filter needs own64_inout");
    if (iter < 1) return fail(ctx, SIVF_E_INVALID, "iter must be >= 1");
    STCHK(check_csr_args(ctx, X, "X"));
    // the same requests as the run below, counted without memory
    Work m{ctx, Work::kMeasure};
    unsigned long long* flags = nullptr;
    STCHK(m.get("vflags", 4, &flags));
    if (iter >= 2) STCHK(m.get("aflags", 2, &flags));
    AssignBufs B;
    STCHK(assign_buffers(ctx, m, X->n_rows, f->k, f->T, &B));
    if (m.used > kScratchBytes)
        return fail(ctx, SIVF_E_UNSUPPORTED,
                    "sivf_assign_noalloc: %lld objects against %d centroids (%d launches) need %zu bytes of "
                    "scratch, above its %zu; use sivf_assign", (long long)X->n_rows, f->k, B.launches, m.used,
                    kScratchBytes);
    void* base = scratch_of(ctx->device);
    if (!base) return fail(ctx, SIVF_E_HIP, "no scratch address for device %d", ctx->device);
    Work w{ctx, Work::kFixed, (char*)base, kScratchBytes};
    Csr Xc;
    STCHK(validate(ctx, X, &Xc, w));
    return assign_impl(ctx, w, Xc, f, iter, assign_inout, own_sim_inout, own64_inout, lambda_out, stats_host);
}

sivf_status sivf_update(sivf_ctx* ctx, const sivf_csr* X, const int32_t* assign, const uint8_t* lambda,
                        sivf_ivf* f, sivf_iter_stats* stats_host) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if (!f || !assign || !lambda) return fail(ctx, SIVF_E_INVALID, "NULL argument");
    Csr Xc;
    STCHK(validate(ctx, X, &Xc));
    return update_impl(ctx, Xc, assign, lambda, f, stats_host);
}

sivf_status sivf_run_lloyd(sivf_ctx* ctx, const sivf_csr* X, int32_t k, const int32_t* init_ids_host, int32_t max_iter,
                           int32_t* assign_out, float* own_sim_out, sivf_ivf** centroids_out,
                           sivf_iter_stats* per_iter_host, int32_t* iters_done_host) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if (max_iter < 1) return fail(ctx, SIVF_E_INVALID, "max_iter must be >= 1");
    if (!init_ids_host) return fail(ctx, SIVF_E_INVALID, "NULL argument");
    // X is validated once: the driver holds the stream for the whole run
    Csr Xc;
    STCHK(validate(ctx, X, &Xc));
    sivf_ivf* f = nullptr;
    STCHK(init_impl(ctx, Xc, k, init_ids_host, &f));
    int32_t* a = assign_out;
    float* own = own_sim_out;
    uint8_t* lam = nullptr;
    sivf_status st = SIVF_OK;
    if (!a) st = ws(ctx, "lloyd_a", Xc.n, &a);
    if (st == SIVF_OK && !own) st = ws(ctx, "lloyd_own", Xc.n, &own);
    if (st == SIVF_OK) st = ws(ctx, "lloyd_lam", k, &lam);
    double* own64 = nullptr;   // exact own similarities (relaxed ICP state)
    if (st == SIVF_OK && ctx->opt.filter_mode == SIVF_MODE_RELAXED)
        st = ws(ctx, "lloyd_own64", std::max<int64_t>(Xc.n, 1), &own64);
    int32_t done = 0;
    for (int32_t r = 1; st == SIVF_OK && r <= max_iter; ++r) {
        sivf_iter_stats stt{};
        Work w{ctx};
        st = assign_impl(ctx, w, Xc, f, r, a, own, own64, lam, &stt);
        if (st != SIVF_OK) break;
        done = r;
        if (per_iter_host) per_iter_host[r - 1] = stt;
        if (r >= 2 && stt.moved == 0) break;
        if (r == max_iter) break;  // the last assignment's centroids stay as they are
        st = update_impl(ctx, Xc, a, lam, f, &stt);
        if (st != SIVF_OK) break;
        if (per_iter_host) per_iter_host[r - 1].t_update_ms = stt.t_update_ms;
    }
    if (st == SIVF_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(ctx, SIVF_E_HIP, "sync failed");
    if (iters_done_host) *iters_done_host = done;
    if (st != SIVF_OK || !centroids_out) {
        free_file(ctx, f);
        if (centroids_out) *centroids_out = nullptr;
        return st;
    }
    *centroids_out = f;
    return SIVF_OK;
}

sivf_status sivf_resume(sivf_ctx* ctx, const sivf_csr* X, const sivf_csr* centroids, const int32_t* a_prev,
                        const int32_t* a_prev2, sivf_ivf** out, float* own_sim_out, double* own64_out) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if (!out || !a_prev || !own_sim_out || !centroids) return fail(ctx, SIVF_E_INVALID, "NULL argument");
    if (ctx->opt.filter_mode == SIVF_MODE_RELAXED && !own64_out)
        return fail(ctx, SIVF_E_INVALID, "the RELAXED filter needs own64_out");
    Csr Xc;
    STCHK(validate(ctx, X, &Xc));
    if (centroids->n_cols != Xc.d)
        return fail(ctx, SIVF_E_SHAPE, "X has %lld columns, centroids %lld", (long long)Xc.d,
                    (long long)centroids->n_cols);
    if (centroids->n_rows < 1 || centroids->n_rows > Xc.n)
        return fail(ctx, SIVF_E_SHAPE, "need 1 <= k <= N (k=%lld, N=%lld)", (long long)centroids->n_rows,
                    (long long)Xc.n);
    const int32_t k = (int32_t)centroids->n_rows;
    STCHK(check_assign(ctx, a_prev, Xc.n, k, "a_prev"));
    if (a_prev2) STCHK(check_assign(ctx, a_prev2, Xc.n, k, "a_prev2"));
    // lambda of the restart point: membership of every cluster unchanged
    // between the last two assignments (all 0 when only one exists)
    uint8_t *changed = nullptr, *lam = nullptr;
    unsigned long long* cnt = nullptr;
    double* dummy = nullptr;
    STCHK(ws(ctx, "resume_changed", k, &changed));
    STCHK(ws(ctx, "resume_lam", k, &lam));
    STCHK(ws(ctx, "resume_cnt", 16, &cnt));
    STCHK(ws(ctx, "resume_obj", 1, &dummy));
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, fill_u8(changed, 0, k, s));
    HIPCHK(ctx, fill_u64(cnt, 0ull, 16, s));
    if (a_prev2 && Xc.n > 0) HIPCHK(ctx, mark_changed(Xc.n, a_prev2, a_prev, changed, s));
    HIPCHK(ctx, finalize_lambda(k, a_prev2 ? 2 : 1, changed, lam, cnt, nullptr, 0, dummy, s));
    sivf_ivf* f = nullptr;
    STCHK(build_impl(ctx, centroids, lam, &f));
    WalkArgs A{};
    A.n = Xc.n;
    A.rp = Xc.rp;
    A.col = Xc.col;
    A.xval = Xc.val;
    A.x_f64 = Xc.f64;
    if (Xc.n > 0) {
        hipError_t e = resume_own(A, f->cur, a_prev, f->lam, own_sim_out, own64_out, (int64_t)ctx->n_cu * 16, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            free_file(ctx, f);
            return fail(ctx, SIVF_E_HIP, "HIP error: %s", hipGetErrorString(e));
        }
    }
    *out = f;
    return SIVF_OK;
}

sivf_status sivf_soft_assign_fwd(sivf_ctx* ctx, const sivf_csr* X, const float* C, int32_t k, float tau, float* lse_out,
                                 double* loss_host) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if (!C || !lse_out) return fail(ctx, SIVF_E_INVALID, "NULL argument");
    if (k < 1) return fail(ctx, SIVF_E_SHAPE, "k must be >= 1");
    if (!(tau > 0.0f) || !std::isfinite(tau)) return fail(ctx, SIVF_E_INVALID, "tau must be positive and finite");
    Csr Xc;
    STCHK(validate(ctx, X, &Xc));
    if (Xc.f64) return fail(ctx, SIVF_E_UNSUPPORTED, "soft assignment takes SIVF_F32 object values");
    float *CT = nullptr, *pmax = nullptr, *psum = nullptr;
    double* loss = nullptr;
    STCHK(ws(ctx, "soft_CT", (int64_t)k * Xc.d, &CT));
    STCHK(ws(ctx, "soft_loss", 1, &loss));
    STCHK(ws(ctx, "soft_pmax", std::max<int64_t>(Xc.n, 1) * 8, &pmax));
    STCHK(ws(ctx, "soft_psum", std::max<int64_t>(Xc.n, 1) * 8, &psum));
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, soft_transpose(C, CT, k, Xc.d, s));
    HIPCHK(ctx, soft_forward(Xc.n, Xc.rp, Xc.col, (const float*)Xc.val, CT, k, tau, lse_out, loss, pmax, psum,
                             ctx->n_cu, s));
    if (loss_host) {
        HIPCHK(ctx, hipMemcpyAsync(loss_host, loss, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
    }
    return SIVF_OK;
}

sivf_status sivf_soft_assign_bwd(sivf_ctx* ctx, const sivf_csr* X, const float* C, int32_t k, float tau, const float* lse,
                                 float grad_loss, float* dC_out, float* dxval_out) {
    if (!ctx) return SIVF_E_INVALID;
    DevGuard g(ctx->device);
    if (!C || !lse) return fail(ctx, SIVF_E_INVALID, "NULL argument");
    if (k < 1) return fail(ctx, SIVF_E_SHAPE, "k must be >= 1");
    if (!(tau > 0.0f) || !std::isfinite(tau)) return fail(ctx, SIVF_E_INVALID, "tau must be positive and finite");
    if (!std::isfinite(grad_loss)) return fail(ctx, SIVF_E_NONFINITE, "grad_loss must be finite");
    Csr Xc;
    STCHK(validate(ctx, X, &Xc));
    if (Xc.f64) return fail(ctx, SIVF_E_UNSUPPORTED, "soft assignment takes SIVF_F32 object values");
    if (!dC_out && !dxval_out) return SIVF_OK;
    const int64_t n = Xc.n, d = Xc.d;
    hipStream_t s = ctx->stream;
    float *CT = nullptr, *dS = nullptr, *dxv = dxval_out, *dCT = nullptr;
    STCHK(ws(ctx, "soft_CT", (int64_t)k * d, &CT));
    // rows per chunk: dS of one chunk is at most 256 MiB
    const int64_t rc = std::max<int64_t>(1, std::min<int64_t>(std::max<int64_t>(n, 1), (int64_t)(64ll << 20) / k));
    STCHK(ws(ctx, "soft_dS", rc * (int64_t)k, &dS));
    if (!dxv) STCHK(ws(ctx, "soft_dx", std::max<int64_t>(Xc.nnz, 1), &dxv));
    HIPCHK(ctx, soft_transpose(C, CT, k, d, s));
    // nonzero offsets of the row chunks: they size the per-group dX partials
    // and bound the pieces of the dC pass
    const int64_t nch = std::max<int64_t>(1, (n + rc - 1) / rc);
    int64_t* offs = nullptr;
    STCHK(ws(ctx, "soft_offs", nch + 1, &offs));
    HIPCHK(ctx, soft_chunk_offsets(Xc.rp, n, rc, nch, offs, s));
    std::vector<int64_t> ho((size_t)nch + 1);
    HIPCHK(ctx, hipMemcpyAsync(ho.data(), offs, (size_t)(nch + 1) * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    int64_t nnz_max = 0;
    for (int64_t j = 0; j < nch; ++j) nnz_max = std::max(nnz_max, ho[(size_t)j + 1] - ho[(size_t)j]);
    float* dxp = nullptr;
    STCHK(ws(ctx, "soft_dxp", std::max<int64_t>(nnz_max, 1) * 8, &dxp));
    int64_t *cnt = nullptr, *colptr = nullptr, *sws = nullptr;
    int32_t *hist = nullptr, *xt_row = nullptr;
    float* xt_val = nullptr;
    DctWs dw{};
    if (dC_out) {
        const int64_t nb = (n + 1023) / 1024;
        STCHK(ws(ctx, "soft_dCT", (int64_t)k * d, &dCT));
        STCHK(ws(ctx, "csc_hist", std::max<int64_t>(nb * d, 1), &hist));
        STCHK(ws(ctx, "csc_cnt", d, &cnt));
        STCHK(ws(ctx, "csc_ptr", d + 1, &colptr));
        STCHK(ws(ctx, "csc_row", std::max<int64_t>(Xc.nnz, 1), &xt_row));
        STCHK(ws(ctx, "csc_val", std::max<int64_t>(Xc.nnz, 1), &xt_val));
        STCHK(ws(ctx, "scan_ws", scan_ws_elems(std::max<int64_t>(d + 1, n + 1)) + 8, &sws));
        HIPCHK(ctx, soft_csc(n, d, Xc.nnz, Xc.rp, Xc.col, (const float*)Xc.val, hist, cnt, colptr, sws, xt_row, xt_val, s));
        // ranges of at most 256 entries are summed whole; longer ones are cut
        // at row blocks: 512 rows for ranges of more than 2048 entries (hot
        // terms), 2048 rows for the rest (mid terms).  Every chunk's pieces
        // are counted first, and the partial rows are sized for the largest.
        dw.piece = 256;
        dw.hot_min = 2048;
        dw.blk_rows = 512;
        dw.mid_blk_rows = 2048;
        STCHK(ws(ctx, "dct_lo", d, &dw.lo));
        STCHK(ws(ctx, "dct_hi", d, &dw.hi));
        STCHK(ws(ctx, "dct_np", d, &dw.np));
        STCHK(ws(ctx, "dct_pstart", d + 1, &dw.pstart));
        STCHK(ws(ctx, "dct_hflag", d, &dw.hflag));
        STCHK(ws(ctx, "dct_hscan", d + 1, &dw.hscan));
        STCHK(ws(ctx, "dct_hot", d, &dw.hot));
        STCHK(ws(ctx, "dct_mflag", d, &dw.mflag));
        STCHK(ws(ctx, "dct_mscan", d + 1, &dw.mscan));
        STCHK(ws(ctx, "dct_mid", d, &dw.mid));
        dw.scan_ws = sws;
        int64_t* counts = nullptr;
        STCHK(ws(ctx, "dct_counts", nch, &counts));
        for (int64_t j = 0; j < nch; ++j)
            HIPCHK(ctx, soft_dct_count(d, std::min(n, j * rc), std::min(n, (j + 1) * rc), colptr, xt_row, dw,
                                       counts + j, s));
        std::vector<int64_t> hc((size_t)nch);
        HIPCHK(ctx, hipMemcpyAsync(hc.data(), counts, (size_t)nch * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        dw.max_pieces = 0;
        for (int64_t j = 0; j < nch; ++j) dw.max_pieces = std::max(dw.max_pieces, hc[(size_t)j]);
        STCHK(ws(ctx, "dct_item", std::max<int64_t>(dw.max_pieces, 1), &dw.item));
        STCHK(ws(ctx, "dct_part", std::max<int64_t>(dw.max_pieces, 1) * (int64_t)k, &dw.part));
    }
    int first = 1;
    for (int64_t c0 = 0, j = 0; c0 < n || first; c0 += rc, ++j) {
        const int64_t c1 = std::min(n, c0 + rc);
        if (c1 > c0)
            HIPCHK(ctx, soft_bwd_rows(c0, c1, ho[(size_t)j], ho[(size_t)j + 1], Xc.rp, Xc.col, (const float*)Xc.val, CT,
                                      k, tau, grad_loss, lse, dS, dxp, dxv, ctx->n_cu, s));
        if (dC_out) HIPCHK(ctx, soft_dct(d, k, c0, c1, first, colptr, xt_row, xt_val, dS, dCT, dw, ctx->n_cu, s));
        first = 0;
        if (c1 >= n) break;
    }
    if (dC_out) HIPCHK(ctx, soft_transpose(dCT, dC_out, d, k, s));
    return SIVF_OK;
}

}  // extern "C"
