// Data-rate probes for the roofline the walk is measured against (built into
// libsivf_probe.so, separate from libsivf.so; bench.py --probe runs them).
//
// The walk is bound by the vector memory data path, not by HBM: its lists and
// dense rows are cache resident, so what limits it is how many bytes per
// clock a compute unit's vector loads can bring into registers.  These
// kernels measure that rate for buffer loads of 4, 8 and 16 bytes per lane
// from regions sized to live in the L1 cache, the L2 cache, the memory-side
// cache and HBM, and the LDS read and write rates, and read the shader clock
// (s_memtime) against the constant 100 MHz clock (s_memrealtime) so the
// rates can be given per clock per compute unit.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ inline uint32_t fold(uint32_t a, uint32_t b) { return a ^ (b + 0x9E3779B9u); }

// Each workgroup sweeps a window of `window` bytes starting at
// (blockIdx * stride) mod region (the buffer holds region + window bytes), 4
// loads per lane per round, consecutive lanes on consecutive addresses.  The
// XOR of everything loaded goes to sink only if it equals `never`, which
// keeps the loads without a store per round.
template <int W>
__global__ __launch_bounds__(256) void k_probe_load(const uint8_t* __restrict__ buf, uint32_t region, uint32_t window,
                                                    uint32_t stride, int rounds, uint32_t never,
                                                    uint32_t* __restrict__ sink, unsigned long long* __restrict__ clk) {
    const uint32_t start = (uint32_t)(((uint64_t)blockIdx.x * stride) % region);
    const __amdgpu_buffer_rsrc_t r = rsrc(buf + start, window);
    const uint32_t step = 256u * W * 4u;   // one round of the workgroup
    uint32_t acc = 0;
    unsigned long long t0 = 0, q0 = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        t0 = __builtin_amdgcn_s_memtime();
        q0 = __builtin_amdgcn_s_memrealtime();
    }
    uint32_t off = 0;
    for (int it = 0; it < rounds; ++it) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int o = (int)(threadIdx.x * W + u * 256 * W);
            if (W == 4) {
                acc = fold(acc, __builtin_amdgcn_raw_buffer_load_b32(r, o, (int)off, 0));
            } else if (W == 8) {
                const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, o, (int)off, 0);
                acc = fold(acc, v.x ^ v.y);
            } else {
                const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, o, (int)off, 0);
                acc = fold(acc, (v.x ^ v.y) ^ (v.z ^ v.w));
            }
        }
        off += step;
        if (off + step > window) off = 0;
    }
    if (acc == never) sink[threadIdx.x] = acc;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clk[0] = __builtin_amdgcn_s_memtime() - t0;
        clk[1] = __builtin_amdgcn_s_memrealtime() - q0;
    }
}

// LDS: every lane reads (or writes) 16 bytes per operation from a 32 KiB
// workgroup buffer, 8 operations per round, consecutive lanes on consecutive
// 16-byte entries (conflict free); the entries rotate by one group of 256
// per round, so a round's addresses differ from the previous round's.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_probe_lds(int rounds, uint32_t never, uint32_t* __restrict__ sink,
                                                   unsigned long long* __restrict__ clk) {
    __shared__ u32x4 lds[2048];
    for (int i = threadIdx.x; i < 2048; i += 256) lds[i] = (u32x4){(uint32_t)i, 1u, 2u, 3u};
    __syncthreads();
    unsigned long long t0 = 0, q0 = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        t0 = __builtin_amdgcn_s_memtime();
        q0 = __builtin_amdgcn_s_memrealtime();
    }
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (int it = 0; it < rounds; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = (threadIdx.x + (u + it) * 256) & 2047;
            if (WRITE) {
                lds[idx] = acc;
                acc.x += 1u;
            } else {
                const u32x4 v = lds[idx];
                acc.x ^= v.x;
                acc.y += v.y;
                acc.z ^= v.z;
                acc.w += v.w;
            }
        }
    }
    if (WRITE) __syncthreads();
    const uint32_t f = WRITE ? lds[(threadIdx.x * 7) & 2047].x : ((acc.x ^ acc.y) ^ (acc.z ^ acc.w));
    if (f == never) sink[threadIdx.x] = f;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clk[0] = __builtin_amdgcn_s_memtime() - t0;
        clk[1] = __builtin_amdgcn_s_memrealtime() - q0;
    }
}

}  // namespace

extern "C" {

// One probe launch on `stream`: kind 0 = vector loads of `width` bytes per
// lane (4, 8 or 16) over a region of `region` bytes of `buf` (each workgroup
// a `window`-byte window, consecutive workgroups `stride` bytes apart);
// kind 1 = LDS reads, kind 2 = LDS writes (16 bytes per lane).  blocks
// workgroups of 256 threads, `rounds` rounds of 4 loads (8 LDS operations)
// per lane.  buf must hold region + window bytes.
// Returns 0, or -1 on bad arguments, or the HIP error.  bytes_host: bytes
// moved; clk_host[0..1]: shader clocks and 100 MHz clocks of workgroup 0.
int sivf_probe_run(int kind, int width, const void* buf, uint32_t region, uint32_t window, uint32_t stride,
                   int blocks, int rounds, void* scratch, void* stream, double* bytes_host,
                   unsigned long long* clk_host) {
    if (blocks < 1 || rounds < 1 || !scratch) return -1;
    hipStream_t s = (hipStream_t)stream;
    uint32_t* sink = (uint32_t*)scratch;
    unsigned long long* clk = (unsigned long long*)((uint8_t*)scratch + 1024);
    const uint32_t never = 0x7F3A5C91u;
    if (kind == 0) {
        if (!buf || (width != 4 && width != 8 && width != 16)) return -1;
        const uint32_t step = 256u * (uint32_t)width * 4u;
        if (window < step || stride == 0) return -1;
        if (width == 4)
            hipLaunchKernelGGL(k_probe_load<4>, dim3(blocks), dim3(256), 0, s, (const uint8_t*)buf, region, window,
                               stride, rounds, never, sink, clk);
        else if (width == 8)
            hipLaunchKernelGGL(k_probe_load<8>, dim3(blocks), dim3(256), 0, s, (const uint8_t*)buf, region, window,
                               stride, rounds, never, sink, clk);
        else
            hipLaunchKernelGGL(k_probe_load<16>, dim3(blocks), dim3(256), 0, s, (const uint8_t*)buf, region, window,
                               stride, rounds, never, sink, clk);
        if (bytes_host) *bytes_host = (double)blocks * 256.0 * width * 4.0 * rounds;
    } else if (kind == 1 || kind == 2) {
        if (kind == 1)
            hipLaunchKernelGGL(k_probe_lds<false>, dim3(blocks), dim3(256), 0, s, rounds, never, sink, clk);
        else
            hipLaunchKernelGGL(k_probe_lds<true>, dim3(blocks), dim3(256), 0, s, rounds, never, sink, clk);
        if (bytes_host) *bytes_host = (double)blocks * 256.0 * 16.0 * 8.0 * rounds;
    } else {
        return -1;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    e = hipMemcpyAsync(clk_host, clk, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? 0 : (int)e;
}

}  // extern "C"
