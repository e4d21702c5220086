// Wavefront-level helpers for 64-lane CDNA waves.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sivf {

__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ inline int lanes_below(unsigned long long mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ inline unsigned long long ballot(bool p) { return __ballot(p); }

// Wave-uniform value of lane `l` (l must be wave-uniform).
__device__ inline int32_t bcast_i32(int32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline float bcast_f32(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline int64_t bcast_i64(int64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline double bcast_f64(double v, int l) {
    return __longlong_as_double(bcast_i64(__double_as_longlong(v), l));
}

// Wave-wide work grab: the whole wave executes the atomic (no lane-divergent
// region around it), only lane 0 contributes `amount`, and lane 0's old value
// is broadcast.  Every lane of the wave must call it.
__device__ inline int64_t wave_grab(unsigned long long* counter, unsigned long long amount) {
    const unsigned long long add = lane_id() == 0 ? amount : 0ull;
    const unsigned long long old = atomicAdd(counter, add);
    return bcast_i64((int64_t)old, 0);
}

__device__ inline int64_t wave_incl_scan_i64(int64_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

__device__ inline int32_t wave_incl_scan_i32(int32_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Butterfly sums: the same fixed association on every call, so results are
// run-to-run deterministic.  Every lane receives the total.
__device__ inline double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline int32_t wave_min_i32(int32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// bf16 storage <-> f32: the 16 high bits of an IEEE binary32.
__device__ __host__ inline float bf16_to_f32(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Round a finite binary32 to bf16, nearest-even (format definition: keep the
// top 16 bits, add half an ulp of bf16 plus the tie-to-even bit).
__device__ __host__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

}  // namespace sivf
