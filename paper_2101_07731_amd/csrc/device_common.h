// Device-side helpers shared by the gfx950 kernels of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcdtw {

template <typename T> __device__ __forceinline__ T inf_v();
template <> __device__ __forceinline__ float inf_v<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_v<double>() { return __builtin_inf(); }

// DPP control codes (GFX9 family): whole-wave shift by one lane.
constexpr int kWaveShr1 = 0x138;  // lane l receives lane l-1
constexpr int kWaveShl1 = 0x130;  // lane l receives lane l+1
constexpr int kWaveRor1 = 0x13C;  // lane l receives lane l-1, lane 0 lane 63
constexpr int kWaveRol1 = 0x134;  // lane l receives lane l+1, lane 63 lane 0

__device__ __forceinline__ uint32_t wave_ror1(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kWaveRor1, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t wave_rol1(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kWaveRol1, 0xF, 0xF, false);
}
// Copies n elements from global memory to LDS with `nthreads` threads, eight
// loads in flight per thread (a loop of load-then-store waits for every
// load in turn).
template <typename T>
__device__ __forceinline__ void copy_to_lds(T* dst, const T* __restrict__ src, int64_t n, int tid, int nthreads) {
    int64_t t = tid;
    for (; t + 7 * (int64_t)nthreads < n; t += 8 * (int64_t)nthreads) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[t + u * (int64_t)nthreads];
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[t + u * (int64_t)nthreads] = v[u];
    }
    for (; t < n; t += nthreads) dst[t] = src[t];
}

// Directed roundings of a non-negative double to float.
__device__ __forceinline__ float round_down_f(double x) {
    float f = (float)x;
    if ((double)f > x) f = __uint_as_float(__float_as_uint(f) - 1u);   // x > 0
    return f;
}
__device__ __forceinline__ float round_up_pos(double x) {
    float f = (float)x;
    if ((double)f < x) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

// Minimum of non-negative floats (or +inf) through their bit patterns, which
// order like the values; no NaN handling is generated.
__device__ __forceinline__ uint32_t umin3(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t t = a < b ? a : b;
    return t < c ? t : c;
}

// Lanes without a source lane keep `old`.
__device__ __forceinline__ float wave_shr1(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, old), __builtin_bit_cast(int, v), kWaveShr1, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_shl1(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, old), __builtin_bit_cast(int, v), kWaveShl1, 0xF, 0xF, false));
}
__device__ __forceinline__ double wave_shr1(double old, double v) {
    int2 o = __builtin_bit_cast(int2, old), x = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_update_dpp(o.x, x.x, kWaveShr1, 0xF, 0xF, false);
    r.y = __builtin_amdgcn_update_dpp(o.y, x.y, kWaveShr1, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double wave_shl1(double old, double v) {
    int2 o = __builtin_bit_cast(int2, old), x = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_update_dpp(o.x, x.x, kWaveShl1, 0xF, 0xF, false);
    r.y = __builtin_amdgcn_update_dpp(o.y, x.y, kWaveShl1, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}

// Next work item of a persistent one-wave loop: lane 0 takes it from the
// counter and the value is read from lane 0 into a scalar register, so the
// item is wave-uniform by construction and every exit and skip of the loop
// that depends on it is a uniform branch.  (A shuffle broadcast leaves the
// value in a vector register; the compiler may then treat the loop exits as
// divergent and split the loop so that lanes 1..63 re-read the broadcast
// while lane 0 waits at the atomic, which never ends.)  Call with all 64
// lanes active.
__device__ __forceinline__ int wave_next_item(int* counter) {
    int v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(counter, 1);
    return __builtin_amdgcn_readlane(v, 0);
}

// A 64-bit value read from lane 0 into scalar registers.
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 0);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 0);
    return ((unsigned long long)hi << 32) | lo;
}

// A condition made wave-uniform from lane 0's value (for conditions that are
// equal in every lane but computed from vector registers).
__device__ __forceinline__ bool wave_uniform(bool c) { return __builtin_amdgcn_readlane((int)c, 0) != 0; }

__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }
template <typename T> __device__ __forceinline__ T vmin3(T a, T b, T c) { return vmin(vmin(a, b), c); }

// Squared Euclidean point cost over NCH chunks of 4 dimensions.  Padded
// dimensions hold 0 in both operands (or +-inf in sentinel points) and
// add nothing.  float: fused multiply-add chain.
template <int NCH>
__device__ __forceinline__ float point_cost(const float4 (&q)[NCH], const float4 (&c)[NCH], float) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        float d0 = q[k].x - c[k].x, d1 = q[k].y - c[k].y, d2 = q[k].z - c[k].z, d3 = q[k].w - c[k].w;
        acc = __builtin_fmaf(d0, d0, acc);
        acc = __builtin_fmaf(d1, d1, acc);
        acc = __builtin_fmaf(d2, d2, acc);
        acc = __builtin_fmaf(d3, d3, acc);
    }
    return acc;
}

// double: every difference, square and sum rounded separately, dimensions
// in increasing order (reproduces a plain FP64 evaluation exactly; the
// zero terms of padded dimensions leave the sum unchanged).
template <int NCH>
__device__ __forceinline__ double point_cost(const float4 (&q)[NCH], const float4 (&c)[NCH], double) {
#pragma clang fp contract(off)
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        double d;
        d = (double)q[k].x - (double)c[k].x; acc = acc + d * d;
        d = (double)q[k].y - (double)c[k].y; acc = acc + d * d;
        d = (double)q[k].z - (double)c[k].z; acc = acc + d * d;
        d = (double)q[k].w - (double)c[k].w; acc = acc + d * d;
    }
    return acc;
}

__device__ __forceinline__ float add_cost(float cost, float best) { return cost + best; }
__device__ __forceinline__ double add_cost(double cost, double best) {
#pragma clang fp contract(off)
    return cost + best;
}

}  // namespace tcdtw
