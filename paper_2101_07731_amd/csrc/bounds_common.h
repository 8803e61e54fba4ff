// Device helpers shared by the bound kernels (LB_PC, LB_TI).
#pragma once
#include "device_common.h"
#include "internal.h"

namespace tcdtw {

__device__ __forceinline__ float rdown(double x) {
    float f = (float)x;
    if ((double)f > x) f = __uint_as_float(__float_as_uint(f) - 1u);
    return f;
}

__device__ __forceinline__ float rup(double x) {
    float f = (float)x;
    if ((double)f < x) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

// max(a, b) of two values that are >= 0 (or +inf), on their bits: no NaN
// quieting of the operands is needed, so the shift of a DPP operand folds in.
__device__ __forceinline__ float umax_f(float a, float b) {
    return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}

// LB_TI's exact point distance from its sum of squares s, as a lower and an
// upper side: the hardware square root (taken as within 2 ulp) for both, except
// that sums below 2^-100 give 0 below and sqrt(2^-100) above, so that the
// instruction's handling of tiny inputs is never relied on.
__device__ __forceinline__ void ti_exact_sides(float s, float& lo, float& hi) {
    constexpr float kTiny = 0x1p-100f;
    hi = __builtin_amdgcn_sqrtf(__builtin_fmaxf(s, kTiny));
    lo = s < kTiny ? 0.0f : hi;
}

__device__ __forceinline__ uint32_t okey(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float okey_to_float(uint32_t k) {
    const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

__device__ __forceinline__ float key_bsf(const unsigned long long* key) {
    const unsigned long long k = __hip_atomic_load(key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __uint_as_float((uint32_t)(k >> 32));
}

// Lane l receives lane l+1's value, lane 63 lane 0's (every source lane is valid, so the
// bound-control bit changes nothing and lets the compiler fold the shift into the consumer).
__device__ __forceinline__ float wave_rol1_f(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), kWaveRol1, 0xF, 0xF, true));
}
// Lane l receives lane l+1's value, lane 63 receives `old`.
__device__ __forceinline__ uint32_t wave_shl1_u32(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, kWaveShl1, 0xF, 0xF, false);
}

// Persistent one-wave loops over many small work items (one pair each) take
// them in batches of B consecutive items, one atomic per batch: thousands of
// waves taking single items from one counter serialise on it.  About `per`
// batches per wave keep the end balanced.
__device__ __forceinline__ int item_batch(int total, int per) {
    return max(1, min(32, total / ((int)gridDim.x * per)));
}
// First item of the wave's next batch of B (same rules as wave_next_item).
__device__ __forceinline__ int wave_next_batch(int* counter, int B) {
    int v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(counter, B);
    return __builtin_amdgcn_readlane(v, 0);
}

typedef __attribute__((address_space(4))) const float const_as_float;   // loads from it are scalar when uniform

// Chunk k (components 4k .. 4k+3, zero past D) of the point at pt; vec: one
// 16-byte load (D a multiple of 4, pt 16-byte aligned).  Chunks at or past D
// (the chunk count is padded up to an instantiated width) read nothing.
// Dword-aligned multi-dword loads (global memory accepts them on gfx950).
struct __attribute__((aligned(4))) f32x4_a4 { float x, y, z, w; };
struct __attribute__((packed, aligned(4))) f32x3_a4 { float x, y, z; };
struct __attribute__((packed, aligned(4))) f32x2_a4 { float x, y; };

__device__ __forceinline__ float4 point_chunk(const float* __restrict__ pt, int k, int D, bool vec) {
    if (vec) return 4 * k < D ? *reinterpret_cast<const float4*>(pt + 4 * k) : make_float4(0.f, 0.f, 0.f, 0.f);
    // the chunk's valid components in one load
    const int left = D - 4 * k;
    const float* c = pt + 4 * k;
    if (left >= 4) {
        const f32x4_a4 v = *reinterpret_cast<const f32x4_a4*>(c);
        return make_float4(v.x, v.y, v.z, v.w);
    }
    if (left == 3) {
        const f32x3_a4 v = *reinterpret_cast<const f32x3_a4*>(c);
        return make_float4(v.x, v.y, v.z, 0.0f);
    }
    if (left == 2) {
        const f32x2_a4 v = *reinterpret_cast<const f32x2_a4*>(c);
        return make_float4(v.x, v.y, 0.0f, 0.0f);
    }
    return make_float4(left == 1 ? c[0] : 0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace tcdtw
