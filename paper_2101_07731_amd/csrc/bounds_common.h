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

typedef __attribute__((address_space(4))) const float const_as_float;   // loads from it are scalar when uniform

// Chunk k (components 4k .. 4k+3, zero past D) of the point at pt; vec: one
// 16-byte load (D a multiple of 4, pt 16-byte aligned).  Chunks at or past D
// (the chunk count is padded up to an instantiated width) read nothing.
__device__ __forceinline__ float4 point_chunk(const float* __restrict__ pt, int k, int D, bool vec) {
    if (vec) return 4 * k < D ? *reinterpret_cast<const float4*>(pt + 4 * k) : make_float4(0.f, 0.f, 0.f, 0.f);
    float v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = 4 * k + c < D ? pt[4 * k + c] : 0.0f;
    return make_float4(v[0], v[1], v[2], v[3]);
}

}  // namespace tcdtw
