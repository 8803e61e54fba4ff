// Candidate index for gfx950: series copy, element-major 64-candidate tiles,
// candidate neighbour distances and the value range.
#include "device_common.h"
#include "internal.h"

namespace tcdtw {

// Float -> unsigned key with the same order (for atomic min / max).
__device__ __forceinline__ uint32_t ordered_key(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline float key_to_float(uint32_t k) {
    const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    __builtin_memcpy(&f, &b, 4);
    return f;
}

__global__ void k_range_init(uint32_t* rk) {
    if (threadIdx.x == 0) { rk[0] = 0xffffffffu; rk[1] = 0u; }
}

// Copies the candidate set (uniform: [count][len][D] at `src`; ragged: per
// series offsets) into `series` (concatenated, same order) and reduces the
// value range into rk[0] (min key) / rk[1] (max key).
__global__ void k_index_series(const float* src, const int64_t* src_off, const int64_t* dst_off,
                               const int32_t* lens, const int32_t* dims, int count, int ulen, int D,
                               int64_t total, float* series, uint32_t* rk) {
    __shared__ uint32_t smin, smax;
    if (threadIdx.x == 0) { smin = 0xffffffffu; smax = 0u; }
    __syncthreads();
    uint32_t lmin = 0xffffffffu, lmax = 0u;
    if (ulen > 0) {
        const int64_t nel = (int64_t)count * ulen * D;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nel;
             e += (int64_t)gridDim.x * blockDim.x) {
            const float v = src[e];
            series[e] = v;
            const uint32_t k = ordered_key(v);
            lmin = min(lmin, k);
            lmax = max(lmax, k);
        }
    } else {
        // one block-stride loop per series (ragged)
        for (int s = blockIdx.x; s < count; s += gridDim.x) {
            const int64_t n = (int64_t)lens[s] * (dims ? dims[s] : D);
            const float* a = src + src_off[s];
            float* b = series + dst_off[s];
            for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
                const float v = a[e];
                b[e] = v;
                const uint32_t k = ordered_key(v);
                lmin = min(lmin, k);
                lmax = max(lmax, k);
            }
        }
    }
    (void)total;
    atomicMin(&smin, lmin);
    atomicMax(&smax, lmax);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMin(&rk[0], smin);
        atomicMax(&rk[1], smax);
    }
}

// Element-major tiles: tiles[(tile * E + e) * 64 + lane] = series[(tile*64+lane) * E + e],
// E = len * D; zero for candidates past the end.
// Layout tiles[tile][e / 4][lane][e % 4]: a lane reads four consecutive
// elements of its candidate with one 16-byte load, a wave 1 KB; elements
// past E (padding to a multiple of 4) are 0.
__global__ void k_index_tiles(const float* series, int count, int E, int ntiles, float* tiles) {
    const int E4 = (E + 3) / 4;
    const int64_t total = (int64_t)ntiles * E4 * 256;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int comp = (int)(idx & 3);
        const int lane = (int)((idx >> 2) & 63);
        const int64_t te4 = idx >> 8;
        const int tile = (int)(te4 / E4);
        const int e = 4 * (int)(te4 - (int64_t)tile * E4) + comp;
        const int r = tile * 64 + lane;
        tiles[idx] = (r < count && e < E) ? series[(int64_t)r * E + e] : 0.0f;
    }
}

// Candidate neighbour distances gamma_j = e(c_{j-1}, c_j), gamma_0 = 0 (Sec. 4.1,
// triangle at the top of a window).  One thread per point.
__global__ void k_index_gamma(const float* series, const int64_t* dst_off, const int32_t* lens,
                              const int32_t* dims, int count, int ulen, int Dall, const int64_t* goff,
                              float* gamma) {
    for (int s = blockIdx.y; s < count; s += gridDim.y) {
        const int L = ulen > 0 ? ulen : lens[s];
        const int D = dims ? dims[s] : Dall;
        const float* a = series + (ulen > 0 ? (int64_t)s * ulen * D : dst_off[s]);
        float* g = gamma + (ulen > 0 ? (int64_t)s * ulen : goff[s]);
        for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < L; j += gridDim.x * blockDim.x) {
            float acc = 0.0f;
            if (j > 0)
                for (int p = 0; p < D; ++p) {
                    const float d = a[(int64_t)j * D + p] - a[(int64_t)(j - 1) * D + p];
                    acc = __builtin_fmaf(d, d, acc);
                }
            g[j] = __builtin_sqrtf(acc);
        }
    }
}

// rk keys -> float[2] (min, max) in place.  A value that is not finite
// (NaN keys order beyond the infinities) leaves a non-finite min or max,
// which is reported in the status word.
__global__ void k_range_finish(uint32_t* rk, uint32_t* status) {
    if (threadIdx.x == 0) {
        const float lo = key_to_float(rk[0]), hi = key_to_float(rk[1]);
        reinterpret_cast<float*>(rk)[0] = lo;
        reinterpret_cast<float*>(rk)[1] = hi;
        if (status && !(__builtin_isfinite(lo) && __builtin_isfinite(hi))) atomicOr(status, kStatusNonFiniteRef);
    }
}

hipError_t launch_index_build(const IndexBuildArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_range_init, dim3(1), dim3(64), 0, s, a.range_keys);
    hipLaunchKernelGGL(k_index_series, dim3(1024), dim3(256), 0, s, a.src, a.src_off, a.dst_off, a.lens, a.dims,
                       a.count, a.ulen, a.D, a.total_len, a.series, a.range_keys);
    if (a.ulen > 0 && a.tiles) {
        hipLaunchKernelGGL(k_index_tiles, dim3(2048), dim3(256), 0, s, a.series, a.count, a.ulen * a.D,
                           a.ntiles, a.tiles);
    }
    const int gy = a.count < 65535 ? a.count : 65535;
    const int gx = (a.maxlen + 255) / 256;
    hipLaunchKernelGGL(k_index_gamma, dim3(gx, gy), dim3(256), 0, s, a.series, a.dst_off, a.lens, a.dims,
                       a.count, a.ulen, a.D, a.gamma_off, a.gamma);
    hipLaunchKernelGGL(k_range_finish, dim3(1), dim3(64), 0, s, a.range_keys, a.status);
    return hipGetLastError();
}

}  // namespace tcdtw
