// Device-side DTW cores shared by the pair kernels and the 1-NN kernels.
//
// Both cores evaluate the DTW recurrence (Sec. 2, Eq. 1) inside the
// Sakoe-Chiba band along anti-diagonals, one cell per lane per step, with
// neighbour values passed by DPP whole-wave shifts.  See dtw_fwd.hip for
// the lane layouts.
#pragma once
#include "device_common.h"
#include "internal.h"

namespace tcdtw {

// ------------------------------------------------------------------ staging
// Copies series `src` (row-major [len][D]) into LDS as [k][L][4] chunks for
// positions pos = 0..L-1 holding series index t = pos + first; positions
// outside [0, len) get `sentinel` in every component.
template <int NCH>
__device__ __forceinline__ void stage_series(float4* dst, int L, int first, const float* src, int len,
                                             int D, float sentinel, int lane, int nlanes) {
    for (int pos = lane; pos < L; pos += nlanes) {
        const int t = pos + first;
        const bool in = (t >= 0 && t < len);
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = 4 * k + e;
                v[e] = in ? (p < D ? src[(int64_t)t * D + p] : 0.0f) : sentinel;
            }
            dst[k * L + pos] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

// ---------------------------------------------------------- diagonal pairs
struct DiagGeom {
    int m, n, W, G, h, R, LQ, LC;
    __host__ __device__ void init(int m_, int n_, int W_) {
        m = m_; n = n_; W = W_;
        G = W + 1;
        h = (W + (W & 1)) / 2;
        R = (m + n) / 2;           // rounds: anti-diagonals 0 .. m+n-2
        LQ = R + W + 1;            // query positions, index i = pos + h - W
        LC = R + W + 2;            // candidate positions, index j = pos - h
    }
    __host__ __device__ int qfirst() const { return h - W; }
    __host__ __device__ int cfirst() const { return -h; }
};

// Early-abandon context of a wave (1-NN mode): every `every` rounds the
// groups whose cells on two consecutive anti-diagonals all exceed `thr`
// are abandoned; the loop ends when every live group is.
struct Abandon {
    const unsigned long long* key;   // packed best-so-far of the wave's query
    float gamma;                     // relative error bound of the float DP
    uint64_t valid_mask;             // lanes of groups with a pair
};

__device__ __forceinline__ float bsf_from_key(unsigned long long k) {
    return __uint_as_float((uint32_t)(k >> 32));
}

// Abandon threshold: a cell value v (float DP) proves DTW > bsf when
// v / (1 + gamma) > bsf; computed in double and rounded up.
__device__ __forceinline__ float abandon_threshold(float bsf, float gamma) {
    const double t = (double)bsf * (1.0 + (double)gamma) * (1.0 + 1e-6);
    float f = (float)t;
    if ((double)f < t) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

// One wave, groups of G lanes each evaluating one pair.  qb / cb: this
// lane's LDS bases (position offsets already applied, see dtw_fwd.hip).
// Returns the lane's slot values after the last round through vE / vO;
// `aband` is set for lanes of abandoned groups.
template <typename T, int NCH, bool SAVE, bool WODD, bool ABANDON>
__device__ __forceinline__ void diag_core(const float4* qb, int LQ, const float4* cb, int LC, int R,
                                          int G, int lg, bool kill_e, bool kill_o, T& vE, T& vO,
                                          uint32_t* codes, const Abandon& ab, bool& aband,
                                          uint64_t grp_mask) {
    const T INF = inf_v<T>();
    float4 qv[NCH], cE[NCH], cO[NCH];
#pragma unroll
    for (int k = 0; k < NCH; ++k) cE[k] = cb[k * LC + 0];
    uint32_t cw = 0;
    float thr = __builtin_inff();
    if (ABANDON) thr = abandon_threshold(bsf_from_key(__hip_atomic_load(ab.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)), ab.gamma);

    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            qv[k] = qb[k * LQ + r];
            cO[k] = cb[k * LC + r + 1];
        }
        {   // E step: anti-diagonal 2r.  up = own odd slot, left = lane-1's odd slot.
            const T cost = point_cost<NCH>(qv, cE, T(0));
            const T up = vO;
            const T left = wave_shr1(INF, vO);
            const T diag = vE;
            T best;
            if (SAVE) {
                uint32_t code = 0;
                best = diag;
                if (up < best) { best = up; code = 1; }
                if (left < best) { best = left; code = 2; }
                cw |= code << ((r & 7) * 4);
            } else {
                best = vmin3(diag, up, left);
            }
            T v = add_cost(cost, best);
            if (kill_e) v = INF;
            vE = v;
        }
        {   // O step: anti-diagonal 2r+1.  up = lane+1's even slot, left = own even slot.
            const T cost = point_cost<NCH>(qv, cO, T(0));
            const T up = wave_shl1(INF, vE);
            const T left = vE;
            const T diag = vO;
            T best;
            if (SAVE) {
                uint32_t code = 0;
                best = diag;
                if (up < best) { best = up; code = 1; }
                if (left < best) { best = left; code = 2; }
                cw |= code << ((r & 7) * 4 + 2);
            } else {
                best = vmin3(diag, up, left);
            }
            T v = add_cost(cost, best);
            if (kill_o) v = INF;
            vO = v;
        }
        if (SAVE && ((r & 7) == 7 || r == R - 1)) {
            if (codes) codes[(int64_t)(r >> 3) * G + lg] = cw;
            cw = 0;
        }
#pragma unroll
        for (int k = 0; k < NCH; ++k) cE[k] = cO[k];
        if (ABANDON && (r & 15) == 15 && r + 1 < R) {
            // every path crosses anti-diagonal 2r or 2r+1 (steps advance i+j by 1 or 2)
            const bool over = (float)vmin(vE, vO) > thr;
            const uint64_t bal = __ballot(over);
            if ((bal & grp_mask) == grp_mask) aband = true;
            if ((bal & ab.valid_mask) == ab.valid_mask) break;
            thr = abandon_threshold(bsf_from_key(__hip_atomic_load(ab.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)), ab.gamma);
        }
    }
}

// ------------------------------------------------------------- row-systolic
constexpr int kRowPad = 65;   // candidate / row-buffer positions left of column 0

// One pair per wave.  sc: staged candidate [k][LC] (position j + kRowPad),
// rowbuf: LC values of type T.  xs: query rows in global memory.
// Returns the DTW value in the lane m-1 mod 64 (others undefined).
template <typename T, int NCH, bool SAVE, bool ABANDON>
__device__ __forceinline__ T rows_core(const float4* sc, T* rowbuf, int LC, const float* xs, int m,
                                       int n, int W, int D, int lane, uint32_t* codes,
                                       const Abandon& ab, bool& aband) {
    const T INF = inf_v<T>();
    for (int pos = lane; pos < LC; pos += kWave) rowbuf[pos] = (pos - kRowPad == -1) ? T(0) : INF;
    __syncthreads();
    const int nb = (m + kRowBlock - 1) / kRowBlock;
    const int band = min(n, 2 * W + kRowBlock);
    const int nwb = (band + kRowBlock - 1 + 15) / 16;
    T result = INF;
    for (int b = 0; b < nb; ++b) {
        const int i0 = b * kRowBlock;
        const int i = i0 + lane;
        float4 qv[NCH];
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = 4 * k + e;
                v[e] = (i < m) ? (p < D ? xs[(int64_t)i * D + p] : 0.0f) : __builtin_inff();
            }
            qv[k] = make_float4(v[0], v[1], v[2], v[3]);
        }
        const int jlo = max(0, i0 - W);
        const int jhi = min(n - 1, i0 + kRowBlock - 1 + W);
        const int T_b = jhi - jlo + kRowBlock;
        const int k0 = jlo - i0 + W - 2 * lane;          // band offset k = t + k0 must lie in [0, 2W]
        const float4* cl = sc + (jlo - lane + kRowPad);  // + k*LC + t
        const T* rb = rowbuf + (jlo + kRowPad);          // + t
        T* wb = rowbuf + (jlo - (kRowBlock - 1) + kRowPad);
        T cur = INF;
        T prevup = (lane == 0) ? rowbuf[jlo - 1 + kRowPad] : INF;
        const bool last = (b == nb - 1);
        const int tend = (n - 1) - jlo + (m - 1 - i0);
        uint32_t cw = 0;
        uint32_t* cp = SAVE ? codes + (int64_t)b * nwb * kWave + lane : nullptr;
        for (int t = 0; t < T_b; ++t) {
            float4 cv[NCH];
#pragma unroll
            for (int k = 0; k < NCH; ++k) cv[k] = cl[k * LC + t];
            const T up = wave_shr1(rb[t], cur);
            const T diag = prevup;
            prevup = up;
            const T left = cur;
            const T cost = point_cost<NCH>(qv, cv, T(0));
            T best;
            if (SAVE) {
                uint32_t code = 0;
                best = diag;
                if (up < best) { best = up; code = 1; }
                if (left < best) { best = left; code = 2; }
                cw |= code << ((t & 15) * 2);
                if ((t & 15) == 15 || t == T_b - 1) {
                    cp[(int64_t)(t >> 4) * kWave] = cw;
                    cw = 0;
                }
            } else {
                best = vmin3(diag, up, left);
            }
            T v = add_cost(cost, best);
            const unsigned kb = (unsigned)(t + k0);
            v = (kb <= (unsigned)(2 * W)) ? v : INF;
            cur = v;
            if (lane == kRowBlock - 1) wb[t] = v;
            if (last && t == tend && lane == m - 1 - i0) result = v;
        }
        __syncthreads();
        if (ABANDON && b + 1 < nb) {
            // every path crosses row i0+63: its minimum bounds the final value from below
            const int r0 = max(0, i0 + kRowBlock - 1 - W), r1 = min(n - 1, i0 + kRowBlock - 1 + W);
            T mn = INF;
            for (int j = r0 + lane; j <= r1; j += kWave) mn = vmin(mn, rowbuf[j + kRowPad]);
            const float thr = abandon_threshold(
                bsf_from_key(__hip_atomic_load(ab.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)), ab.gamma);
            const bool over = (float)mn > thr;
            if (__ballot(over) == ~0ull) { aband = true; break; }
        }
    }
    return result;
}

}  // namespace tcdtw
