// LB_TI (LB_TIP with optional TOP, Sec. 4.1-4.2, Fig. 3) for bands wider
// than the one-wave band-offset mapping of k_lb_ti (W_eff > 63).
//
// Column mapping: a wave walks the candidate in blocks of 64 consecutive
// columns, lane l owning column j = j0 + l, and runs the rows of the
// block's band, max(0, j0 - W) .. min(m - 1, j0 + 63 + W), wave-uniformly.
// A column keeps its state (V, Y) = (L + U, 2U) and its running minimum of
// max(0, L) in its own lane from row to row, so Eqs. 7-8 (row i-1 to row i
// on the same column: V' = max(V, 2d), Y' = Y + 2d) need no exchange between
// lanes; a lane takes part in rows j - W .. j + W only.
//  * Exact rows (i = 0, and i mod P = 0 for P > 0) are wave-uniform: the
//    query point q_i is read with scalar loads and the lane's candidate
//    point c_j stays in registers for the whole block.
//  * The top cell of row i is column i + W; it starts that column: under
//    TOP with the exact e(q_i, c_{i+W}) (computed for every row while the
//    pair is staged), otherwise by Eqs. 9-10 from its left neighbour
//    (i, j - 1) in the same row, which is lane l - 1 (for lane 0, the
//    previous block's last column, kept from that block's row j0 - W).
// Every cell sees the same float32 operations in the same order as in
// k_lb_ti, so the per-cell values and the rounding allowance are the same;
// only the order of the final sum differs (covered by the deflation).
//
// Rows run in three phases per block: columns starting (some lanes before
// their first row), every lane inside its band (no per-lane tests), and
// columns ending.
#include "bounds_common.h"

namespace tcdtw {

extern __shared__ float2 lds_ti_cols[];

// sum of squares of q - c (components in index order)
template <int NCH>
__device__ __forceinline__ float exact_sq(const const_as_float* qp, int D, const float4 (&c)[NCH]) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        const float cv[4] = {c[k].x, c[k].y, c[k].z, c[k].w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int p = 4 * k + t;
            const float qv = p < D ? qp[p] : 0.0f;   // padded components are 0 in both points
            const float d = qv - cv[t];
            s = __builtin_fmaf(d, d, s);
        }
    }
    return s;
}

template <bool TOP, int NCH>
__global__ __launch_bounds__(64) void k_lb_ti_cols(TiArgs a) {
    const int lane = threadIdx.x;
    const int m = a.m, n = a.n, D = a.D, W = a.W, P = a.P;
    float2* tdq = lds_ti_cols;                         // [m] (2 d_i, 2 t_i) per row, t_i the TOP distance
    const float INF = __builtin_inff();
    const uint32_t INF_BITS = 0x7f800000u;
    const double u = 1.0 / 16777216.0;
    // longest recursion chain since an exact value (rows, plus one top step per row without TOP)
    const int rmax = P > 0 ? (TOP ? P - 1 : 2 * (P - 1) + 1) : (TOP ? m : 2 * m + 1);
    // safe value V - (1 + s) Y / 2 with s = (1.5 D + 20 + r_max) u 1.02, the factor rounded up
    const float k1h = 0.5f * rup(1.0 + (1.5 * D + 20.0 + rmax) * u * 1.02);
    const double defl = 1.0 - (double)(n + 5) * u * 1.001;
    unsigned long long evaluated = 0;   // pairs this wave evaluated
    const int total = __builtin_amdgcn_readfirstlane(a.prefix[a.nq]);
    const int B = item_batch(total, 16);
    for (;;) {
        const int base = wave_next_batch(a.counter, B);
        if (base >= total) break;
        const int bend = min(base + B, total);
        for (int item = base; item < bend; ++item) {
            const int q = __builtin_amdgcn_readfirstlane(a.item_query[item]);
            const int e = item - __builtin_amdgcn_readfirstlane(a.prefix[q]);
            const int ref = a.in_list ? __builtin_amdgcn_readfirstlane((int)a.in_list[(int64_t)q * a.cap + e]) : e;
            if (a.key) {
                // selective deployment: only pairs whose bound so far exceeds e^2 bsf
                const float cur = a.lb_in[(int64_t)q * a.cap + e];
                const float bsf = key_bsf(a.key + (int64_t)q * kKeyStride);
                if (wave_uniform(!((double)cur > a.e2 * (double)bsf))) {
                    if (lane == 0) a.out_lb[(int64_t)q * a.cap + e] = -1.0f;
                    continue;
                }
            }
            const float* qs = a.Q + (int64_t)q * m * D;
            const float* cs = a.C + (int64_t)ref * n * D;
            const float* gam = a.gamma + (int64_t)ref * n;
            const bool qvec = (D & 3) == 0 && (reinterpret_cast<uintptr_t>(qs) & 15) == 0;
            const bool cvec = (D & 3) == 0 && (reinterpret_cast<uintptr_t>(cs) & 15) == 0;
            __syncthreads();
            for (int i = lane; i < m; i += kWave) {
                float top = INF;
                if (TOP && i + W < n) {
                    float4 qv[NCH], cv[NCH];
#pragma unroll
                    for (int k = 0; k < NCH; ++k) {
                        qv[k] = point_chunk(qs + (int64_t)i * D, k, D, qvec);
                        cv[k] = point_chunk(cs + (int64_t)(i + W) * D, k, D, cvec);
                    }
                    float s = 0.0f;
#pragma unroll
                    for (int k = 0; k < NCH; ++k) {
                        float t;
                        t = qv[k].x - cv[k].x; s = __builtin_fmaf(t, t, s);
                        t = qv[k].y - cv[k].y; s = __builtin_fmaf(t, t, s);
                        t = qv[k].z - cv[k].z; s = __builtin_fmaf(t, t, s);
                        t = qv[k].w - cv[k].w; s = __builtin_fmaf(t, t, s);
                    }
                    top = __builtin_sqrtf(s);
                }
                const float di = a.qstep[(int64_t)q * m + i];
                tdq[i] = make_float2(2.0f * di, 2.0f * top);
            }
            __syncthreads();
            const const_as_float* qsc = (const const_as_float*)qs;
            float acc = 0.0f;
            float carryV = 0.0f, carryY = 0.0f;   // column j0 - 1 at row j0 - W (for Eqs. 9-10)
            for (int j0 = 0; j0 < n; j0 += kWave) {
                const int j = j0 + lane;
                const bool col = j < n;
                float4 c[NCH];
#pragma unroll
                for (int k = 0; k < NCH; ++k) c[k] = point_chunk(cs + (int64_t)min(j, n - 1) * D, k, D, cvec);
                const float gj = (!TOP && col && j >= 1) ? gam[j] : 0.0f;
                const float gj2 = 2.0f * gj;
                float V = 0.0f, Y = 0.0f;
                uint32_t cm = INF_BITS;           // running minimum of the column, >= 0 or +inf: min on the bits
                const int ilo = max(0, j0 - W), ihi = min(m - 1, j0 + kWave - 1 + W);
                const int jlast = min(n, j0 + kWave) - 1;  // the block's last column
                // rows where columns start (up to the last column's first row), where every
                // column of the block is inside its band, and where columns end
                const int a_end = min(ihi, jlast - W);
                const int b_end = min(ihi, j0 + W);
                const int carry_row = j0 + kWave - W;      // the next block's first top row
                int since = P > 0 ? ilo % P : 1;
                float2 t = tdq[ilo];
                int i = ilo;
                auto step = [&](bool generic) __attribute__((always_inline)) {
                    const float2 tc = t;
                    if (i < ihi) t = tdq[i + 1];           // one row ahead
                    const bool exact = (i == 0) || (P > 0 && since == 0);
                    const int r = i - (j - W);            // row index inside the column's band, 0 .. 2W
                    if (exact) {
                        float lo, hi;
                        ti_exact_sides(exact_sq<NCH>(qsc + (int64_t)i * D, D, c), lo, hi);
                        V = lo + hi;
                        Y = hi + hi;
                    } else {
                        const float v = umax_f(V, tc.x);            // Eqs. 7-8: L + U
                        const float y = Y + tc.x;                   // Eq. 8, doubled
                        if (generic && TOP) {
                            V = r == 0 ? tc.y : v;
                            Y = r == 0 ? tc.y : y;
                        } else {
                            V = v;
                            Y = y;
                        }
                        if (generic && !TOP) {
                            // the top cell from its left neighbour in the same row, Eqs. 9-10
                            const float Vl = wave_shr1(carryV, V), Yl = wave_shr1(carryY, Y);
                            if (r == 0) {
                                V = umax_f(Vl, gj2);
                                Y = Yl + gj2;
                            }
                        }
                    }
                    // the safe value clamped at 0 on its bits (negative values have negative bits)
                    const uint32_t safe = (uint32_t)max(__float_as_int(__builtin_fmaf(-k1h, Y, V)), 0);
                    const bool act = !generic || (col && (unsigned)r <= (unsigned)(2 * W));
                    cm = min(cm, act ? safe : INF_BITS);
                    if (!TOP && i == carry_row) {
                        carryV = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(V), kWave - 1));
                        carryY = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Y), kWave - 1));
                    }
                    since = (since + 1 == P) ? 0 : since + 1;
                };
                // a row of the full band: every lane is inside its column's band
                auto plain = [&](float2 tc) __attribute__((always_inline)) {
                    V = umax_f(V, tc.x);                            // Eqs. 7-8: L + U
                    Y = Y + tc.x;                                   // Eq. 8, doubled
                    cm = min(cm, (uint32_t)max(__float_as_int(__builtin_fmaf(-k1h, Y, V)), 0));
                };
                // plain rows up to `stop` (exclusive): four, two, then one per step
                auto plain_rows = [&](int stop) __attribute__((always_inline)) {
                    for (; i + 4 <= stop; i += 4) {
                        const float2 t1 = tdq[i + 1], t2 = tdq[i + 2], t3 = tdq[i + 3];
                        plain(t);
                        plain(t1);
                        plain(t2);
                        t = tdq[i + 4];
                        plain(t3);
                    }
                    if (i + 2 <= stop) {
                        const float2 t1 = tdq[i + 1];
                        plain(t);
                        t = tdq[i + 2];
                        plain(t1);
                        i += 2;
                    }
                    if (i < stop) {
                        const float2 tc = t;
                        t = tdq[i + 1];
                        plain(tc);
                        ++i;
                    }
                };
                for (; i <= a_end; ++i) step(true);
                if (jlast == j0 + kWave - 1 && i <= b_end) {
                    // the first row of the full band is the carry row (Eqs. 9-10 without TOP)
                    step(true);
                    ++i;
                    // then blocks of an exact row and the plain rows up to the next one
                    const int e1 = b_end + 1;
                    const int next = (i == 0 || (P > 0 && since == 0)) ? i : (P > 0 ? i + P - since : e1);
                    plain_rows(min(next, e1));
                    while (i < e1) {
                        t = tdq[i + 1];
                        float lo, hi;
                        ti_exact_sides(exact_sq<NCH>(qsc + (int64_t)i * D, D, c), lo, hi);
                        V = lo + hi;
                        Y = hi + hi;
                        cm = min(cm, (uint32_t)max(__float_as_int(__builtin_fmaf(-k1h, Y, V)), 0));
                        ++i;
                        plain_rows(P > 0 ? min(i + P - 1, e1) : e1);
                    }
                    since = P > 0 ? i % P : 1;
                }
                for (; i <= ihi; ++i) step(true);
                if (col && cm < INF_BITS) {
                    const float v = __uint_as_float(cm);
                    acc = __builtin_fmaf(v, v, acc);
                }
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
            if (lane == 0) a.out_lb[(int64_t)q * a.cap + e] = rdown((double)acc * defl);
            ++evaluated;
        }
    }
    if (a.evaluated && lane == 0 && evaluated) atomicAdd(a.evaluated, evaluated);
}

size_t ti_cols_lds_bytes(int m) { return (size_t)(m + 2) * 8 + 16; }

template <bool TOP>
static hipError_t launch_ti_cols_top(const TiArgs& a, int nblocks, hipStream_t s) {
    const size_t lds = ti_cols_lds_bytes(a.m);
    switch (nch_pad(a.D)) {
        case 1: hipLaunchKernelGGL((k_lb_ti_cols<TOP, 1>), dim3(nblocks), dim3(64), lds, s, a); break;
        case 2: hipLaunchKernelGGL((k_lb_ti_cols<TOP, 2>), dim3(nblocks), dim3(64), lds, s, a); break;
        case 3: hipLaunchKernelGGL((k_lb_ti_cols<TOP, 3>), dim3(nblocks), dim3(64), lds, s, a); break;
        case 4: hipLaunchKernelGGL((k_lb_ti_cols<TOP, 4>), dim3(nblocks), dim3(64), lds, s, a); break;
        case 6: hipLaunchKernelGGL((k_lb_ti_cols<TOP, 6>), dim3(nblocks), dim3(64), lds, s, a); break;
        case 8: hipLaunchKernelGGL((k_lb_ti_cols<TOP, 8>), dim3(nblocks), dim3(64), lds, s, a); break;
        case 12: hipLaunchKernelGGL((k_lb_ti_cols<TOP, 12>), dim3(nblocks), dim3(64), lds, s, a); break;
        case 16: hipLaunchKernelGGL((k_lb_ti_cols<TOP, 16>), dim3(nblocks), dim3(64), lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lb_ti_cols(const TiArgs& a, int nblocks, hipStream_t s) {
    return a.top ? launch_ti_cols_top<true>(a, nblocks, s) : launch_ti_cols_top<false>(a, nblocks, s);
}

}  // namespace tcdtw
