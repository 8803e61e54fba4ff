// Advanced lower bounds of the cascade for gfx950: the point-clustering bound
// LB_PC (Sec. 5) and the triangle bound LB_TI (Sec. 4.1-4.2), evaluated on
// per-query candidate lists (the gated pairs of the 1-NN search, or every
// candidate for the dense bound matrix), and the routing of gated pairs
// (Sec. 6, selective deployment).
//
// Rounding: every value returned never exceeds the exact bound of the
// float32 inputs (u = 2^-24):
//  * LB_PC: a sum of n non-negative per-point minima, each a fused
//    multiply-add chain of D terms; scaled by 1 - (n + D + 5) u and rounded
//    down;
//  * LB_TI: a computed triangle bound L_f after r recursion steps from an
//    exact distance differs from the exact recursion by at most
//    (D/2 + 3 + r) u U_f (U_f the matching upper bound, which grows by the
//    same steps as the allowance), so L_f - (D/2 + 5 + r_max) u U_f is used
//    before the clamp at zero; the sum of the squared column minima is
//    scaled by 1 - (n + 5) u and rounded down.
#include <algorithm>
#include <type_traits>

#include "bounds_common.h"

namespace tcdtw {

extern __shared__ float4 lds4[];

// --------------------------------------------------------- query steps
// delta[q][i] = e(q_{i-1}, q_i) (delta[q][0] = 0), the query-side distances
// of Eqs. 7-8, computed once per query (Sec. 4.1).
__global__ void k_query_steps(const float* __restrict__ Q, int nq, int m, int D, float* __restrict__ delta) {
    const int64_t total = (int64_t)nq * m;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % m);
        float s = 0.0f;
        if (i > 0) {
            const float* a = Q + t * D;
            for (int p = 0; p < D; ++p) {
                const float d = a[p] - a[p - D];
                s = __builtin_fmaf(d, d, s);
            }
        }
        delta[t] = __builtin_sqrtf(s);
    }
}

// ------------------------------------------------------------------- K4
// Boxes of one query's expanded windows (Sec. 5, quantisation-based
// clustering with uniform window grouping): one wave per (group, query).
// Cell assignment in float32 exactly as written: per-dimension range of the
// window's points, cell length max((hi - lo) / Lv, floor), digit
// min(Lv - 1, floor((x - lo) / len)), key = digits in base Lv with
// dimension 0 most significant.  The first K-1 distinct cells in key order
// own a box each; later cells share box K.  Boxes are the tight [min, max]
// of their member points.  LDS: keys (u64), first-occurrence flags, then
// K*D*2 ordered-int box bounds.
__global__ __launch_bounds__(64) void k_pc_boxes(PcArgs a) {
    const int lane = threadIdx.x;
    const int g = blockIdx.x, q = blockIdx.y;
    const int m = a.m, n = a.n, D = a.D, W = a.W, w = a.w, K = a.K, Lv = a.Lv;
    const int jfirst = g * w, jlast = min(n - 1, g * w + w - 1);
    const int ilo = max(0, jfirst - W), ihi = min(m - 1, jlast + W);
    const int npts = ihi - ilo + 1;
    const float* Q = a.Q + (int64_t)q * m * D;
    unsigned long long* keys = reinterpret_cast<unsigned long long*>(lds4);
    int32_t* first = reinterpret_cast<int32_t*>(keys + a.max_pts);
    uint32_t* bx = reinterpret_cast<uint32_t*>(first + a.max_pts);   // [K][D][2]
    for (int t = lane; t < K * D; t += kWave) {
        bx[2 * t] = 0xffffffffu;
        bx[2 * t + 1] = 0u;
    }
    for (int i = lane; i < npts; i += kWave) keys[i] = 0ull;
    __syncthreads();
    for (int p = 0; p < D; ++p) {
        float lo = __builtin_inff(), hi = -__builtin_inff();
        for (int i = ilo + lane; i <= ihi; i += kWave) {
            const float x = Q[(int64_t)i * D + p];
            lo = __builtin_fminf(lo, x);
            hi = __builtin_fmaxf(hi, x);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo = __builtin_fminf(lo, __shfl_xor(lo, o));
            hi = __builtin_fmaxf(hi, __shfl_xor(hi, o));
        }
        float fl = a.floor_len;
        if (!(fl > 0.0f) && a.range) fl = (float)(1e-5 * (double)(a.range[1] - a.range[0]));
        float len = (hi - lo) / (float)Lv;
        if (len < fl) len = fl;
        for (int i = ilo + lane; i <= ihi; i += kWave) {
            const float x = Q[(int64_t)i * D + p];
            int dgt = 0;
            if (len > 0.0f) dgt = (int)__builtin_floorf((x - lo) / len);
            if (dgt > Lv - 1) dgt = Lv - 1;
            keys[i - ilo] = keys[i - ilo] * (unsigned long long)Lv + (unsigned long long)dgt;
        }
        __syncthreads();
    }
    // first occurrence of each key, then the rank of each point's key among the distinct keys
    int M = 0;
    for (int i = lane; i < npts; i += kWave) {
        const unsigned long long ki = keys[i];
        int f = 1;
        for (int t = 0; t < i; ++t) f &= (keys[t] != ki) ? 1 : 0;
        first[i] = f;
        M += f;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) M += __shfl_xor(M, o);
    __syncthreads();
    for (int i = lane; i < npts; i += kWave) {
        const unsigned long long ki = keys[i];
        int rank = 0;
        for (int t = 0; t < npts; ++t) rank += (first[t] && keys[t] < ki) ? 1 : 0;
        const int b = rank < K - 1 ? rank : K - 1;
        for (int p = 0; p < D; ++p) {
            const uint32_t kv = okey(Q[(int64_t)(ilo + i) * D + p]);
            atomicMin(&bx[2 * (b * D + p)], kv);
            atomicMax(&bx[2 * (b * D + p) + 1], kv);
        }
    }
    __syncthreads();
    const int nb = M < K ? M : K;
    float* out = a.boxes + ((int64_t)q * a.ngroups + g) * K * D * 2;
    for (int t = lane; t < K * D; t += kWave) {
        const int b = t / D;
        out[2 * t] = b < nb ? okey_to_float(bx[2 * t]) : __builtin_inff();
        out[2 * t + 1] = b < nb ? okey_to_float(bx[2 * t + 1]) : -__builtin_inff();
    }
    if (lane == 0) a.nbox[(int64_t)q * a.ngroups + g] = nb;
}

// ------------------------------------------------------------------- K5
// LB_PC of one listed pair per wave (Sec. 5, Fig. 4(a)): lanes over the
// candidate's points (consecutive points, so the loads are coalesced); for
// each point the smallest squared distance to a box of its group (the
// query's boxes are a few KB, read through the caches), summed over points.
// In search mode a pair is only evaluated when its LB_MV exceeds e^2 bsf,
// and the evaluation stops once the partial sum already proves the pair
// prunable.  With candidate-side boxes (Sec. 8, roles swapped) the points
// are the query's and the boxes the candidate's, grouped over query positions.
template <int DMAX>
__global__ __launch_bounds__(64) void k_lb_pc(PcArgs a) {
    const int lane = threadIdx.x;
    const bool cand = a.cand != 0;
    const int D = a.D, n = cand ? a.m : a.n, K = a.K, w = a.w;
    const double defl = 1.0 - (double)(n + D + 5) * (1.0 / 16777216.0) * 1.001;
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
            float bsf = __builtin_inff();
            if (a.key) {
                bsf = key_bsf(a.key + (int64_t)q * kKeyStride);
                // selective deployment: only pairs with LB_MV > e^2 bsf
                const float mv = a.lb_mv[(int64_t)q * a.nc + ref];
                if (wave_uniform(!((double)mv > a.e2 * (double)bsf))) {
                    if (lane == 0) a.out_lb[(int64_t)q * a.cap + e] = -1.0f;   // not evaluated
                    continue;
                }
            }
            // the evaluated points, and the series whose boxes they are measured against
            const float* c = cand ? a.Q + (int64_t)q * n * D : a.C + (int64_t)ref * n * D;
            const int owner = cand ? ref : q;
            const float* bxq = a.boxes + (int64_t)owner * a.ngroups * K * D * 2;
            const int32_t* nbq = a.nbox + (int64_t)owner * a.ngroups;
            const double stop = a.key ? (double)bsf / a.keep : __builtin_inf();
            float acc = 0.0f;
            for (int j0 = 0; j0 < n; j0 += kWave) {
                const int j = j0 + lane;
                if (j < n) {
                    const int g = j / w;
                    const int nb = nbq[g];
                    const float* bg = bxq + (int64_t)g * K * D * 2;
                    float cv[DMAX];
#pragma unroll
                    for (int p = 0; p < DMAX; ++p) cv[p] = p < D ? c[(int64_t)j * D + p] : 0.0f;
                    float best = __builtin_inff();
                    for (int b = 0; b < nb; ++b) {
                        // the box's (lo, hi) pairs, all loads issued before any use (dimensions
                        // past D re-read dimension 0 and are skipped below)
                        const float2* bb = reinterpret_cast<const float2*>(bg + b * D * 2);
                        float2 lh[DMAX];
#pragma unroll
                        for (int p = 0; p < DMAX; ++p) lh[p] = bb[p < D ? p : 0];
                        float s = 0.0f;
#pragma unroll
                        for (int p = 0; p < DMAX; ++p) {
                            if (p < D) {
                                const float t = __builtin_fmaxf(__builtin_fmaxf(lh[p].x - cv[p], cv[p] - lh[p].y), 0.0f);
                                s = __builtin_fmaf(t, t, s);
                            }
                        }
                        best = __builtin_fminf(best, s);
                    }
                    acc += best;
                }
                if (a.key && j0 + kWave < n) {
                    float tot = acc;
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) tot += __shfl_xor(tot, o);
                    if (wave_uniform((double)tot * defl > stop)) break;
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

// ------------------------------------------------------------------- K6
// LB_PC with the query's boxes (Sec. 5), lanes over candidates: a wave takes
// up to 64 listed candidates of one query, so the query's boxes of a group
// are the same for every lane; they are read through the scalar cache into
// scalar registers (through a constant-address-space pointer: the boxes are
// never written while the kernel runs, and uniform loads from that address
// space are scalar loads), and
// each lane walks its own candidate's points in order.  Per (point, box,
// dimension): two subtractions with a scalar operand, a 3-way max with 0 and
// an FMA; per box a minimum.  DC: the point width D when it is fixed at
// compile time (no test per dimension, the box's bounds read by wide scalar
// loads), 0 when it is read at run time.  The distance of x to [lo, hi] is
// x - med3(x, lo, hi): one operation fewer per point than max(lo - x,
// x - hi, 0) once the box's lo sits in a vector register (gfx950 reads one
// scalar operand per instruction; the move serves the PPS points of a step),
// and equal to it bit for bit up to the sign, which the square removes.

// Squared distance of a point (NCH chunks) to the box at bb ([D][2] lo, hi).
template <int NCH, int DC>
__device__ __forceinline__ float box_dist(const const_as_float* bb, int D, const float4 (&c)[NCH]) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        const float cv[4] = {c[k].x, c[k].y, c[k].z, c[k].w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int p = 4 * k + t;
            if (DC > 0 ? p < DC : p < D) {
                const float v = cv[t] - __builtin_amdgcn_fmed3f(cv[t], bb[2 * p], bb[2 * p + 1]);
                s = __builtin_fmaf(v, v, s);
            }
        }
    }
    return s;
}

template <int NCH, int DC, int PPS>
__global__ __launch_bounds__(64) void k_lb_pc_lanes(PcArgs a) {
    constexpr bool EXACT = DC == 4 * NCH;
    const int lane = threadIdx.x;
    const int D = DC > 0 ? DC : a.D, n = a.n, K = a.K, w = a.w, G = a.ngroups;
    const double defl = 1.0 - (double)(n + D + 5) * (1.0 / 16777216.0) * 1.001;
    const bool vec = EXACT && (reinterpret_cast<uintptr_t>(a.C) & 15) == 0;
    unsigned long long evaluated = 0;   // pairs this wave evaluated
    for (;;) {
        const int item = wave_next_item(a.counter);
        if (item >= a.prefix[a.nq]) break;
        const int q = __builtin_amdgcn_readfirstlane(a.item_query[item]);
        const int e = (item - __builtin_amdgcn_readfirstlane(a.prefix[q])) * kWave + lane;
        const int cnt = a.in_list ? a.in_cnt[q] : a.in_uniform;
        bool live = e < cnt;
        const int ref = live ? (a.in_list ? (int)a.in_list[(int64_t)q * a.cap + e] : e) : 0;
        double stop = __builtin_inf();
        if (a.key) {
            const float bsf = key_bsf(a.key + (int64_t)q * kKeyStride);
            // selective deployment: only pairs with LB_MV > e^2 bsf
            if (live && !((double)a.lb_mv[(int64_t)q * a.nc + ref] > a.e2 * (double)bsf)) {
                a.out_lb[(int64_t)q * a.cap + e] = -1.0f;   // not evaluated
                live = false;
            }
            stop = (double)bsf / a.keep;
        }
        const uint64_t lv = __ballot(live);
        if (lv == 0) continue;
        evaluated += (unsigned long long)__popcll(lv);
        const float* cs = a.C + (int64_t)ref * n * D;
        const float* bq = a.boxes + (int64_t)q * G * K * D * 2;
        const int32_t* nbq = a.nbox + (int64_t)q * G;
        float acc = 0.0f;
        // The candidate's points in runs of PPS (j .. j+PPS-1) inside a group; the next run's
        // points are loaded while the current run is measured against its group's boxes (PPS
        // points against two boxes per step: 2 PPS independent chains, and each box's scalar
        // load serves PPS points).
        auto load_run = [&](int jj, int jj1, float4 (&x)[PPS][NCH]) __attribute__((always_inline)) {
#pragma unroll
            for (int u = 0; u < PPS; ++u) {
                const int jb = jj + u < jj1 ? jj + u : jj;
#pragma unroll
                for (int k = 0; k < NCH; ++k) x[u][k] = point_chunk(cs + (int64_t)jb * D, k, D, vec);
            }
        };
        int g = 0, j = 0, j1 = min(n, w);
        float4 c[PPS][NCH];
        load_run(0, j1, c);
        for (;;) {
            int jn = j + PPS, gn = g, j1n = j1;
            if (jn >= j1) {
                gn = g + 1;
                jn = gn * w;
                j1n = min(n, jn + w);
            }
            const bool more = gn < G;
            float4 p[PPS][NCH];
            load_run(more ? jn : 0, more ? j1n : 1, p);   // (past the end: point 0, unused)
            const int nb = __builtin_amdgcn_readfirstlane(nbq[g]);
            const const_as_float* bc = (const const_as_float*)(bq + (int64_t)g * K * D * 2);
            float mm[PPS];
#pragma unroll
            for (int u = 0; u < PPS; ++u) mm[u] = __builtin_inff();
            int b = 0;
            for (; b + 1 < nb; b += 2) {
                const const_as_float* b0 = bc + b * D * 2;
                const const_as_float* b1 = b0 + D * 2;
#pragma unroll
                for (int u = 0; u < PPS; ++u)
                    mm[u] = __builtin_fminf(mm[u], __builtin_fminf(box_dist<NCH, DC>(b0, D, c[u]),
                                                                   box_dist<NCH, DC>(b1, D, c[u])));
            }
            if (b < nb) {
                const const_as_float* b0 = bc + b * D * 2;
#pragma unroll
                for (int u = 0; u < PPS; ++u) mm[u] = __builtin_fminf(mm[u], box_dist<NCH, DC>(b0, D, c[u]));
            }
#pragma unroll
            for (int u = 0; u < PPS; ++u)
                if (u == 0 || j + u < j1) acc += mm[u];
            // group g done: the partial sum is already a bound; stop once it proves every live
            // pair prunable
            if (gn != g && a.key && (g & 7) == 7 && more &&
                __ballot(live && !((double)acc * defl > stop)) == 0)
                break;
            if (!more) break;
#pragma unroll
            for (int u = 0; u < PPS; ++u)
#pragma unroll
                for (int k = 0; k < NCH; ++k) c[u][k] = p[u][k];
            j = jn;
            g = gn;
            j1 = j1n;
        }
        if (live) a.out_lb[(int64_t)q * a.cap + e] = rdown((double)acc * defl);
    }
    if (a.evaluated && lane == 0 && evaluated) atomicAdd(a.evaluated, evaluated);
}

// LB_PC with the query's boxes (Sec. 5), lanes over the candidate's points,
// for narrow points (d <= 4) and series of at most 192 positions: a wave
// takes up to 64 listed candidates of one query and measures them one after
// another.  Lane l holds positions 3l .. 3l+2 of every candidate (inside one
// group, the group length being a multiple of three) and the KM boxes of
// that group in registers, read once per work item (boxes past the group's
// count are +inf, so they never win the minimum).  The wave reads each
// candidate in one contiguous stretch, and a candidate the trigger skips
// costs nothing; the pair's sum is each lane's three minima added in order,
// then summed across the wave (the deflation covers any summation order).
template <int DC, int KM>
__global__ __launch_bounds__(64) void k_lb_pc_pts(PcArgs a) {
    const int lane = threadIdx.x;
    const int n = a.n, G = a.ngroups;
    const double defl = 1.0 - (double)(n + DC + 5) * (1.0 / 16777216.0) * 1.001;
    const int j0 = 3 * lane;
    const int g = j0 < n ? j0 / a.w : 0;
    const float INF = __builtin_inff();
    unsigned long long evaluated = 0;   // pairs this wave evaluated
    for (;;) {
        const int item = wave_next_item(a.counter);
        if (item >= a.prefix[a.nq]) break;
        const int q = __builtin_amdgcn_readfirstlane(a.item_query[item]);
        const int e0 = (item - __builtin_amdgcn_readfirstlane(a.prefix[q])) * kWave;
        const int cnt = __builtin_amdgcn_readfirstlane(a.in_list ? a.in_cnt[q] : a.in_uniform);
        const int e1 = min(cnt, e0 + kWave);
        // this lane's group's boxes
        float lo[KM][DC], hi[KM][DC];
        {
            const int nb = j0 < n ? a.nbox[(int64_t)q * G + g] : 0;
            const float* bq = a.boxes + ((int64_t)q * G + g) * a.K * DC * 2;
#pragma unroll
            for (int b = 0; b < KM; ++b)
#pragma unroll
                for (int p = 0; p < DC; ++p) {
                    lo[b][p] = b < nb ? bq[(b * DC + p) * 2] : INF;
                    hi[b][p] = b < nb ? bq[(b * DC + p) * 2 + 1] : INF;
                }
        }
        float bsf = INF;
        if (a.key) bsf = key_bsf(a.key + (int64_t)q * kKeyStride);
        auto ref_of = [&](int e) __attribute__((always_inline)) -> int {
            return a.in_list ? (int)__builtin_amdgcn_readfirstlane((int)a.in_list[(int64_t)q * a.cap + e]) : e;
        };
        // selective deployment: only pairs with LB_MV > e^2 bsf
        auto gated = [&](int ref) __attribute__((always_inline)) -> bool {
            return a.key && !((double)a.lb_mv[(int64_t)q * a.nc + ref] > a.e2 * (double)bsf);
        };
        auto load = [&](int ref, float4 (&x)[3]) __attribute__((always_inline)) {
            const float* cs = a.C + (int64_t)ref * n * DC;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int j = j0 + t < n ? j0 + t : 0;
                x[t] = point_chunk(cs + (int64_t)j * DC, 0, DC, false);
            }
        };
        int e = e0;
        int ref = e < e1 ? ref_of(e) : 0;
        float4 x[3];
        load(ref, x);
        while (e < e1) {
            // the next listed candidate's points are read while this one is measured
            const int en = e + 1;
            const int refn = en < e1 ? ref_of(en) : ref;
            float4 xn[3];
            load(refn, xn);
            if (gated(ref)) {
                if (lane == 0) a.out_lb[(int64_t)q * a.cap + e] = -1.0f;   // not evaluated
            } else {
                float s = 0.0f;
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const float cv[4] = {x[t].x, x[t].y, x[t].z, x[t].w};
                    float m = INF;
#pragma unroll
                    for (int b = 0; b < KM; ++b) {
                        float d = 0.0f;
#pragma unroll
                        for (int p = 0; p < DC; ++p) {
                            const float v = cv[p] - __builtin_amdgcn_fmed3f(cv[p], lo[b][p], hi[b][p]);
                            d = __builtin_fmaf(v, v, d);
                        }
                        m = __builtin_fminf(m, d);
                    }
                    s += j0 + t < n ? m : 0.0f;
                }
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
                if (lane == 0) a.out_lb[(int64_t)q * a.cap + e] = rdown((double)s * defl);
                ++evaluated;
            }
#pragma unroll
            for (int t = 0; t < 3; ++t) x[t] = xn[t];
            e = en;
            ref = refn;
        }
    }
    if (a.evaluated && lane == 0 && evaluated) atomicAdd(a.evaluated, evaluated);
}

// dst[r * NCH + k] = chunk k of point r * rstride of the series at src, for
// rows r < rows, by one wave with eight chunks per lane in flight.
template <int NCH>
__device__ __forceinline__ void stage_point_chunks(float4* dst, const float* __restrict__ src, int rows, int rstride,
                                                   int D, bool vec, int lane) {
    const int total = rows * NCH;
    auto at = [&](int t) __attribute__((always_inline)) {
        return point_chunk(src + (int64_t)(t / NCH) * rstride * D, t % NCH, D, vec);
    };
    int t = lane;
    for (; t + 7 * kWave < total; t += 8 * kWave) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = at(t + u * kWave);
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[t + u * kWave] = v[u];
    }
    for (; t < total; t += kWave) dst[t] = at(t);
}

// LB_TI (LB_TIP with optional TOP, Sec. 4.1-4.2, Fig. 3) of one listed
// pair per wave.  Lane k (and k + 64 with two slots) holds band offset k,
// i.e. cell (i, i - W + k) of row i.  The cell of row i+1 on the same
// column is offset k - 1, so a cell's state and the running column minimum
// of max(0, L) move one lane down per row (DPP shift); a column's minimum
// is final when it leaves offset 0.
//
// A cell keeps (V, Y) = (L + U, 2U) instead of (L, U).  Eqs. 7-8 take the
// step d = |q_i - q_{i-1}| as L' = max(L - d, d - U), U' = U + d, so
// V' = max(V, 2d) and Y' = Y + 2d: one maximum and one addition per cell,
// each reading its operand straight from the neighbouring lane, and
// L' = V' - Y'/2 only enters the safe value V' - (1 + s) Y'/2 (one fused
// multiply-add).  Doubling is exact, so Y rounds exactly as U would.
// Eqs. 9-10 for the top cell without TOP have the same form with gamma_j
// and the left neighbour's (V, Y).
// Exact rows (i = 0 and i mod P = 0) compute e(q_i, c_j) (query point
// broadcast from LDS, candidate point per lane) and set V = Y = 2e (the
// hardware square root, see ti_exact_sides);
// the top cell of each row takes the precomputed e(q_i, c_{i+W}) under
// TOP.  TOP and the point width (NCH float4 chunks, zero-padded) are
// template parameters.
//
// Rows run in three phases: the first W + 1 rows and the rows whose band
// reaches past the candidate's end test every lane for a cell; between
// them every band offset is a cell, so a lane's mask is fixed and a
// leaving column always has one.  There, the P - 1 rows between two exact
// rows form one branch-free loop.
template <int SLOTS, bool TOP, int NCH>
__global__ __launch_bounds__(64) void k_lb_ti(TiArgs a) {
    const int lane = threadIdx.x;
    const int m = a.m, n = a.n, D = a.D, W = a.W, P = a.P;
    // LDS, staged per pair so that the row loop never waits on global memory:
    // [NCH][n] candidate points, chunk-major: a row's lanes read consecutive 16-byte words
    float4* cst = lds4;
    float4* qex = cst + (int64_t)n * NCH;              // [exact rows][NCH] query points of the exact rows
    // [m + 2] per row i: (2 d_i, 2 t_i) with t_i the TOP distance e(q_i, c_{i+W}) or, without
    // TOP, gamma_{i+W}; entries m and m + 1 are padding, read ahead past the last row
    float2* tdq = reinterpret_cast<float2*>(qex + (int64_t)ti_exact_rows(m, P) * NCH);
    const int KB = 2 * W + 1;                          // band offsets 0 .. 2W
    const float INF = __builtin_inff();
    const uint32_t INF_BITS = 0x7f800000u;
    const double u = 1.0 / 16777216.0;
    // longest recursion chain since an exact value (rows, plus one top step per row without TOP)
    const int rmax = P > 0 ? (TOP ? P - 1 : 2 * (P - 1) + 1) : (TOP ? m : 2 * m + 1);
    // safe value V - (1 + s) Y / 2 with s = (1.5 D + 20 + r_max) u 1.02, the factor rounded up
    const float k1h = 0.5f * rup(1.0 + (1.5 * D + 20.0 + rmax) * u * 1.02);
    const double defl = 1.0 - (double)(n + 5) * u * 1.001;
    const int kt = KB - 1;                             // top offset
    const int kl = kt > 0 ? kt - 1 : 0;                // its left neighbour
    // rows [ib, ie): every offset 0 .. 2W of the row is a column of the candidate (i >= W, i + W < n)
    // and the column leaving offset 0 had a cell (i >= W + 1); without TOP, the top cell also
    // needs a left neighbour (W >= 1)
    const int ib = min(m, W + 1);
    const int ie = (!TOP && W == 0) ? ib : max(ib, min(m, n - W));
    unsigned long long evaluated = 0;   // pairs this wave evaluated
    const int total = __builtin_amdgcn_readfirstlane(a.prefix[a.nq]);
    const int B = item_batch(total, 16);
    for (;;) {
        const int base = wave_next_batch(a.counter, B);
        if (base >= total) break;
        const int bend = min(base + B, total);
        for (int item = base; item < bend; ++item) {
            const int q = a.item_query[item];
            const int e = item - a.prefix[q];
            const int ref = a.in_list ? (int)a.in_list[(int64_t)q * a.cap + e] : e;
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
            // points as whole 16-byte chunks when D is a multiple of 4 and both series are aligned
            const bool vec = (D & 3) == 0 && ((reinterpret_cast<uintptr_t>(qs) | reinterpret_cast<uintptr_t>(cs)) & 15) == 0;
            __syncthreads();
            {
                const float* qsp = a.qstep + (int64_t)q * m;
                const float* gam = a.gamma + (int64_t)ref * n;
                int i = lane;
                for (; i + 3 * kWave < m; i += 4 * kWave) {
                    float v[4], g[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        v[r] = qsp[i + r * kWave];
                        g[r] = (!TOP && i + r * kWave + W < n) ? gam[i + r * kWave + W] : 0.0f;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) tdq[i + r * kWave] = make_float2(2.0f * v[r], 2.0f * g[r]);
                }
                for (; i < m; i += kWave) {
                    const float v = qsp[i], g = (!TOP && i + W < n) ? gam[i + W] : 0.0f;
                    tdq[i] = make_float2(2.0f * v, 2.0f * g);
                }
                if (lane < 2) tdq[m + lane] = make_float2(0.0f, INF);
            }
            {
                // chunk-major staging: cst[k * n + r] is chunk k of point r; SU points per lane
                // (eight chunks at narrow points) in flight
                constexpr int SU = NCH <= 2 ? 4 : (NCH <= 4 ? 2 : 1);
                int r = lane;
                for (; r + (SU - 1) * kWave < n; r += SU * kWave) {
                    float4 v[NCH][SU];
#pragma unroll
                    for (int k = 0; k < NCH; ++k)
#pragma unroll
                        for (int u = 0; u < SU; ++u) v[k][u] = point_chunk(cs + (int64_t)(r + u * kWave) * D, k, D, vec);
#pragma unroll
                    for (int k = 0; k < NCH; ++k)
#pragma unroll
                        for (int u = 0; u < SU; ++u) cst[k * n + r + u * kWave] = v[k][u];
                }
                for (; r < n; r += kWave) {
#pragma unroll
                    for (int k = 0; k < NCH; ++k) cst[k * n + r] = point_chunk(cs + (int64_t)r * D, k, D, vec);
                }
            }
            // exact rows are i = 0 and (P > 0) the multiples of P: row i's point at qex[i / P]
            stage_point_chunks<NCH>(qex, qs, ti_exact_rows(m, P), P > 0 ? P : 0, D, vec, lane);
            if (TOP) {
                // e(q_i, c_{i+W}): query chunks of several rows in flight, candidate chunks from LDS;
                // components summed in index order (padding adds exact zeros)
                __syncthreads();
                constexpr int RU = NCH <= 2 ? 2 : 1;
                for (int i0 = lane; i0 < m; i0 += RU * kWave) {
                    float4 qv[RU][NCH];
#pragma unroll
                    for (int r = 0; r < RU; ++r) {
                        const int i = i0 + r * kWave;
#pragma unroll
                        for (int k = 0; k < NCH; ++k)
                            qv[r][k] = i < m ? point_chunk(qs + (int64_t)i * D, k, D, vec) : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
#pragma unroll
                    for (int r = 0; r < RU; ++r) {
                        const int i = i0 + r * kWave;
                        if (i >= m) break;
                        const int j = i + W;
                        float d = INF;
                        if (j < n) {
                            float s = 0.0f;
#pragma unroll
                            for (int k = 0; k < NCH; ++k) {
                                const float4 c = cst[k * n + j];
                                float t = qv[r][k].x - c.x; s = __builtin_fmaf(t, t, s);
                                t = qv[r][k].y - c.y; s = __builtin_fmaf(t, t, s);
                                t = qv[r][k].z - c.z; s = __builtin_fmaf(t, t, s);
                                t = qv[r][k].w - c.w; s = __builtin_fmaf(t, t, s);
                            }
                            d = __builtin_sqrtf(s);
                        }
                        tdq[i].y = 2.0f * d;
                    }
                }
            }
            __syncthreads();
            float V[SLOTS], Y[SLOTS];
            uint32_t cm[SLOTS];  // running column minimum, >= 0 or +inf (no cell yet): kept as bits
            int32_t bias[SLOTS]; // bits: 0 for band offsets (k <= 2W), those of +inf past them
            bool istop[SLOTS];
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                V[s] = 0.0f; Y[s] = 0.0f; cm[s] = INF_BITS;
                bias[s] = lane + 64 * s < KB ? 0 : (int32_t)INF_BITS;
                istop[s] = lane + 64 * s == kt;
            }
            float acc = 0.0f;
            int exr = 0;         // staged query point of the next exact row (qex[i / P])

            // Row i with t = tdq[i].  GEN: test every lane for a cell of the candidate (first and
            // last rows); EXACT: an exact row.  Lanes that are not cells carry values that only ever
            // reach other non-cells (the cell below keeps the column) or the top offset, which
            // every row overwrites, so every lane evaluates the same arithmetic and only the column
            // minimum is masked (a safe value raised to +inf).
            auto row = [&](int i, float2 t, auto gen_tag, auto exact_tag) __attribute__((always_inline)) {
                constexpr bool GEN = decltype(gen_tag)::value;
                constexpr bool EXACT = decltype(exact_tag)::value;
                // row i-1 state of the same column (offset k+1); what lane 63 of the last slot
                // receives moves down only into non-cells or the top offset
                float Vn[SLOTS], Yn[SLOTS];
                uint32_t cmn[SLOTS];
                if (SLOTS == 1) {
                    Vn[0] = wave_rol1_f(V[0]);
                    Yn[0] = wave_rol1_f(Y[0]);
                    cmn[0] = wave_shl1_u32(0xffffffffu, cm[0]);
                } else {
                    Vn[0] = wave_shl1(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(V[SLOTS - 1]), 0)), V[0]);
                    Yn[0] = wave_shl1(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(Y[SLOTS - 1]), 0)), Y[0]);
                    cmn[0] = wave_shl1_u32((uint32_t)__builtin_amdgcn_readlane((int)cm[SLOTS - 1], 0), cm[0]);
                    Vn[SLOTS - 1] = wave_shl1(0.0f, V[SLOTS - 1]);
                    Yn[SLOTS - 1] = wave_shl1(0.0f, Y[SLOTS - 1]);
                    cmn[SLOTS - 1] = wave_shl1_u32(0xffffffffu, cm[SLOTS - 1]);
                }
                // the column at offset 0 of row i-1 is not in row i's band: its minimum is final
                // (lane 0 holds it and keeps the sum; the other lanes' sums are never read)
                {
                    const float lv = __uint_as_float(cm[0]);
                    const float leaving = GEN ? (cm[0] < INF_BITS ? lv : 0.0f) : lv;
                    acc = __builtin_fmaf(leaving, leaving, acc);
                }
                if (EXACT) {
#pragma unroll
                    for (int s = 0; s < SLOTS; ++s) {
                        const int jr = i - W + lane + 64 * s;
                        const int jc = GEN ? min(max(jr, 0), n - 1) : min(jr, n - 1);
                        const float4* qrow = qex + exr * NCH;
                        const float4* crow = cst + jc;
                        float sacc = 0.0f;
#pragma unroll
                        for (int k = 0; k < NCH; ++k) {
                            const float4 qv = qrow[k], cv = crow[k * n];
                            float d;
                            d = qv.x - cv.x; sacc = __builtin_fmaf(d, d, sacc);
                            d = qv.y - cv.y; sacc = __builtin_fmaf(d, d, sacc);
                            d = qv.z - cv.z; sacc = __builtin_fmaf(d, d, sacc);
                            d = qv.w - cv.w; sacc = __builtin_fmaf(d, d, sacc);
                        }
                        float lo, hi;
                        ti_exact_sides(sacc, lo, hi);
                        V[s] = lo + hi;
                        Y[s] = hi + hi;
                    }
                    ++exr;
                } else {
                    float v[SLOTS], y[SLOTS];
#pragma unroll
                    for (int s = 0; s < SLOTS; ++s) {
                        v[s] = umax_f(Vn[s], t.x);            // Eqs. 7-8: L + U
                        y[s] = Yn[s] + t.x;                   // Eq. 8, doubled
                    }
                    float tv = t.y, ty = t.y;
                    if (!TOP) {
                        // the top cell from its left neighbour (i, j-1) of this row, Eqs. 9-10
                        // (2 gamma_j of the top column j = i + W is the row's t.y)
                        const float vsel = (SLOTS > 1 && (kl >> 6) != 0) ? v[SLOTS - 1] : v[0];
                        const float ysel = (SLOTS > 1 && (kl >> 6) != 0) ? y[SLOTS - 1] : y[0];
                        const float Vl = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vsel), kl & 63));
                        const float Yl = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ysel), kl & 63));
                        tv = umax_f(Vl, t.y);
                        ty = Yl + t.y;
                    }
#pragma unroll
                    for (int s = 0; s < SLOTS; ++s) {
                        V[s] = istop[s] ? tv : v[s];
                        Y[s] = istop[s] ? ty : y[s];
                    }
                    if (!TOP && GEN && kt == 0) {
                        // no left neighbour (W = 0): the top cell is exact
                        const int j = i + W;
                        if (lane == 0 && j < n) {
                            float sacc = 0.0f;
                            for (int p = 0; p < D; ++p) {
                                const float d = qs[(int64_t)i * D + p] - cs[(int64_t)j * D + p];
                                sacc = __builtin_fmaf(d, d, sacc);
                            }
                            float lo, hi;
                            ti_exact_sides(sacc, lo, hi);
                            V[0] = lo + hi;
                            Y[0] = hi + hi;
                        }
                    }
                }
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    int32_t b = bias[s];
                    if (GEN) {
                        const int jr = i - W + lane + 64 * s;
                        b = (bias[s] == 0 && (unsigned)jr < (unsigned)n) ? 0 : (int32_t)INF_BITS;
                    }
                    // a safe lower bound of the Euclidean point distance clamped at 0, as bits: the
                    // signed maximum with 0 maps every negative value to 0; with the bits of +inf
                    // (a lane that is no cell) it gives +inf or more, which no column minimum takes
                    const float sv = __builtin_fmaf(-k1h, Y[s], V[s]);
                    cm[s] = min(cmn[s], (uint32_t)max(__float_as_int(sv), b));
                }
            };
            using T1 = std::integral_constant<bool, true>;
            using F0 = std::integral_constant<bool, false>;
            // Every loop reads the next row's values ahead; `since` counts the rows after the last
            // exact one (the exact rows are i = 0 and, for P > 0, the multiples of P).
            int i = 0;
            int since = 0;
            float2 tn = tdq[0];
            auto gen_row = [&]() __attribute__((always_inline)) {
                const float2 t = tn;
                tn = tdq[i + 1];
                if (i == 0 || since == 0) row(i, t, T1{}, T1{});
                else row(i, t, T1{}, F0{});
                since = (P > 0 && since + 1 == P) ? 0 : since + 1;
                ++i;
            };
            // non-exact rows up to `stop`: four, two, then one per step, with no test per row
            auto plain_rows = [&](int stop) __attribute__((always_inline)) {
                for (; i + 4 <= stop; i += 4) {
                    const float2 t1 = tdq[i + 1], t2 = tdq[i + 2], t3 = tdq[i + 3];
                    row(i, tn, F0{}, F0{});
                    row(i + 1, t1, F0{}, F0{});
                    row(i + 2, t2, F0{}, F0{});
                    tn = tdq[i + 4];
                    row(i + 3, t3, F0{}, F0{});
                }
                if (i + 2 <= stop) {
                    const float2 t1 = tdq[i + 1];
                    row(i, tn, F0{}, F0{});
                    tn = tdq[i + 2];
                    row(i + 1, t1, F0{}, F0{});
                    i += 2;
                }
                if (i < stop) {
                    const float2 t = tn;
                    tn = tdq[i + 1];
                    row(i, t, F0{}, F0{});
                    ++i;
                }
            };
            while (i < ib) gen_row();
            if (i < ie) {
                // between the edges: blocks of an exact row and the P - 1 rows after it
                int next = P > 0 ? i + (since == 0 ? 0 : P - since) : ie;   // the next exact row
                plain_rows(min(next, ie));
                while (i < ie) {
                    const float2 t = tn;
                    tn = tdq[i + 1];
                    row(i, t, F0{}, T1{});
                    ++i;
                    plain_rows(min(i + P - 1, ie));
                }
                since = P > 0 ? i % P : 1;
            }
            while (i < m) gen_row();
            // columns still in the band after the last row
            float tail = 0.0f;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int k = lane + 64 * s;
                const int j = m - 1 - W + k;
                if (k < KB && j >= 0 && j < n && cm[s] < INF_BITS) {
                    const float v = __uint_as_float(cm[s]);
                    tail += v * v;
                }
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) tail += __shfl_xor(tail, o);
            if (lane == 0) a.out_lb[(int64_t)q * a.cap + e] = rdown((double)(acc + tail) * defl);
            ++evaluated;
        }
    }
    if (a.evaluated && lane == 0 && evaluated) atomicAdd(a.evaluated, evaluated);
}

// ---------------------------------------------------------------- routing
// After an advanced bound: lb = max(bound so far, new bound) (a value < 0
// means "not evaluated").  Pairs with lb * keep > bsf are skipped (counted),
// the others go to the next bound's list (with their lb) when that bound is
// deployed for them, else to the DTW list.  Wave ballot + one atomic per
// wave and output list.
__global__ __launch_bounds__(256) void k_route(RouteArgs a) {
    const int q = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int cnt = a.in_cnt[q];
    const bool valid = e < cnt;
    const double bsf = (double)key_bsf(a.key + (int64_t)q * kKeyStride);
    int ref = 0;
    float lb = 0.0f;
    if (valid) {
        ref = (int)a.in_list[(int64_t)q * a.cap + e];
        const float prev = a.lb_prev ? a.lb_prev[(int64_t)q * a.cap + e] : a.lb_mv[(int64_t)q * a.nc + ref];
        const float nb = a.lb_new ? a.lb_new[(int64_t)q * a.cap + e] : -1.0f;   // null: not evaluated
        lb = nb > prev ? nb : prev;
    }
    const bool pruned = valid && ((double)lb * a.keep > bsf);
    const bool next = valid && !pruned && a.next_list && ((double)lb > a.next_e2 * bsf);
    const bool dtw = valid && !pruned && !next;
    const uint64_t bd = __ballot(dtw), bn = __ballot(next), bp = __ballot(pruned);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int based = 0, basen = 0;
    if (lane == 0) {
        if (bd) based = atomicAdd(&a.dtw_cnt[q], __popcll(bd));
        if (bn) basen = atomicAdd(&a.next_cnt[q], __popcll(bn));
        if (bp) atomicAdd(&a.pruned[q], __popcll(bp));
    }
    based = __shfl(based, 0);
    basen = __shfl(basen, 0);
    if (dtw) a.dtw_list[(int64_t)q * a.cap + based + __popcll(bd & below)] = (uint32_t)ref;
    if (next) {
        const int pos = basen + __popcll(bn & below);
        a.next_list[(int64_t)q * a.cap + pos] = (uint32_t)ref;
        a.next_lb[(int64_t)q * a.cap + pos] = lb;
    }
}

// ----------------------------------------------------------------- launch
hipError_t launch_query_steps(const float* Q, int nq, int m, int D, float* delta, hipStream_t s) {
    const int64_t total = (int64_t)nq * m;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_query_steps, dim3(blocks), dim3(256), 0, s, Q, nq, m, D, delta);
    return hipGetLastError();
}

size_t pc_boxes_lds_bytes(int max_pts, int K, int D) {
    return (size_t)max_pts * (8 + 4) + (size_t)K * D * 2 * 4 + 16;
}

hipError_t launch_pc_boxes(const PcArgs& a, hipStream_t s) {
    const size_t lds = pc_boxes_lds_bytes(a.max_pts, a.K, a.D);
    // the boxed series in launches of at most 65535 (the grid's y limit)
    for (int q0 = 0; q0 < a.nq; q0 += 65535) {
        PcArgs b = a;
        b.nq = std::min(65535, a.nq - q0);
        b.Q = a.Q + (int64_t)q0 * a.m * a.D;
        b.boxes = a.boxes + (int64_t)q0 * a.ngroups * a.K * a.D * 2;
        b.nbox = a.nbox + (int64_t)q0 * a.ngroups;
        hipLaunchKernelGGL(k_pc_boxes, dim3(a.ngroups, b.nq), dim3(64), lds, s, b);
    }
    return hipGetLastError();
}

template <int NCH, int DC, int PPS>
static void launch_pc_lanes(const PcArgs& a, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_lb_pc_lanes<NCH, DC, PPS>), dim3(nblocks), dim3(64), 0, s, a);
}

// Narrow points take a whole group per step when the group length is a multiple of six, else
// three points when it is a multiple of three (more loads in flight, no idle slot in a group),
// else two; wide points two.
template <int NCH, int DC>
static void launch_pc_lanes_dc(const PcArgs& a, int nblocks, hipStream_t s) {
    if (NCH <= 2 && a.w % 6 == 0) launch_pc_lanes<NCH, DC, NCH <= 2 ? 6 : 2>(a, nblocks, s);
    else if (NCH <= 2 && a.w % 3 == 0) launch_pc_lanes<NCH, DC, NCH <= 2 ? 3 : 2>(a, nblocks, s);
    else launch_pc_lanes<NCH, DC, 2>(a, nblocks, s);
}

// D fixed at compile time for points of up to 8 dimensions; wider points whole chunks or D at
// run time
template <int DC>
static void launch_pc_pts(const PcArgs& a, int nblocks, hipStream_t s) {
    if (a.K <= 4) hipLaunchKernelGGL((k_lb_pc_pts<DC, 4>), dim3(nblocks), dim3(64), 0, s, a);
    else if (a.K <= 6) hipLaunchKernelGGL((k_lb_pc_pts<DC, 6>), dim3(nblocks), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((k_lb_pc_pts<DC, 8>), dim3(nblocks), dim3(64), 0, s, a);
}

template <int NCH>
static void launch_lb_pc_lanes_nch(const PcArgs& a, int nblocks, hipStream_t s) {
    // narrow points of short series: lanes over the candidate's points
    if (NCH == 1 && a.w % 3 == 0 && a.n <= 3 * kWave && a.K <= 8) {
        switch (a.D) {
            case 1: launch_pc_pts<1>(a, nblocks, s); return;
            case 2: launch_pc_pts<2>(a, nblocks, s); return;
            case 3: launch_pc_pts<3>(a, nblocks, s); return;
            default: launch_pc_pts<4>(a, nblocks, s); return;
        }
    }
    if constexpr (NCH <= 2) {
        switch (a.D - 4 * (NCH - 1)) {
            case 1: launch_pc_lanes_dc<NCH, 4 * NCH - 3>(a, nblocks, s); break;
            case 2: launch_pc_lanes_dc<NCH, 4 * NCH - 2>(a, nblocks, s); break;
            case 3: launch_pc_lanes_dc<NCH, 4 * NCH - 1>(a, nblocks, s); break;
            default: launch_pc_lanes_dc<NCH, 4 * NCH>(a, nblocks, s); break;
        }
    } else {
        if (a.D == 4 * NCH) launch_pc_lanes_dc<NCH, 4 * NCH>(a, nblocks, s);
        else launch_pc_lanes_dc<NCH, 0>(a, nblocks, s);
    }
}

hipError_t launch_lb_pc_lanes(const PcArgs& a, int nblocks, hipStream_t s) {
    switch (nch_pad(a.D)) {
        case 1: launch_lb_pc_lanes_nch<1>(a, nblocks, s); break;
        case 2: launch_lb_pc_lanes_nch<2>(a, nblocks, s); break;
        case 3: launch_lb_pc_lanes_nch<3>(a, nblocks, s); break;
        case 4: launch_lb_pc_lanes_nch<4>(a, nblocks, s); break;
        case 6: launch_lb_pc_lanes_nch<6>(a, nblocks, s); break;
        case 8: launch_lb_pc_lanes_nch<8>(a, nblocks, s); break;
        case 12: launch_lb_pc_lanes_nch<12>(a, nblocks, s); break;
        case 16: launch_lb_pc_lanes_nch<16>(a, nblocks, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lb_pc(const PcArgs& a, int nblocks, hipStream_t s) {
    if (a.D <= 4) hipLaunchKernelGGL(k_lb_pc<4>, dim3(nblocks), dim3(64), 0, s, a);
    else if (a.D <= 8) hipLaunchKernelGGL(k_lb_pc<8>, dim3(nblocks), dim3(64), 0, s, a);
    else if (a.D <= 16) hipLaunchKernelGGL(k_lb_pc<16>, dim3(nblocks), dim3(64), 0, s, a);
    else if (a.D <= 32) hipLaunchKernelGGL(k_lb_pc<32>, dim3(nblocks), dim3(64), 0, s, a);
    else hipLaunchKernelGGL(k_lb_pc<64>, dim3(nblocks), dim3(64), 0, s, a);
    return hipGetLastError();
}

size_t ti_lds_bytes(int m, int n, int D, int P, int W) {
    if (2 * W + 1 > 2 * kWave) return ti_cols_lds_bytes(m);
    const size_t nch = (size_t)nch_pad(D);
    return ((size_t)n * nch + (size_t)ti_exact_rows(m, P) * nch) * 16 + (size_t)(m + 2) * 8 + 16;
}

template <int SLOTS, int NCH>
static void launch_lb_ti_nch(const TiArgs& a, int nblocks, size_t lds, hipStream_t s) {
    if (a.top) hipLaunchKernelGGL((k_lb_ti<SLOTS, true, NCH>), dim3(nblocks), dim3(64), lds, s, a);
    else hipLaunchKernelGGL((k_lb_ti<SLOTS, false, NCH>), dim3(nblocks), dim3(64), lds, s, a);
}

template <int SLOTS>
static hipError_t launch_lb_ti_slots(const TiArgs& a, int nblocks, size_t lds, hipStream_t s) {
    switch (nch_pad(a.D)) {
        case 1: launch_lb_ti_nch<SLOTS, 1>(a, nblocks, lds, s); break;
        case 2: launch_lb_ti_nch<SLOTS, 2>(a, nblocks, lds, s); break;
        case 3: launch_lb_ti_nch<SLOTS, 3>(a, nblocks, lds, s); break;
        case 4: launch_lb_ti_nch<SLOTS, 4>(a, nblocks, lds, s); break;
        case 6: launch_lb_ti_nch<SLOTS, 6>(a, nblocks, lds, s); break;
        case 8: launch_lb_ti_nch<SLOTS, 8>(a, nblocks, lds, s); break;
        case 12: launch_lb_ti_nch<SLOTS, 12>(a, nblocks, lds, s); break;
        case 16: launch_lb_ti_nch<SLOTS, 16>(a, nblocks, lds, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lb_ti(const TiArgs& a, int nblocks, hipStream_t s) {
    // bands of up to 128 offsets: one or two offsets per lane; wider: the column mapping
    if (2 * a.W + 1 > 2 * kWave) return launch_lb_ti_cols(a, nblocks, s);
    const size_t lds = ti_lds_bytes(a.m, a.n, a.D, a.P, a.W);
    return 2 * a.W + 1 <= 64 ? launch_lb_ti_slots<1>(a, nblocks, lds, s) : launch_lb_ti_slots<2>(a, nblocks, lds, s);
}

hipError_t launch_route(const RouteArgs& a, int max_in, hipStream_t s) {
    if (max_in <= 0) return hipSuccess;
    dim3 grid((max_in + 255) / 256, a.nq);
    hipLaunchKernelGGL(k_route, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// items per query for a list processed in chunks of `per` entries
__global__ __launch_bounds__(1024) void k_list_scan(const int32_t* cnt, int cnt_uniform, int nq, int per,
                                                    int32_t* prefix, int32_t* counter) {
    __shared__ int32_t part[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) { carry = 0; prefix[0] = 0; *counter = 0; }
    __syncthreads();
    for (int base = 0; base < nq; base += 1024) {
        const int q = base + threadIdx.x;
        const int c = cnt_uniform > 0 ? cnt_uniform : (q < nq ? cnt[q] : 0);
        part[threadIdx.x] = q < nq ? (c + per - 1) / per : 0;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int add = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (q < nq) prefix[q + 1] = carry + part[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_list_items(const int32_t* __restrict__ prefix, int nq,
                                                    int32_t* __restrict__ item_query) {
    for (int q = blockIdx.x; q < nq; q += gridDim.x) {
        const int b = prefix[q], e = prefix[q + 1];
        for (int t = b + threadIdx.x; t < e; t += blockDim.x) item_query[t] = q;
    }
}

hipError_t launch_list_items(const int32_t* cnt, int cnt_uniform, int nq, int per, int32_t* prefix,
                             int32_t* item_query, int32_t* counter, hipStream_t s) {
    hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(1024), 0, s, cnt, cnt_uniform, nq, per, prefix, counter);
    hipLaunchKernelGGL(k_list_items, dim3(nq < 4096 ? nq : 4096), dim3(256), 0, s, prefix, nq, item_query);
    return hipGetLastError();
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int n) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) dst[t] = src[t];
}

hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_i32, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256), 0, s, src,
                       dst, n);
    return hipGetLastError();
}

}  // namespace tcdtw
