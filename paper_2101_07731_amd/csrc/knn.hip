// 1-NN search kernels for gfx950 (uniform query and candidate lengths):
// query envelope, LB_MV, best-so-far seeding, ballot compaction, DTW of the
// survivors with early abandoning (persistent work queue), float64
// re-scoring of near-tie finalists.
//
// Soundness of every float32 decision:
//   * a bound is a sum of N non-negative float32 terms accumulated by fused
//     multiply-add; scaled by (1 - (N+3) u) and rounded down it never
//     exceeds the exact bound (u = 2^-24);
//   * the float32 DP value D_f of a band cell satisfies
//     D_f / (1 + g) <= D <= D_f / (1 - g) with g = (m + n + D) u (path
//     length plus point-cost roundings), so bsf_up = D_f / (1 - g)
//     (rounded up) never undercuts the exact DTW of a candidate, and a
//     pair is abandoned only when D_f / (1 + g) > bsf_up on two
//     consecutive anti-diagonals;
//   * candidates whose D_f lies within (1 + g) / (1 - g) of the smallest
//     are re-scored in float64, in the order of a plain FP64 evaluation.
#include <algorithm>

#include "dtw_core.h"
#include "internal.h"

namespace tcdtw {

// ------------------------------------------------------------------ setup
__global__ void k_knn_init(int nq, unsigned long long* key, int32_t* cnt, int32_t* gcnt,
                           int32_t* counters, unsigned long long* stats, int32_t* c0, int32_t* c1,
                           int32_t* c2, unsigned long long* topk, int k) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (topk)
        for (int64_t x = t; x < (int64_t)nq * k; x += (int64_t)gridDim.x * blockDim.x)
            topk[x] = 0x7f800000ffffffffull;
    for (int q = t; q < nq; q += gridDim.x * blockDim.x) {
        key[(int64_t)q * kKeyStride] = 0x7f800000ffffffffull;     // best-so-far +inf, no candidate yet
        cnt[q] = 0;
        if (gcnt) gcnt[q] = 0;
        if (c0) c0[q] = 0;
        if (c1) c1[q] = 0;
        if (c2) c2[q] = 0;
    }
    if (t < kNumCounters) counters[t] = 0;
    if (t < kNumStats) stats[t] = 0;
}

// Query envelope (Sec. 3, LB_MV): for candidate position j, the max / min
// of each query dimension over query rows [j - W, j + W] clipped to [0, m).
// Layout env[qtile][e][QT][2] (e = j*D + p), so one 64-byte scalar load
// gives the (U, L) pairs of a tile's QT queries for one element.
__global__ void k_envelope(const float* __restrict__ Q, int nq, int m, int n, int D, int W,
                           float* __restrict__ env, uint32_t* status) {
    bool bad = false;   // a non-finite query value (the minimum and maximum skip NaN)
    const int E = n * D;
    const int Ep = (E + 3) / 4 * 4;     // padded like the candidate tiles; padding gets (+inf, -inf)
    const int nqt = (nq + kQT - 1) / kQT;
    const int64_t total = (int64_t)nqt * kQT * Ep;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(idx % Ep);
        const int q = (int)(idx / Ep);
        const int j = e / D, p = e - j * D;
        float U = __builtin_inff(), L = -__builtin_inff();
        if (q < nq && e < E) {
            const int i0 = max(0, j - W), i1 = min(m - 1, j + W);
            const float* s = Q + (int64_t)q * m * D + p;
            U = s[(int64_t)i0 * D];
            L = U;
            bad |= !__builtin_isfinite(U);
#pragma unroll 8
            for (int i = i0 + 1; i <= i1; ++i) {    // unrolled: eight loads in flight
                const float v = s[(int64_t)i * D];
                U = __builtin_fmaxf(U, v);
                L = __builtin_fminf(L, v);
                bad |= !__builtin_isfinite(v);
            }
        }
        float* o = env + (((int64_t)(q / kQT) * Ep + e) * kQT + (q % kQT)) * 2;
        o[0] = U;
        o[1] = L;
    }
    if (bad && status) atomicOr(status, kStatusNonFiniteQuery);
}

// LB_MV (Sec. 3, squared form) of up to kQT queries against 64 candidates
// per wave.  Candidates come from the element-major tiles (a lane reads
// four elements of its candidate with one 16-byte load), the envelope from
// wave-uniform scalar loads.  The term of element e is t^2 with
// t = c - med3(c, L, U): c - U above the envelope, -(L - c) below it, 0
// inside -- the float32 values of max(c - U, L - c, 0), one operation fewer.
// QT: query slots of the tile that are evaluated (kQT, or fewer when the
// whole batch has fewer queries); LD: loads in flight per lane (deeper when
// the arithmetic per element is light and HBM is the bound).
// With few query tiles (queries arriving one at a time) a launch over
// candidate tiles alone would hold too few waves to keep HBM busy, so the
// elements are split into gridDim.z segments of seg4 groups of four: each
// segment writes its raw partial sums to `part` ([z][nq][nc]) and k_lb_sum
// adds them in segment order.  (A last-arriving block adding them instead
// would need a device-scope release per block, which writes back the
// XCD's whole L2.)  The deflation covers any summation order of the E
// terms.
// CPL: candidate tiles per wave.  With four or more query slots a wave
// takes two tiles, so each envelope value moved into a vector register
// serves two med3 operations (3.5 VALU operations per element, query and
// candidate instead of 4).
template <int QT, int LD = (QT <= 2 ? 4 : 2), int CPL = (QT >= 4 ? 2 : 1)>
__global__ __launch_bounds__(256) void k_lb_mv(const float* __restrict__ tiles, int ntiles, int E,
                                               const float* __restrict__ env, int nq, int nc,
                                               double deflate, float* __restrict__ lb, int seg4,
                                               float* __restrict__ part) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile0 = (blockIdx.x * 4 + wave) * CPL;
    if (tile0 >= ntiles) return;
    const int qt = blockIdx.y;
    const int E4 = (E + 3) / 4, Ep = 4 * E4;
    const int f0 = blockIdx.z * seg4, f1 = min(E4, f0 + seg4);
    const float4* __restrict__ cp[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {   // a tile past the end reads the first one again (its results are dropped)
        const int t = tile0 + c < ntiles ? tile0 + c : tile0;
        cp[c] = reinterpret_cast<const float4*>(tiles) + (int64_t)t * E4 * 64 + lane;
    }
    const float* __restrict__ ep = env + (int64_t)qt * Ep * kQT * 2;
    float acc[CPL][QT];
#pragma unroll
    for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int k = 0; k < QT; ++k) acc[c][k] = 0.0f;
    auto term = [&](const float (&cv)[CPL], int e) __attribute__((always_inline)) {
        const float* __restrict__ u = ep + (int64_t)e * kQT * 2;
#pragma unroll
        for (int k = 0; k < QT; ++k) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const float t = cv[c] - __builtin_amdgcn_fmed3f(cv[c], u[2 * k + 1], u[2 * k]);
                acc[c][k] = __builtin_fmaf(t, t, acc[c][k]);
            }
        }
    };
    auto terms4 = [&](const float4 (&a)[CPL], int e) __attribute__((always_inline)) {
        float x[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) x[c] = a[c].x;
        term(x, e);
#pragma unroll
        for (int c = 0; c < CPL; ++c) x[c] = a[c].y;
        term(x, e + 1);
#pragma unroll
        for (int c = 0; c < CPL; ++c) x[c] = a[c].z;
        term(x, e + 2);
#pragma unroll
        for (int c = 0; c < CPL; ++c) x[c] = a[c].w;
        term(x, e + 3);
    };
    int f = f0;
    for (; f + LD <= f1; f += LD) {   // LD 16-byte loads (4 LD elements) per tile in flight per lane
        float4 a[LD][CPL];
#pragma unroll
        for (int i = 0; i < LD; ++i)
#pragma unroll
            for (int c = 0; c < CPL; ++c) a[i][c] = cp[c][(int64_t)(f + i) * 64];
#pragma unroll
        for (int i = 0; i < LD; ++i) terms4(a[i], 4 * (f + i));
    }
    for (; f < f1; ++f) {
        float4 a[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) a[c] = cp[c][(int64_t)f * 64];
        terms4(a, 4 * f);
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int r = (tile0 + c) * 64 + lane;
        if (tile0 + c >= ntiles || r >= nc) continue;
#pragma unroll
        for (int k = 0; k < QT; ++k) {
            const int q = qt * kQT + k;
            if (q >= nq) continue;
            if (gridDim.z == 1) lb[(int64_t)q * nc + r] = round_down_f((double)acc[c][k] * deflate);
            else part[((int64_t)blockIdx.z * nq + q) * nc + r] = acc[c][k];
        }
    }
}

// Sum of the segment partials in segment order; the loads of eight
// segments are issued together.
__global__ __launch_bounds__(256) void k_lb_sum(const float* __restrict__ part, int nseg, int64_t n,
                                                double deflate, float* __restrict__ lb) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        int z = 0;
        for (; z + 8 <= nseg; z += 8) {
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = part[(int64_t)(z + i) * n + t];
#pragma unroll
            for (int i = 0; i < 8; ++i) s += v[i];
        }
        for (; z < nseg; ++z) s += part[(int64_t)z * n + t];
        lb[t] = round_down_f((double)s * deflate);
    }
}

// Seeds: the R candidates with the smallest LB_MV of each query (one wave
// per query; ties between equal bounds in any order).
template <int RMAX>
__global__ __launch_bounds__(64) void k_topr(const float* __restrict__ lb, int nc, int R,
                                             const int32_t* __restrict__ q_cb, const int32_t* __restrict__ q_ce,
                                             int32_t* __restrict__ seeds) {
    const int q = blockIdx.x, lane = threadIdx.x;
    float v[RMAX];
    int id[RMAX];
#pragma unroll
    for (int k = 0; k < RMAX; ++k) { v[k] = __builtin_inff(); id[k] = 0x7fffffff; }
    const float* row = lb + (int64_t)q * nc;
    auto insert = [&](float x, int xi) __attribute__((always_inline)) {
        if (x < v[RMAX - 1]) {
#pragma unroll
            for (int k = 0; k < RMAX; ++k) {   // insertion into the sorted local list
                if (x < v[k]) {
                    const float tv = v[k]; const int ti = id[k];
                    v[k] = x; id[k] = xi;
                    x = tv; xi = ti;
                }
            }
        }
    };
    // with banks of several dims only the query's bank [cb, ce) holds candidates
    const int cb = q_cb ? q_cb[q] : 0, ce = q_cb ? q_ce[q] : nc;
    int r = cb + lane;
    for (; r + 3 * kWave < ce; r += 4 * kWave) {   // four loads in flight per lane
        float x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = row[r + u * kWave];
#pragma unroll
        for (int u = 0; u < 4; ++u) insert(x[u], r + u * kWave);
    }
    for (; r < ce; r += kWave) insert(row[r], r);
    for (int k = 0; k < R; ++k) {
        float bv = v[0];
        int bi = id[0];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const float ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov < bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (id[0] == bi) {
#pragma unroll
            for (int t = 0; t + 1 < RMAX; ++t) { v[t] = v[t + 1]; id[t] = id[t + 1]; }
            v[RMAX - 1] = __builtin_inff();
            id[RMAX - 1] = 0x7fffffff;
        }
        if (lane == 0) seeds[(int64_t)q * R + k] = (bi < nc) ? bi : -1;
    }
}

// Compaction (Sec. 2 DTW-NN filtering; Sec. 6 selective deployment): every
// non-seed pair whose bound, shrunk by the prune margin, exceeds the
// query's best-so-far is skipped; the rest goes to the DTW list, or to the
// advanced-bound list when gating is on and LB_MV > e^2 bsf.  A block of
// 256 threads covers kCompactPer candidates of one query (four per
// thread): wave ballots, a prefix over the block's waves and rounds in
// LDS, and one atomic per block and list (a counter per query takes many
// fewer atomics than with one per wave).
constexpr int kCompactRounds = 4;
constexpr int kCompactPer = 256 * kCompactRounds;

__global__ __launch_bounds__(256) void k_compact(const float* __restrict__ lb, int nc,
                                                 const int32_t* __restrict__ q_cb, const int32_t* __restrict__ q_ce,
                                                 const int32_t* __restrict__ seeds, int R,
                                                 const unsigned long long* __restrict__ key,
                                                 double keep, double gate_e2, int use_gate,
                                                 uint32_t* __restrict__ list, int32_t* cnt,
                                                 uint32_t* __restrict__ glist, int32_t* gcnt, int cap,
                                                 unsigned long long* stats) {
    constexpr int NW = 4;   // waves per block
    __shared__ int sd[kCompactRounds][NW], sg[kCompactRounds][NW];
    __shared__ int base_d, base_g;
    const int q = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double bsf = (double)bsf_from_key(key[(int64_t)q * kKeyStride]);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t bd[kCompactRounds], bg[kCompactRounds];
    bool todtw[kCompactRounds], gated[kCompactRounds];
#pragma unroll
    for (int it = 0; it < kCompactRounds; ++it) {
        const int r = blockIdx.x * kCompactPer + it * 256 + threadIdx.x;
        // with banks of several dims only the query's own bank holds candidates
        const bool valid = r < nc && (!q_cb || (r >= q_cb[q] && r < q_ce[q]));
        bool seed = false;
        for (int k = 0; k < R; ++k) seed |= (seeds[(int64_t)q * R + k] == r);
        const double v = (valid && lb) ? (double)lb[(int64_t)q * nc + r] : 0.0;
        const bool live = valid && !seed;
        const bool pruned = live && (v * keep > bsf);
        gated[it] = live && !pruned && use_gate && (v > gate_e2 * bsf);
        todtw[it] = live && !pruned && !gated[it];
        bd[it] = __ballot(todtw[it]);
        bg[it] = __ballot(gated[it]);
        if (lane == 0) {
            sd[it][wave] = __popcll(bd[it]);
            sg[it][wave] = __popcll(bg[it]);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // exclusive prefix in (round, wave) order, then one atomic per list
        int td = 0, tg = 0;
        for (int it = 0; it < kCompactRounds; ++it)
            for (int w = 0; w < NW; ++w) {
                const int cd = sd[it][w], cg = sg[it][w];
                sd[it][w] = td; sg[it][w] = tg;
                td += cd; tg += cg;
            }
        base_d = td ? atomicAdd(&cnt[q], td) : 0;
        base_g = tg ? atomicAdd(&gcnt[q], tg) : 0;
    }
    __syncthreads();
    (void)stats;   // the pruned count is derived per query at the end (pairs - seeds - listed)
#pragma unroll
    for (int it = 0; it < kCompactRounds; ++it) {
        const uint32_t r = (uint32_t)(blockIdx.x * kCompactPer + it * 256 + threadIdx.x);
        if (todtw[it]) list[(int64_t)q * cap + base_d + sd[it][wave] + __popcll(bd[it] & below)] = r;
        if (gated[it]) glist[(int64_t)q * cap + base_g + sg[it][wave] + __popcll(bg[it] & below)] = r;
    }
}

// prefix[q+1] = prefix[q] + ceil(cnt[q] / P); also clears the work counter.
__global__ __launch_bounds__(1024) void k_chunk_scan(const int32_t* cnt, int cnt_uniform, int nq, int P,
                                                     int32_t* prefix, int32_t* counter) {
    __shared__ int32_t part[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) { carry = 0; prefix[0] = 0; *counter = 0; }
    __syncthreads();
    for (int base = 0; base < nq; base += 1024) {
        const int q = base + threadIdx.x;
        const int c = cnt_uniform > 0 ? cnt_uniform : (q < nq ? cnt[q] : 0);
        const int v = q < nq ? (c + P - 1) / P : 0;
        part[threadIdx.x] = v;
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

// item_query[item] = q for the work items of query q (one block per query).
__global__ __launch_bounds__(256) void k_item_map(const int32_t* __restrict__ prefix, int nq,
                                                  int32_t* __restrict__ item_query) {
    for (int q = blockIdx.x; q < nq; q += gridDim.x) {
        const int b = prefix[q], e = prefix[q + 1];
        for (int t = b + threadIdx.x; t < e; t += blockDim.x) item_query[t] = q;
    }
}

// --------------------------------------------------------------- DTW lists
// A wave takes work items (query q, chunk of P list entries) from a global
// counter until none are left: persistent waves balance the uneven
// per-query list lengths.  The query is staged once per item group, the P
// candidates of the chunk share the wave (diagonal mapping) or the wave
// runs one pair (row mapping, P = 1).
__device__ __forceinline__ int find_query(const int32_t* prefix, int nq, int item) {
    int lo = 0, hi = nq;   // largest q with prefix[q] <= item
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

// k > 1: the query's k slots hold the packed keys of k distinct computed
// candidates (initially +inf); a new key replaces the largest slot when it
// is smaller (compare-and-swap, retried while other inserts change the
// slots: every failure is another insert's success, so the loop ends).
// The query's threshold key then drops to the largest slot: an upper bound
// of the k-th smallest exact distance, since every slot bounds a distinct
// candidate's distance from above.  Wave-cooperative (the whole wave calls
// it with the same arguments): lane i reads slot i, so a pass over the
// slots is one round trip of coherent loads.
__device__ __forceinline__ void topk_insert_wave(unsigned long long* slots, int K, unsigned long long x,
                                                 unsigned long long* thr) {
    const int lane = threadIdx.x & 63;
    auto wave_max = [&](unsigned long long& v, int& at) __attribute__((always_inline)) {
        v = lane < K ? __hip_atomic_load(slots + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
        at = lane;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const unsigned long long ov = __shfl_xor(v, o);
            const int oa = __shfl_xor(at, o);
            if (ov > v || (ov == v && oa < at)) { v = ov; at = oa; }
        }
    };
    // Every value that decides an exit is read from lane 0 into scalar
    // registers, so both exits are uniform branches (a loop exit on a
    // shuffled vector value may be compiled as divergent, leaving lanes
    // 1..63 spinning on the result of a parked lane 0).
    x = readlane_u64(x);
    for (;;) {
        unsigned long long mx;
        int mi;
        wave_max(mx, mi);
        mx = readlane_u64(mx);
        mi = __builtin_amdgcn_readlane(mi, 0);
        if (x >= mx) return;
        unsigned long long old = 0;
        if (lane == 0) old = atomicCAS(slots + mi, mx, x);
        if (readlane_u64(old) == mx) break;
    }
    unsigned long long m2;
    int at;
    wave_max(m2, at);
    if (lane == 0) atomicMin(thr, m2);
}

// Publishes an upper bound of the exact DTW of (q, ref), D <= v / (1 - gamma),
// as the query's best-so-far key (1-NN; one lane) or into its k best (k-NN;
// the whole wave with the same arguments).
__device__ __forceinline__ unsigned long long dist_key(float v, float gamma, int ref) {
    const float up = round_up_pos((double)v / (1.0 - (double)gamma));
    return ((unsigned long long)__float_as_uint(up) << 32) | (uint32_t)ref;
}
__device__ __forceinline__ void publish(const KnnDtwArgs& a, int q, int ref, float v, float gamma) {
    atomicMin(&a.key[(int64_t)q * kKeyStride], dist_key(v, gamma, ref));
}

// Diagonal mapping with ring buffers: each staged series keeps only RS
// consecutive positions (slot = position mod RS).  The live window of a
// round is about W + 2 positions; every RF = RS / 4 rounds the RF positions
// that fell behind are overwritten with the next ones, loaded into
// registers one refill ahead.  Series 0 is the query, series 1 + g the
// candidate of group g.
// Rounds between early-abandon checks.
constexpr int kCheckRounds = 32;

// NPASS: 64-lane passes of one refill ((1 + P) * RF positions), so that the
// prefetch registers are only as many as the launch needs.
// INDEP: independent DTW (DTW_I): one DP value per dimension and lane, the
// pair's distance the sum over the dimensions; groups are a power of two
// wide (the abandon test reduces within a group by xor shuffles).
template <int NCH, bool WODD, int RS, int NPASS, bool INDEP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NCH <= 2 && NPASS <= 2 && !INDEP ? 4 : 1))) void k_knn_dtw_ring(KnnDtwArgs a) {
    constexpr int NV = INDEP ? 4 * NCH : 1;   // DP values per lane and slot
    constexpr int RF = RS / 4, STR = RS;
    constexpr int MAXPASS = NPASS;
    const int lane = threadIdx.x;
    DiagGeom g;
    g.init(a.m, a.n, a.W);
    const int G = g.G, h = g.h, R = g.R, P = a.P, W = a.W, GS = a.gs;
    const int per_series = NCH * STR;
    const int grp = lane / GS;
    const int lg = lane - grp * GS;
    const bool pad = lg >= G;   // padding lane of a group (see knn_lane_stride)
    const int total = a.prefix[a.nq];
    unsigned long long w_started = 0, w_aband = 0, w_cells = 0;
    for (;;) {
        const int item = wave_next_item(a.counter);
        if (item >= total) break;
        const int q = a.item_query[item];
        const int chunk = item - a.prefix[q];
        const int base = chunk * P;
        const int np = min(P, a.cnt_uniform > 0 ? a.cnt_uniform - base : a.cnt[q] - base);
        const int nser = 1 + np;
        const float* qsrc = a.Q + (int64_t)q * a.m * a.D;
        auto series_src = [&](int s) __attribute__((always_inline)) -> const float* {
            if (s == 0) return qsrc;
            const int ref = (int)a.list[(int64_t)q * a.cap + base + s - 1];
            return a.C + (int64_t)(ref < 0 ? 0 : ref) * a.n * a.D;
        };
        // point of position pos of series s (outside the series: +inf for the
        // query, -inf for a candidate, so that those cells cost +inf)
        auto fetch = [&](int s, int pos, float4 (&v)[NCH]) __attribute__((always_inline)) {
            if (s == 0) load_point<NCH>(qsrc, a.m, a.D, pos + g.qfirst(), __builtin_inff(), v);
            else load_point<NCH>(series_src(s), a.n, a.D, pos + g.cfirst(), -__builtin_inff(), v);
        };
        auto put = [&](int s, int pos, const float4 (&v)[NCH]) __attribute__((always_inline)) {
            const int slot = pos & (RS - 1);
#pragma unroll
            for (int k = 0; k < NCH; ++k) lds4[s * per_series + k * STR + slot] = v[k];
        };
        __syncthreads();
        // initial positions 0 .. RS-1 of every series
        for (int x = lane; x < nser * RS; x += kWave) {
            float4 v[NCH];
            const int s = x / RS, pos = x - (x / RS) * RS;
            fetch(s, pos, v);
            put(s, pos, v);
        }
        // prefetch of the first refill: positions RS .. RS+RF-1
        float4 pf[MAXPASS][NCH];
#pragma unroll
        for (int p = 0; p < MAXPASS; ++p) {
            const int x = p * kWave + lane;
            if (x < nser * RF) fetch(x / RF, RS + (x % RF), pf[p]);
        }
        __syncthreads();

        const bool spare = grp >= np;
        const int gsrc = spare ? 0 : grp;
        // Band-edge kills (one per parity) also isolate neighbouring groups;
        // padding lanes and lanes of absent pairs hold +inf on the killed
        // diagonal, which is the only one their neighbours read.
        const bool kill_e = WODD && (lg == 0 || spare || pad);
        const bool kill_o = !WODD && (lg == G - 1 || spare || pad);
        const int qbase = 0;
        const int cbase = (1 + gsrc) * per_series;
        float vE[NV], vO[NV];
#pragma unroll
        for (int p = 0; p < NV; ++p) {
            vE[p] = (!spare && lg == h) ? 0.0f : __builtin_inff();
            vO[p] = __builtin_inff();
        }
        auto step = [&](const float4 (&qv)[NCH], const float4 (&ci)[NCH], const float4 (&co)[NCH])
                        __attribute__((always_inline)) {
            if constexpr (INDEP) diag_steps_indep<NCH, WODD>(qv, ci, co, kill_e, kill_o, vE, vO);
            else diag_steps_rot<NCH, WODD>(qv, ci, co, kill_e, kill_o, vE[0], vO[0]);
        };
        const uint64_t gbits = (G >= 64) ? ~0ull : ((1ull << G) - 1);
        uint64_t valid_mask = 0;
        for (int gg = 0; gg < np; ++gg) valid_mask |= gbits << (gg * GS);
        const uint64_t gm = spare ? 0ull : gbits << (grp * GS);
        bool aband = false;
        const bool abandon = a.abandon != 0;
        // the best-so-far is read by a coherent (slow) load whose value is first needed at
        // the first check: nothing waits for it at the start of the item
        unsigned long long pend = 0;
        if (abandon) pend = __hip_atomic_load(a.key + (int64_t)q * kKeyStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // Round r reads query position r + W - lg and candidate positions
        // r + lg (cin, the previous round's cout) and r + lg + 1 (cout).
        auto ldq = [&](int rr, float4 (&v)[NCH]) __attribute__((always_inline)) {
            const int sl = (rr + W - lg) & (RS - 1);
#pragma unroll
            for (int k = 0; k < NCH; ++k) v[k] = lds4[qbase + sl + k * STR];
        };
        auto ldc = [&](int pos, float4 (&v)[NCH]) __attribute__((always_inline)) {
            const int sl = (pos + lg) & (RS - 1);
#pragma unroll
            for (int k = 0; k < NCH; ++k) v[k] = lds4[cbase + sl + k * STR];
        };
        // Refills and early-abandon checks run at the first loop boundary at
        // or past their round: a refill at boundary b overwrites positions
        // below b (read only before round b) with positions from b + RS - RF
        // on (first read after round b + RS - RF - W - 2, more than six
        // rounds later), and a check is valid after any round.
        int next_refill = RF, next_check = kCheckRounds;
        bool done = false;
        auto boundary = [&](int r) __attribute__((always_inline)) -> bool {
            if (abandon && r >= next_check) {
                next_check += kCheckRounds;
                // the key loaded at the start of the item (a best-so-far only
                // decreases, so an older value is a safe threshold)
                const float thr = abandon_threshold(bsf_from_key(pend), a.gamma);
                // every warping path crosses one of the anti-diagonals 2r-2, 2r-1
                bool over;
                if constexpr (INDEP) {
                    // the distance is at least the sum over dimensions of each
                    // dimension's smallest value on those anti-diagonals (in the group)
                    float sum = 0.0f;
#pragma unroll
                    for (int p = 0; p < NV; ++p) {
                        float mp = (pad || spare) ? __builtin_inff() : vmin(vE[p], vO[p]);
                        for (int o = GS >> 1; o >= 1; o >>= 1) mp = vmin(mp, __shfl_xor(mp, o));
                        sum += mp;
                    }
                    over = sum > thr;
                } else {
                    over = vmin(vE[0], vO[0]) > thr;
                }
                const uint64_t bal = __ballot(over);
                if ((bal & gm) == gm) aband = true;
                if ((bal & valid_mask) == valid_mask) return true;
            }
            if (r >= next_refill) {
                const int b = next_refill;
                next_refill += RF;
                // positions b-RF+RS .. b+RS-1 (prefetched), then prefetch the next refill
#pragma unroll
                for (int p = 0; p < MAXPASS; ++p) {
                    const int x = p * kWave + lane;
                    if (x < nser * RF) put(x / RF, b - RF + RS + (x % RF), pf[p]);
                }
#pragma unroll
                for (int p = 0; p < MAXPASS; ++p) {
                    const int x = p * kWave + lane;
                    if (x < nser * RF) fetch(x / RF, b + RS + (x % RF), pf[p]);
                }
            }
            return false;
        };
        // Six rounds per iteration, software-pipelined: each round loads the
        // next round's query point and new candidate point before computing,
        // so the LDS latency overlaps a round of arithmetic.  Two query and
        // three candidate register sets rotate with period 6.  (Five sets of
        // d > 16 dimensions do not fit: those launches run two rounds per
        // iteration without prefetching.)
        float4 Q0[NCH], Q1[NCH], C0[NCH], C1[NCH], C2[NCH];
        ldc(0, C0);
        ldq(0, Q0);
        ldc(1, C1);
        int r = 0;
        if constexpr (NCH > 4) {
            while (r + 2 <= R) {
                if (boundary(r)) { done = true; break; }
                ldq(r, Q0); ldc(r + 1, C1);
                step(Q0, C0, C1);
                ldq(r + 1, Q0); ldc(r + 2, C0);
                step(Q0, C1, C0);
                r += 2;
            }
        }
        while (NCH <= 4 && r + 6 <= R) {
            if (boundary(r)) { done = true; break; }
            ldq(r + 1, Q1); ldc(r + 2, C2);
            step(Q0, C0, C1);
            ldq(r + 2, Q0); ldc(r + 3, C0);
            step(Q1, C1, C2);
            ldq(r + 3, Q1); ldc(r + 4, C1);
            step(Q0, C2, C0);
            ldq(r + 4, Q0); ldc(r + 5, C2);
            step(Q1, C0, C1);
            ldq(r + 5, Q1); ldc(r + 6, C0);
            step(Q0, C1, C2);
            ldq(r + 6, Q0); ldc(r + 7, C1);
            step(Q1, C2, C0);
            r += 6;
        }
        // the remaining rounds one at a time (C0 holds round r's cin)
        while (!done && r < R) {
            if (boundary(r)) { done = true; break; }
            ldq(r, Q0);
            ldc(r + 1, C1);
            step(Q0, C0, C1);
#pragma unroll
            for (int k = 0; k < NCH; ++k) C0[k] = C1[k];
            ++r;
        }
        (void)done;
        const int rounds = r;
        const int sigma = (a.n - a.m) + 2 * h;
        const int myref = spare ? -1 : (int)a.list[(int64_t)q * a.cap + base + grp];
        const bool res_lane = !spare && lg == (sigma >> 1);
        float res = 0.0f;
        if constexpr (INDEP) {
#pragma unroll
            for (int p = 0; p < NV; ++p)   // the dimensions' distances in increasing order
                if (p < a.D) res += (sigma & 1) ? vO[p] : vE[p];
        } else {
            res = (sigma & 1) ? vO[0] : vE[0];
        }
        if (res_lane) {
            float out = __builtin_inff();
            if (!aband && myref >= 0) {
                out = res;
                if (a.k <= 1) publish(a, q, myref, res, a.gamma);
            }
            a.list_dist[(int64_t)q * a.cap + base + grp] = out;
        }
        if (a.k > 1) {   // k-NN: one wave-cooperative insert per finished pair
            uint64_t pend_groups = __ballot(res_lane && !aband && myref >= 0);
            while (pend_groups) {
                const int src = __builtin_ctzll(pend_groups);
                pend_groups &= pend_groups - 1;
                const unsigned long long key = __shfl(dist_key(res, a.gamma, myref), src);
                topk_insert_wave(a.topk + (int64_t)q * a.k, a.k, key, &a.key[(int64_t)q * kKeyStride]);
            }
        }
        const uint64_t bstart = __ballot(!spare && lg == 0 && myref >= 0);
        const uint64_t bab = __ballot(aband && !spare && lg == 0 && myref >= 0);
        {
            const int ns = __popcll(bstart), na = __popcll(bab);
            w_started += ns;
            w_aband += na;
            const double part = (double)a.band_cells * (double)rounds / (double)R;
            w_cells += (unsigned long long)(ns - na) * (unsigned long long)a.band_cells +
                       (unsigned long long)((double)na * part);
        }
    }
    if (lane == 0 && w_started) {
        atomicAdd(&a.stats[kStDtwStarted], w_started);
        atomicAdd(&a.stats[kStDtwAbandoned], w_aband);
        atomicAdd(&a.stats[kStCells], w_cells);
    }
}

template <int NCH>
__global__ __launch_bounds__(64) void k_knn_dtw_rows(KnnDtwArgs a) {
    const int lane = threadIdx.x;
    const int sc = 0;
    const int total = a.prefix[a.nq];
    unsigned long long w_started = 0, w_aband = 0, w_cells = 0;
    for (;;) {
        const int item = wave_next_item(a.counter);
        if (item >= total) break;
        const int q = a.item_query[item];
        const int e = item - a.prefix[q];
        const int ref = (int)a.list[(int64_t)q * a.cap + e];
        const float* cser = a.C + (int64_t)(ref < 0 ? 0 : ref) * a.n * a.D;
        __syncthreads();
        Abandon ab{a.key + (int64_t)q * kKeyStride, a.gamma, ~0ull};
        bool aband = false;
        float v;
        int blocks = 0;
        if (a.abandon)
            v = rows_core<float, NCH, false, true>(sc, a.Q + (int64_t)q * a.m * a.D, cser, a.m,
                                                   a.n, a.W, a.D, lane, nullptr, ab, aband, &blocks);
        else
            v = rows_core<float, NCH, false, false>(sc, a.Q + (int64_t)q * a.m * a.D, cser, a.m,
                                                    a.n, a.W, a.D, lane, nullptr, ab, aband, &blocks);
        const int rl = (a.m - 1) % kRowBlock;
        if (lane == rl) {
            float out = __builtin_inff();
            if (!aband && ref >= 0) {
                out = v;
                if (a.k <= 1) publish(a, q, ref, v, a.gamma);
            }
            a.list_dist[(int64_t)q * a.cap + e] = out;
        }
        if (a.k > 1 && __shfl((int)(!aband && ref >= 0), rl)) {   // k-NN: wave-cooperative insert
            const unsigned long long key = __shfl(dist_key(v, a.gamma, ref), rl);
            topk_insert_wave(a.topk + (int64_t)q * a.k, a.k, key, &a.key[(int64_t)q * kKeyStride]);
        }
        if (ref >= 0) {
            const int nb = (a.m + kRowBlock - 1) / kRowBlock;
            w_started += 1;
            w_aband += aband ? 1 : 0;
            w_cells += aband ? (unsigned long long)((double)a.band_cells * blocks / nb)
                             : (unsigned long long)a.band_cells;
        }
    }
    if (lane == 0 && w_started) {
        atomicAdd(&a.stats[kStDtwStarted], w_started);
        atomicAdd(&a.stats[kStDtwAbandoned], w_aband);
        atomicAdd(&a.stats[kStCells], w_cells);
    }
}

// ---------------------------------------------------------------- finalize
// One wave per query: the k-th smallest float32 DTW over the seeds and the
// survivors (k = 1: the smallest), then a float64 re-scoring of every
// candidate within (1 + g) / (1 - g) of it; the k smallest float64 values
// win, ties to the lowest candidate index.  (A candidate among the exact k
// nearest has exact DTW at most the k-th exact distance, which is at most
// the k-th smallest v / (1 - g); so its float value is at most that times
// (1 + g).  Pruned and abandoned candidates exceed the k-th exact distance.)
template <int NCH, bool WODD, bool ROWS>
__global__ __launch_bounds__(64) void k_knn_finalize(KnnFinalArgs a) {
    const int q = blockIdx.x, lane = threadIdx.x;
    const int ns = a.R, nl = a.cnt[q], K = a.k;
    // An upper bound of the k-th smallest float32 value over the seeds and the
    // list: the query's threshold key, the largest of its k best keys (k = 1:
    // the best), each v / (1 - gamma) rounded up for a completed DTW's float32
    // value v.  A bound above the k-th value only adds finalists.
    (void)K;
    const float kth = bsf_from_key(a.key[(int64_t)q * kKeyStride]);
    const double thr = (double)kth * a.ratio;
    // the k best (float64 value, index) so far, ascending; kept by lane 0
    __shared__ double tk_v[kMaxK];
    __shared__ int tk_i[kMaxK];
    int tk_n = 0;

    double best = __builtin_inf();
    int bestidx = 0x7fffffff;
    int rescored = 0;
    DiagGeom g;
    g.init(a.m, a.n, a.W);
    const int LQ = g.LQ, LC = g.LC;
    const int sq = 0;
    const int sc = ROWS ? 0 : LQ * NCH;
    const int sc1 = LQ;    // candidate of the single-dimension staging (independent DTW)
    if (!ROWS && !a.indep)
        stage_series<NCH>(sq, LQ, g.qfirst(), a.Q + (int64_t)q * a.m * a.D, a.m, a.D, __builtin_inff(),
                          lane, kWave);
    for (int pass = 0; pass < 2; ++pass) {
        const int total = pass == 0 ? ns : nl;
        for (int b0 = 0; b0 < total; b0 += kWave) {
            const int k = b0 + lane;
            int ref = -1;
            float dv = __builtin_inff();
            if (k < total) {
                ref = pass == 0 ? a.seeds[(int64_t)q * ns + k] : (int)a.list[(int64_t)q * a.cap + k];
                dv = pass == 0 ? a.seed_dist[(int64_t)q * ns + k] : a.list_dist[(int64_t)q * a.cap + k];
            }
            uint64_t fin = __ballot(ref >= 0 && (double)dv <= thr);
            while (fin) {
                const int src = __builtin_ctzll(fin);
                fin &= fin - 1;
                const int r = __shfl(ref, src);
                __syncthreads();
                double v;
                if (ROWS) {
                    Abandon ab{nullptr, 0.0f, 0};
                    bool aband = false;
                    v = rows_core<double, NCH, false, false>(sc, a.Q + (int64_t)q * a.m * a.D,
                                                             a.C + (int64_t)r * a.n * a.D, a.m, a.n, a.W,
                                                             a.D, lane, nullptr, ab, aband);
                    v = __shfl(v, (a.m - 1) % kRowBlock);
                } else if (a.indep) {
                    // independent DTW: the univariate DTW of every dimension, summed in
                    // increasing dimension order
                    v = 0.0;
                    const int G = g.G, lg = lane;
                    const bool spare = lane >= G;
                    const bool kill_e = WODD && (lg == 0 || spare);
                    const bool kill_o = !WODD && (lg == G - 1);
                    const int qb = sq + (a.W - (spare ? 0 : lg));
                    const int cb = sc1 + (spare ? 0 : lg);
                    const int sigma = (a.n - a.m) + 2 * g.h;
                    for (int p = 0; p < a.D; ++p) {
                        __syncthreads();
                        stage_dim(sq, LQ, g.qfirst(), a.Q + (int64_t)q * a.m * a.D, a.m, a.D, p,
                                  __builtin_inff(), lane, kWave);
                        stage_dim(sc1, LC, g.cfirst(), a.C + (int64_t)r * a.n * a.D, a.n, a.D, p,
                                  -__builtin_inff(), lane, kWave);
                        __syncthreads();
                        double vE = __builtin_inf(), vO = __builtin_inf();
                        if (lg == g.h) vE = 0.0;
                        Abandon ab{nullptr, 0.0f, 0};
                        bool aband = false;
                        diag_core<double, 1, false, WODD, false>(qb, LQ, cb, LC, g.R, G, lg, kill_e, kill_o,
                                                                 vE, vO, nullptr, ab, aband, 0);
                        const double mine = (sigma & 1) ? vO : vE;
                        v = v + __shfl(mine, sigma >> 1);
                    }
                } else {
                    stage_series<NCH>(sc, LC, g.cfirst(), a.C + (int64_t)r * a.n * a.D, a.n, a.D,
                                      -__builtin_inff(), lane, kWave);
                    __syncthreads();
                    const int G = g.G, lg = lane;
                    const bool spare = lane >= G;
                    const bool kill_e = WODD && (lg == 0 || spare);
                    const bool kill_o = !WODD && (lg == G - 1);
                    const int qb = sq + (a.W - (spare ? 0 : lg));
                    const int cb = sc + (spare ? 0 : lg);
                    double vE = __builtin_inf(), vO = __builtin_inf();
                    if (lg == g.h) vE = 0.0;
                    Abandon ab{nullptr, 0.0f, 0};
                    bool aband = false;
                    diag_core<double, NCH, false, WODD, false>(qb, LQ, cb, LC, g.R, G, lg, kill_e, kill_o,
                                                               vE, vO, nullptr, ab, aband, 0);
                    const int sigma = (a.n - a.m) + 2 * g.h;
                    const double mine = (sigma & 1) ? vO : vE;
                    v = __shfl(mine, sigma >> 1);
                }
                ++rescored;
                if (v < best || (v == best && r < bestidx)) { best = v; bestidx = r; }
                if (K > 1 && lane == 0 &&
                    (tk_n < K || v < tk_v[K - 1] || (v == tk_v[K - 1] && r < tk_i[K - 1]))) {
                    int pos = tk_n < K ? tk_n : K - 1;
                    while (pos > 0 && (tk_v[pos - 1] > v || (tk_v[pos - 1] == v && tk_i[pos - 1] > r))) {
                        tk_v[pos] = tk_v[pos - 1];
                        tk_i[pos] = tk_i[pos - 1];
                        --pos;
                    }
                    tk_v[pos] = v;
                    tk_i[pos] = r;
                    if (tk_n < K) ++tk_n;
                }
            }
        }
    }
    if (lane == 0) {
        if (K == 1) {
            a.nn_idx[q] = bestidx == 0x7fffffff ? -1 : bestidx;
            a.nn_dist[q] = (float)best;
        } else {
            for (int t = 0; t < K; ++t) {
                a.nn_idx[(int64_t)q * K + t] = t < tk_n ? tk_i[t] : -1;
                a.nn_dist[(int64_t)q * K + t] = t < tk_n ? (float)tk_v[t] : __builtin_inff();
            }
        }
        atomicAdd(&a.stats[kStRescored], (unsigned long long)rescored);
        int nseeds = 0;
        for (int k = 0; k < ns; ++k) nseeds += a.seeds[(int64_t)q * ns + k] >= 0;
        const int gl = a.gcnt ? a.gcnt[q] : 0;
        const int direct = a.cnt_mv ? a.cnt_mv[q] : nl;
        const int pruned = a.nc - nseeds - direct - gl;
        if (pruned > 0) atomicAdd(&a.stats[kStPrunedMv], (unsigned long long)pruned);
        if (a.pruned_pc && a.pruned_pc[q]) atomicAdd(&a.stats[kStPrunedPc], (unsigned long long)a.pruned_pc[q]);
        if (a.pruned_ti && a.pruned_ti[q]) atomicAdd(&a.stats[kStPrunedTi], (unsigned long long)a.pruned_ti[q]);
    }
}

// ------------------------------------------------------------------ launch
hipError_t launch_knn_prep(const KnnPlanDev& p, hipStream_t s, bool init) {
    if (init)
        hipLaunchKernelGGL(k_knn_init, dim3((p.nq + 255) / 256 + 1), dim3(256), 0, s, p.nq, p.key, p.cnt,
                           p.gcnt, p.counters, p.stats, p.clear[0], p.clear[1], p.clear[2], p.topk, p.k);

    if (p.env) {
        const int64_t total = (int64_t)((p.nq + kQT - 1) / kQT) * kQT * (((int64_t)p.n * p.D + 3) / 4 * 4);
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
        hipLaunchKernelGGL(k_envelope, dim3(blocks), dim3(256), 0, s, p.Q, p.nq, p.m, p.n, p.D, p.W, p.env,
                           p.status);
    }
    return hipGetLastError();
}

// Tiles per wave of the LB_MV launch (see k_lb_mv).
static int lb_mv_cpl(int nq) { return nq > 2 ? 2 : 1; }

int lb_mv_segments(int ntiles, int nq, int E) {
    const int tpb = 4 * lb_mv_cpl(nq);
    const int64_t blocks = (int64_t)((ntiles + tpb - 1) / tpb) * ((nq + kQT - 1) / kQT);
    if (blocks >= 2048) return 1;   // eight waves per CU already
    int64_t S = (8192 + blocks - 1) / blocks;
    const int ld = nq <= 2 ? 4 : 2;   // loads in flight of the kernel that runs
    S = std::min<int64_t>(S, std::max(1, (E + 3) / 4 / (8 * ld)));   // eight rounds of loads per segment
    return (int)std::max<int64_t>(S, 1);
}

hipError_t launch_lb_mv(const KnnPlanDev& p, float* lb, hipStream_t s) {
    const int E = p.n * p.D;
    const double u = 1.0 / 16777216.0;
    const double deflate = 1.0 - (double)(E + 3) * u * 1.001;
    const int S = p.part ? p.nseg : 1;
    const int E4 = (E + 3) / 4;
    const int seg = (E4 + S - 1) / S;   // in groups of 4 elements
    const int tpb = 4 * lb_mv_cpl(p.nq);
    dim3 grid((p.ntiles + tpb - 1) / tpb, (p.nq + kQT - 1) / kQT, S);
    auto kern = p.nq > 4 ? k_lb_mv<kQT> : p.nq > 2 ? k_lb_mv<4> : p.nq > 1 ? k_lb_mv<2> : k_lb_mv<1>;
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, p.tiles, p.ntiles, E, p.env, p.nq, p.nc, deflate, lb, seg,
                       p.part);
    if (S > 1) {
        const int64_t n = (int64_t)p.nq * p.nc;
        const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(k_lb_sum, dim3(blocks), dim3(256), 0, s, p.part, S, n, deflate, lb);
    }
    return hipGetLastError();
}

hipError_t launch_topr(const KnnPlanDev& p, hipStream_t s) {
    if (p.R <= 8)
        hipLaunchKernelGGL(k_topr<8>, dim3(p.nq), dim3(64), 0, s, p.lb, p.nc, p.R, p.q_cb, p.q_ce, p.seeds);
    else
        hipLaunchKernelGGL(k_topr<kMaxSeeds>, dim3(p.nq), dim3(64), 0, s, p.lb, p.nc, p.R, p.q_cb, p.q_ce, p.seeds);
    return hipGetLastError();
}

hipError_t launch_compact(const KnnPlanDev& p, double keep, double gate_e2, int use_gate, hipStream_t s) {
    dim3 grid((p.nc + kCompactPer - 1) / kCompactPer, p.nq);
    hipLaunchKernelGGL(k_compact, grid, dim3(256), 0, s, p.lb, p.nc, p.q_cb, p.q_ce, p.seeds, p.R, p.key, keep,
                       gate_e2, use_gate, p.list, p.cnt, p.glist, p.gcnt, p.cap, p.stats);
    return hipGetLastError();
}

template <int NCH, int RS, int NPASS>
static void launch_ring_w(const KnnDtwArgs& a, int nblocks, size_t lds, hipStream_t s) {
    constexpr bool kIndep = NCH <= 4;   // independent DTW is built for up to 16 dimensions
    if (a.indep && kIndep) {
        if (a.W & 1) hipLaunchKernelGGL((k_knn_dtw_ring<NCH, true, RS, NPASS, kIndep>), dim3(nblocks), dim3(64), lds, s, a);
        else hipLaunchKernelGGL((k_knn_dtw_ring<NCH, false, RS, NPASS, kIndep>), dim3(nblocks), dim3(64), lds, s, a);
        return;
    }
    if (a.W & 1) hipLaunchKernelGGL((k_knn_dtw_ring<NCH, true, RS, NPASS, false>), dim3(nblocks), dim3(64), lds, s, a);
    else hipLaunchKernelGGL((k_knn_dtw_ring<NCH, false, RS, NPASS, false>), dim3(nblocks), dim3(64), lds, s, a);
}

template <int NCH, int RS>
static void launch_ring(const KnnDtwArgs& a, int npass, int nblocks, size_t lds, hipStream_t s) {
    if (npass <= 1) launch_ring_w<NCH, RS, 1>(a, nblocks, lds, s);
    else if (NCH <= 4 && npass == 2) launch_ring_w<NCH, RS, (NCH <= 4 ? 2 : 1)>(a, nblocks, lds, s);
    else if (NCH <= 4) launch_ring_w<NCH, RS, (NCH <= 4 ? 3 : 1)>(a, nblocks, lds, s);
}

template <int NCH>
static hipError_t launch_dtw_lists_nch(const KnnDtwArgs& a, bool rows, int nblocks, size_t lds,
                                       hipStream_t s) {
    if (rows) {
        hipLaunchKernelGGL(k_knn_dtw_rows<NCH>, dim3(nblocks), dim3(64), lds, s, a);
    } else {
        const int RS = ring_size(a.W);
        const int npass = ((1 + a.P) * (RS / 4) + kWave - 1) / kWave;
        if (npass > knn_ring_max_passes(NCH)) return hipErrorInvalidValue;
        if (RS == 64) launch_ring<NCH, 64>(a, npass, nblocks, lds, s);
        else launch_ring<NCH, 128>(a, npass, nblocks, lds, s);
    }
    return hipGetLastError();
}

hipError_t launch_chunk_scan(const KnnDtwArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(1024), 0, s, a.cnt, a.cnt_uniform, a.nq, a.P,
                       const_cast<int32_t*>(a.prefix), a.counter);
    hipLaunchKernelGGL(k_item_map, dim3(a.nq < 4096 ? a.nq : 4096), dim3(256), 0, s, a.prefix, a.nq,
                       const_cast<int32_t*>(a.item_query));
    return hipGetLastError();
}

// The persistent DTW kernel; launch_chunk_scan must precede it on the stream.
hipError_t launch_dtw_lists(const KnnDtwArgs& a, int nblocks, hipStream_t s) {
    const bool rows = a.W > kDiagMaxW;
    const int nch = nch_pad(a.D);
    const size_t lds = knn_dtw_lds_bytes(a.m, a.n, a.W, a.D, a.P);
    switch (nch) {
        case 1: return launch_dtw_lists_nch<1>(a, rows, nblocks, lds, s);
        case 2: return launch_dtw_lists_nch<2>(a, rows, nblocks, lds, s);
        case 3: return launch_dtw_lists_nch<3>(a, rows, nblocks, lds, s);
        case 4: return launch_dtw_lists_nch<4>(a, rows, nblocks, lds, s);
        case 6: return launch_dtw_lists_nch<6>(a, rows, nblocks, lds, s);
        case 8: return launch_dtw_lists_nch<8>(a, rows, nblocks, lds, s);
        case 12: return launch_dtw_lists_nch<12>(a, rows, nblocks, lds, s);
        case 16: return launch_dtw_lists_nch<16>(a, rows, nblocks, lds, s);
    }
    return hipErrorInvalidValue;
}

size_t knn_dtw_lds_bytes(int m, int n, int W, int D, int P) {
    (void)m;
    if (W > kDiagMaxW) return rows_core_lds(n, nch_pad(D), 4);
    return (size_t)(1 + P) * ring_size(W) * nch_pad(D) * 16;
}

int knn_ring_max_passes(int nch) { return nch <= 4 ? 3 : 1; }

int knn_dtw_max_pairs(int W, int D, bool indep) {
    if (W > kDiagMaxW) return 1;
    int P = kWave / knn_lane_stride(W, indep);
    const int RF = ring_size(W) / 4;
    const int maxpass = knn_ring_max_passes(nch_pad(D));
    while (P > 1 && (1 + P) * RF > maxpass * kWave) --P;
    return P;
}

size_t knn_final_lds_bytes(int m, int n, int W, int D) {
    if (W > kDiagMaxW) return rows_core_lds(n, nch_pad(D), 8);
    DiagGeom g;
    g.init(m, n, W);
    return (size_t)(g.LQ + g.LC) * nch_pad(D) * 16;
}

template <int NCH>
static hipError_t launch_final_nch(const KnnFinalArgs& a, size_t lds, hipStream_t s) {
    if (a.W > kDiagMaxW)
        hipLaunchKernelGGL((k_knn_finalize<NCH, false, true>), dim3(a.nq), dim3(64), lds, s, a);
    else if (a.W & 1)
        hipLaunchKernelGGL((k_knn_finalize<NCH, true, false>), dim3(a.nq), dim3(64), lds, s, a);
    else
        hipLaunchKernelGGL((k_knn_finalize<NCH, false, false>), dim3(a.nq), dim3(64), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_knn_finalize(const KnnFinalArgs& a, hipStream_t s) {
    const size_t lds = knn_final_lds_bytes(a.m, a.n, a.W, a.D);
    switch (nch_pad(a.D)) {
        case 1: return launch_final_nch<1>(a, lds, s);
        case 2: return launch_final_nch<2>(a, lds, s);
        case 3: return launch_final_nch<3>(a, lds, s);
        case 4: return launch_final_nch<4>(a, lds, s);
        case 6: return launch_final_nch<6>(a, lds, s);
        case 8: return launch_final_nch<8>(a, lds, s);
        case 12: return launch_final_nch<12>(a, lds, s);
        case 16: return launch_final_nch<16>(a, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace tcdtw
