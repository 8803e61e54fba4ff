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

// ------------------------------------------------------------------ setup
__global__ void k_knn_init(int nq, unsigned long long* key, int32_t* cnt, int32_t* gcnt,
                           int32_t* counters, unsigned long long* stats) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int q = t; q < nq; q += gridDim.x * blockDim.x) {
        key[q] = 0x7f800000ffffffffull;     // best-so-far +inf, no candidate yet
        cnt[q] = 0;
        if (gcnt) gcnt[q] = 0;
    }
    if (t < kNumCounters) counters[t] = 0;
    if (t < kNumStats) stats[t] = 0;
}

// Query envelope (Sec. 3, LB_MV): for candidate position j, the max / min
// of each query dimension over query rows [j - W, j + W] clipped to [0, m).
// Layout env[qtile][e][QT][2] (e = j*D + p), so one 64-byte scalar load
// gives the (U, L) pairs of a tile's QT queries for one element.
__global__ void k_envelope(const float* __restrict__ Q, int nq, int m, int n, int D, int W,
                           float* __restrict__ env) {
    const int E = n * D;
    const int nqt = (nq + kQT - 1) / kQT;
    const int64_t total = (int64_t)nqt * kQT * E;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(idx % E);
        const int q = (int)(idx / E);
        const int j = e / D, p = e - j * D;
        float U = __builtin_inff(), L = -__builtin_inff();
        if (q < nq) {
            const int i0 = max(0, j - W), i1 = min(m - 1, j + W);
            const float* s = Q + (int64_t)q * m * D + p;
            U = s[(int64_t)i0 * D];
            L = U;
            for (int i = i0 + 1; i <= i1; ++i) {
                const float v = s[(int64_t)i * D];
                U = __builtin_fmaxf(U, v);
                L = __builtin_fminf(L, v);
            }
        }
        float* o = env + (((int64_t)(q / kQT) * E + e) * kQT + (q % kQT)) * 2;
        o[0] = U;
        o[1] = L;
    }
}

// LB_MV (Sec. 3, squared form) of kQT queries against 64 candidates per
// wave.  Candidates come from the element-major tiles (one coalesced
// 256-byte load per element), the envelope from wave-uniform scalar loads;
// per element and query: two subtractions, a max3 and an FMA.
__global__ __launch_bounds__(256) void k_lb_mv(const float* __restrict__ tiles, int ntiles, int E,
                                               const float* __restrict__ env, int nq, int nc,
                                               double deflate, float* __restrict__ lb) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= ntiles) return;
    const int qt = blockIdx.y;
    const float* __restrict__ cp = tiles + (int64_t)tile * E * 64 + lane;
    const float* __restrict__ ep = env + (int64_t)qt * E * kQT * 2;
    float acc[kQT];
#pragma unroll
    for (int k = 0; k < kQT; ++k) acc[k] = 0.0f;
    for (int e = 0; e < E; ++e) {
        const float c = cp[(int64_t)e * 64];
        const float* __restrict__ u = ep + (int64_t)e * kQT * 2;
#pragma unroll
        for (int k = 0; k < kQT; ++k) {
            const float d = __builtin_fmaxf(__builtin_fmaxf(c - u[2 * k], u[2 * k + 1] - c), 0.0f);
            acc[k] = __builtin_fmaf(d, d, acc[k]);
        }
    }
    const int r = tile * 64 + lane;
    if (r >= nc) return;
#pragma unroll
    for (int k = 0; k < kQT; ++k) {
        const int q = qt * kQT + k;
        if (q < nq) lb[(int64_t)q * nc + r] = round_down_f((double)acc[k] * deflate);
    }
}

// Seeds: the R candidates with the smallest LB_MV of each query (one wave
// per query; ties between equal bounds in any order).
template <int RMAX>
__global__ __launch_bounds__(64) void k_topr(const float* __restrict__ lb, int nc, int R,
                                             int32_t* __restrict__ seeds) {
    const int q = blockIdx.x, lane = threadIdx.x;
    float v[RMAX];
    int id[RMAX];
#pragma unroll
    for (int k = 0; k < RMAX; ++k) { v[k] = __builtin_inff(); id[k] = 0x7fffffff; }
    const float* row = lb + (int64_t)q * nc;
    for (int r = lane; r < nc; r += kWave) {
        float x = row[r];
        int xi = r;
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
    }
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
// advanced-bound list when gating is on and LB_MV > e^2 bsf.  Wave ballot
// plus one atomic per wave and list.
__global__ __launch_bounds__(256) void k_compact(const float* __restrict__ lb, int nc,
                                                 const int32_t* __restrict__ seeds, int R,
                                                 const unsigned long long* __restrict__ key,
                                                 double keep, double gate_e2, int use_gate,
                                                 uint32_t* __restrict__ list, int32_t* cnt,
                                                 uint32_t* __restrict__ glist, int32_t* gcnt, int cap,
                                                 unsigned long long* stats) {
    const int q = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const double bsf = (double)bsf_from_key(key[q]);
    const bool valid = r < nc;
    bool seed = false;
    for (int k = 0; k < R; ++k) seed |= (seeds[(int64_t)q * R + k] == r);
    const double v = (valid && lb) ? (double)lb[(int64_t)q * nc + r] : 0.0;
    const bool live = valid && !seed;
    const bool pruned = live && (v * keep > bsf);
    const bool gated = live && !pruned && use_gate && (v > gate_e2 * bsf);
    const bool todtw = live && !pruned && !gated;
    const uint64_t bd = __ballot(todtw), bg = __ballot(gated), bp = __ballot(pruned);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int based = 0, baseg = 0;
    if (lane == 0) {
        if (bd) based = atomicAdd(&cnt[q], __popcll(bd));
        if (bg) baseg = atomicAdd(&gcnt[q], __popcll(bg));
        if (bp) atomicAdd(&stats[kStPrunedMv], (unsigned long long)__popcll(bp));
    }
    based = __shfl(based, 0);
    baseg = __shfl(baseg, 0);
    if (todtw) list[(int64_t)q * cap + based + __popcll(bd & below)] = (uint32_t)r;
    if (gated) glist[(int64_t)q * cap + baseg + __popcll(bg & below)] = (uint32_t)r;
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

__device__ __forceinline__ void publish(const KnnDtwArgs& a, int q, int ref, float v, float gamma) {
    const float up = round_up_pos((double)v / (1.0 - (double)gamma));
    const unsigned long long k = ((unsigned long long)__float_as_uint(up) << 32) | (uint32_t)ref;
    atomicMin(&a.key[q], k);
}

template <int NCH, bool WODD>
__global__ __launch_bounds__(64) void k_knn_dtw_diag(KnnDtwArgs a) {
    extern __shared__ float4 smem[];
    const int lane = threadIdx.x;
    DiagGeom g;
    g.init(a.m, a.n, a.W);
    const int G = g.G, h = g.h, R = g.R, LQ = g.LQ, LC = g.LC, P = a.P;
    float4* sq = smem;
    float4* scs = smem + LQ * NCH;
    const int grp = lane / G;
    const int lg = lane - grp * G;
    const int total = a.prefix[a.nq];
    int staged_q = -1;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(a.counter, 1);
        item = __shfl(item, 0);
        if (item >= total) break;
        const int q = find_query(a.prefix, a.nq, item);
        const int chunk = item - a.prefix[q];
        const int base = chunk * P;
        const int np = min(P, a.cnt_uniform > 0 ? a.cnt_uniform - base : a.cnt[q] - base);
        __syncthreads();
        if (q != staged_q) {
            stage_series<NCH>(sq, LQ, g.qfirst(), a.Q + (int64_t)q * a.m * a.D, a.m, a.D,
                              __builtin_inff(), lane, kWave);
            staged_q = q;
        }
        for (int gg = 0; gg < np; ++gg) {
            const int ref = (int)a.list[(int64_t)q * a.cap + base + gg];
            stage_series<NCH>(scs + gg * LC * NCH, LC, g.cfirst(),
                              a.C + (int64_t)(ref < 0 ? 0 : ref) * a.n * a.D, a.n, a.D,
                              -__builtin_inff(), lane, kWave);
        }
        __syncthreads();
        const bool spare = grp >= np;
        const int gsrc = spare ? 0 : grp;
        const bool kill_e = WODD && (lg == 0 || spare);
        const bool kill_o = !WODD && (lg == G - 1);
        const float4* qb = sq + (a.W - lg);
        const float4* cb = scs + gsrc * LC * NCH + lg;
        float vE = __builtin_inff(), vO = __builtin_inff();
        if (!spare && lg == h) vE = 0.0f;
        const uint64_t valid_mask = (np * G >= 64) ? ~0ull : ((1ull << (np * G)) - 1);
        const uint64_t gm = spare ? 0ull : (((G >= 64) ? ~0ull : ((1ull << G) - 1)) << (grp * G));
        Abandon ab{a.key + q, a.gamma, valid_mask};
        bool aband = false;
        if (a.abandon)
            diag_core<float, NCH, false, WODD, true>(qb, LQ, cb, LC, R, G, lg, kill_e, kill_o, vE, vO,
                                                     nullptr, ab, aband, gm);
        else
            diag_core<float, NCH, false, WODD, false>(qb, LQ, cb, LC, R, G, lg, kill_e, kill_o, vE, vO,
                                                      nullptr, ab, aband, gm);
        const int sigma = (a.n - a.m) + 2 * h;
        const int myref = spare ? -1 : (int)a.list[(int64_t)q * a.cap + base + grp];
        if (!spare && lg == (sigma >> 1)) {
            const float v = (sigma & 1) ? vO : vE;
            float out = __builtin_inff();
            if (!aband && myref >= 0) {
                out = v;
                publish(a, q, myref, v, a.gamma);
            }
            a.list_dist[(int64_t)q * a.cap + base + grp] = out;
        }
        const uint64_t bstart = __ballot(!spare && lg == 0 && myref >= 0);
        const uint64_t bab = __ballot(aband && !spare && lg == 0 && myref >= 0);
        if (lane == 0) {
            atomicAdd(&a.stats[kStDtwStarted], (unsigned long long)__popcll(bstart));
            if (bab) atomicAdd(&a.stats[kStDtwAbandoned], (unsigned long long)__popcll(bab));
        }
    }
}

template <int NCH>
__global__ __launch_bounds__(64) void k_knn_dtw_rows(KnnDtwArgs a) {
    extern __shared__ float4 smem[];
    const int lane = threadIdx.x;
    const int LC = a.n + 2 * kRowPad;
    float4* sc = smem;
    float* rowbuf = reinterpret_cast<float*>(smem + (size_t)LC * NCH);
    const int total = a.prefix[a.nq];
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(a.counter, 1);
        item = __shfl(item, 0);
        if (item >= total) break;
        const int q = find_query(a.prefix, a.nq, item);
        const int e = item - a.prefix[q];
        const int ref = (int)a.list[(int64_t)q * a.cap + e];
        __syncthreads();
        stage_series<NCH>(sc, LC, -kRowPad, a.C + (int64_t)(ref < 0 ? 0 : ref) * a.n * a.D, a.n, a.D,
                          -__builtin_inff(), lane, kWave);
        Abandon ab{a.key + q, a.gamma, ~0ull};
        bool aband = false;
        float v;
        if (a.abandon)
            v = rows_core<float, NCH, false, true>(sc, rowbuf, LC, a.Q + (int64_t)q * a.m * a.D, a.m,
                                                   a.n, a.W, a.D, lane, nullptr, ab, aband);
        else
            v = rows_core<float, NCH, false, false>(sc, rowbuf, LC, a.Q + (int64_t)q * a.m * a.D, a.m,
                                                    a.n, a.W, a.D, lane, nullptr, ab, aband);
        if (lane == (a.m - 1) % kRowBlock) {
            float out = __builtin_inff();
            if (!aband && ref >= 0) {
                out = v;
                publish(a, q, ref, v, a.gamma);
            }
            a.list_dist[(int64_t)q * a.cap + e] = out;
        }
        if (lane == 0 && ref >= 0) {
            atomicAdd(&a.stats[kStDtwStarted], 1ull);
            if (aband) atomicAdd(&a.stats[kStDtwAbandoned], 1ull);
        }
    }
}

// ---------------------------------------------------------------- finalize
// One wave per query: the smallest float32 DTW over the seeds and the
// survivors, then a float64 re-scoring of every candidate within
// (1 + g) / (1 - g) of it; the smallest float64 value wins, ties to the
// lowest candidate index.
template <int NCH, bool WODD, bool ROWS>
__global__ __launch_bounds__(64) void k_knn_finalize(KnnFinalArgs a) {
    extern __shared__ float4 smem[];
    const int q = blockIdx.x, lane = threadIdx.x;
    float mn = __builtin_inff();
    const int ns = a.R, nl = a.cnt[q];
    for (int k = lane; k < ns; k += kWave)
        if (a.seeds[(int64_t)q * ns + k] >= 0) mn = __builtin_fminf(mn, a.seed_dist[(int64_t)q * ns + k]);
    for (int k = lane; k < nl; k += kWave) mn = __builtin_fminf(mn, a.list_dist[(int64_t)q * a.cap + k]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mn = __builtin_fminf(mn, __shfl_xor(mn, o));
    const double thr = (double)mn * a.ratio;

    double best = __builtin_inf();
    int bestidx = 0x7fffffff;
    int rescored = 0;
    DiagGeom g;
    g.init(a.m, a.n, a.W);
    const int LQ = g.LQ, LC = g.LC;
    float4* sq = smem;
    float4* sc = ROWS ? smem : smem + LQ * NCH;
    if (!ROWS)
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
                    const int LCr = a.n + 2 * kRowPad;
                    double* rowbuf = reinterpret_cast<double*>(sc + (size_t)LCr * NCH);
                    stage_series<NCH>(sc, LCr, -kRowPad, a.C + (int64_t)r * a.n * a.D, a.n, a.D,
                                      -__builtin_inff(), lane, kWave);
                    Abandon ab{nullptr, 0.0f, 0};
                    bool aband = false;
                    v = rows_core<double, NCH, false, false>(sc, rowbuf, LCr, a.Q + (int64_t)q * a.m * a.D,
                                                             a.m, a.n, a.W, a.D, lane, nullptr, ab, aband);
                    v = __shfl(v, (a.m - 1) % kRowBlock);
                } else {
                    stage_series<NCH>(sc, LC, g.cfirst(), a.C + (int64_t)r * a.n * a.D, a.n, a.D,
                                      -__builtin_inff(), lane, kWave);
                    __syncthreads();
                    const int G = g.G, lg = lane;
                    const bool spare = lane >= G;
                    const bool kill_e = WODD && (lg == 0 || spare);
                    const bool kill_o = !WODD && (lg == G - 1);
                    const float4* qb = sq + (a.W - (spare ? 0 : lg));
                    const float4* cb = sc + (spare ? 0 : lg);
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
            }
        }
    }
    if (lane == 0) {
        a.nn_idx[q] = bestidx == 0x7fffffff ? -1 : bestidx;
        a.nn_dist[q] = (float)best;
        atomicAdd(&a.stats[kStRescored], (unsigned long long)rescored);
    }
}

// ------------------------------------------------------------------ launch
hipError_t launch_knn_prep(const KnnPlanDev& p, hipStream_t s) {
    hipLaunchKernelGGL(k_knn_init, dim3((p.nq + 255) / 256 + 1), dim3(256), 0, s, p.nq, p.key, p.cnt,
                       p.gcnt, p.counters, p.stats);
    if (p.env) {
        const int64_t total = (int64_t)((p.nq + kQT - 1) / kQT) * kQT * p.n * p.D;
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
        hipLaunchKernelGGL(k_envelope, dim3(blocks), dim3(256), 0, s, p.Q, p.nq, p.m, p.n, p.D, p.W, p.env);
    }
    return hipGetLastError();
}

hipError_t launch_lb_mv(const KnnPlanDev& p, float* lb, hipStream_t s) {
    const int E = p.n * p.D;
    const double u = 1.0 / 16777216.0;
    const double deflate = 1.0 - (double)(E + 3) * u * 1.001;
    dim3 grid((p.ntiles + 3) / 4, (p.nq + kQT - 1) / kQT);
    hipLaunchKernelGGL(k_lb_mv, grid, dim3(256), 0, s, p.tiles, p.ntiles, E, p.env, p.nq, p.nc, deflate, lb);
    return hipGetLastError();
}

hipError_t launch_topr(const KnnPlanDev& p, hipStream_t s) {
    hipLaunchKernelGGL(k_topr<kMaxSeeds>, dim3(p.nq), dim3(64), 0, s, p.lb, p.nc, p.R, p.seeds);
    return hipGetLastError();
}

hipError_t launch_compact(const KnnPlanDev& p, double keep, double gate_e2, int use_gate, hipStream_t s) {
    dim3 grid((p.nc + 255) / 256, p.nq);
    hipLaunchKernelGGL(k_compact, grid, dim3(256), 0, s, p.lb, p.nc, p.seeds, p.R, p.key, keep, gate_e2,
                       use_gate, p.list, p.cnt, p.glist, p.gcnt, p.cap, p.stats);
    return hipGetLastError();
}

template <int NCH>
static hipError_t launch_dtw_lists_nch(const KnnDtwArgs& a, bool rows, int nblocks, size_t lds,
                                       hipStream_t s) {
    if (rows)
        hipLaunchKernelGGL(k_knn_dtw_rows<NCH>, dim3(nblocks), dim3(64), lds, s, a);
    else if (a.W & 1)
        hipLaunchKernelGGL((k_knn_dtw_diag<NCH, true>), dim3(nblocks), dim3(64), lds, s, a);
    else
        hipLaunchKernelGGL((k_knn_dtw_diag<NCH, false>), dim3(nblocks), dim3(64), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_dtw_lists(const KnnDtwArgs& a, int nblocks, hipStream_t s) {
    // chunk prefix over the queries, then the persistent DTW kernel
    hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(1024), 0, s, a.cnt, a.cnt_uniform, a.nq, a.P,
                       const_cast<int32_t*>(a.prefix), a.counter);
    const bool rows = a.W > kDiagMaxW;
    DiagGeom g;
    g.init(a.m, a.n, a.W);
    const int nch = nch_pad(a.D);
    const size_t lds = rows ? rows_lds_bytes(a.n, a.W, a.D, false)
                            : (size_t)(g.LQ + a.P * g.LC) * nch * 16;
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
    if (W > kDiagMaxW) return rows_lds_bytes(n, W, D, false);
    DiagGeom g;
    g.init(m, n, W);
    return (size_t)(g.LQ + P * g.LC) * nch_pad(D) * 16;
}

size_t knn_final_lds_bytes(int m, int n, int W, int D) {
    if (W > kDiagMaxW) return rows_lds_bytes(n, W, D, true);
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
