// 1-NN search over a reference bank of uneven lengths (one D per bank) for
// queries of uneven lengths: the cascade of the uniform search (Sec. 2 DTW
// nearest neighbour, Sec. 3 LB_MV, best-so-far seeding, compaction, DTW
// with early abandoning, float64 re-scoring) with a window per pair:
// W = floor(max(m, n) num / den) (or the absolute window), W_eff = max(W,
// |m - n|), capped at max(m, n) - 1.
//
//  * LB_MV needs the query envelope over each pair's own window
//    [j - W, j + W] of candidate position j.  Each query gets sparse tables
//    of running maxima and minima per dimension (level k holds the extremes
//    of 2^k consecutive points), so any window is covered by two blocks of
//    one level; a wave evaluates one pair with lanes over candidate points,
//    reading the table rows of consecutive windows (coalesced).
//  * DTW runs on the row mapping (any window, LDS independent of W) with the
//    pair's geometry read per item; early abandoning and the packed
//    best-so-far keys work as in the uniform search.
//  * The float64 re-scoring bounds each pair's relative float32 error by
//    the largest of the query's pairs.
//  * Banks of several dimensions (q_dim set): each query is compared with
//    the candidates of its own D only, a contiguous range [q_cb, q_ce) of
//    the index; bounds outside it are +inf (never seeds, always pruned), and
//    the DTW and re-scoring kernels, instantiated for the largest D, run
//    each item with the chunk count of its own D.
#include <algorithm>

#include "dtw_core.h"
#include "internal.h"

namespace tcdtw {

__device__ __forceinline__ int weff_dev(int m, int n, int window, int num, int den) {
    const int longer = m > n ? m : n;
    long long W = den > 0 ? ((long long)longer * num) / den : window;
    const int diff = m > n ? m - n : n - m;
    if (W < diff) W = diff;
    if (W > longer - 1) W = longer - 1;
    return (int)W;
}

// Band cells of an m x n pair with W >= |m - n| (every row has a cell):
// sum over rows of min(n-1, i+W) - max(0, i-W) + 1, in closed form.
__device__ __forceinline__ long long band_cells_dev(int m, int n, int W) {
    const long long k = min(max(n - W, 0), m);          // rows with i + W <= n - 1
    const long long s1 = k * (k - 1) / 2 + k * W + (long long)(m - k) * (n - 1);
    const long long t = max(0, m - W);                  // rows with i >= W
    return s1 - t * (t - 1) / 2 + m;
}

__device__ __forceinline__ int levels_of(int m) { return 32 - __builtin_clz((unsigned)m); }

__device__ __forceinline__ float rdown_f(double x) {
    float f = (float)x;
    if ((double)f > x) f = __uint_as_float(__float_as_uint(f) - 1u);
    return f;
}

__device__ __forceinline__ float rup_f(double x) {
    float f = (float)x;
    if ((double)f < x) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

// Relative error bound of the float32 DP of an m x n pair (as in the uniform search).
__device__ __forceinline__ float dp_gamma_dev(int m, int n, int nch) {
    return (float)(1.01 * (double)(m + n + 4 * nch + 2) / 16777216.0);
}

// ------------------------------------------------------- query tables
// One block per query: level 0 is the query; level k at start t holds the
// max (min) of points t .. t + 2^k - 1 of each dimension.  Layout per
// query: max levels [L][m][D], then min levels [L][m][D].
__global__ __launch_bounds__(256) void k_rq_tables(RaggedKnnArgs a) {
    const int q = blockIdx.x;
    const int m = a.q_len[q], D = a.q_dim ? a.q_dim[q] : a.D;
    const int L = levels_of(m);
    const int64_t md = (int64_t)m * D;
    const float* src = a.Q + a.q_off[q];
    float* mx = a.tab + a.t_off[q];
    float* mn = mx + (int64_t)L * md;
    bool bad = false;
    for (int64_t e = threadIdx.x; e < md; e += blockDim.x) {
        const float v = src[e];
        mx[e] = v;
        mn[e] = v;
        bad |= !__builtin_isfinite(v);
    }
    if (bad && a.status) atomicOr(a.status, kStatusNonFiniteQuery);
    __syncthreads();
    for (int k = 1; k < L; ++k) {
        const int half = 1 << (k - 1);
        const int64_t cnt = (int64_t)(m - (1 << k) + 1) * D;
        float* xk = mx + k * md;
        float* nk = mn + k * md;
        const float* xp = xk - md;
        const float* np = nk - md;
        for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
            xk[e] = __builtin_fmaxf(xp[e], xp[e + (int64_t)half * D]);
            nk[e] = __builtin_fminf(np[e], np[e + (int64_t)half * D]);
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- LB_MV
// One wave per (query, candidate); blocks of 4 waves over candidates,
// grid.y over queries.  Rounding as in the uniform LB_MV: the sum of
// N = n D + 6 float32 terms (each lane's partial sum, then 6 shuffle
// levels) is scaled by 1 - (N + 3) u and rounded down.  With D a multiple
// of 4 (VEC) the table rows and the candidate point are read as float4
// chunks (every row offset is then a multiple of 4 floats), NCH chunks
// unrolled so that all loads of a point are in flight together.
// Distance of v to [Lw, U] up to sign (v - U above, v - Lw below, 0 inside);
// its square is the envelope term.
__device__ __forceinline__ float mv_term(float v, float U, float Lw) {
    return v - __builtin_amdgcn_fmed3f(v, Lw, U);
}

template <int NCH, bool VEC>
__global__ __launch_bounds__(256) void k_rlb_mv(RaggedKnnArgs a) {
    const int q = a.q0 + blockIdx.y;
    const int lane = threadIdx.x & 63;
    // with banks of several dims the grid covers the largest bank and each query its own
    const int c = (a.q_dim ? a.q_cb[q] : 0) + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= (a.q_dim ? a.q_ce[q] : a.nc)) return;   // whole waves
    const int m = a.q_len[q], n = a.c_len[c], D = a.q_dim ? a.q_dim[q] : a.D;
    const int W = weff_dev(m, n, a.window, a.num, a.den);
    const int L = levels_of(m);
    const int64_t md = (int64_t)m * D;
    const float* mx = a.tab + a.t_off[q];
    const float* mn = mx + (int64_t)L * md;
    const float* cs = a.C + a.c_off[c];
    const int D4 = D >> 2;
    const bool vec = VEC && (D & 3) == 0;   // with banks of several D, decided per query
    float acc = 0.0f;
    for (int j = lane; j < n; j += kWave) {
        const int lo = max(0, j - W), hi = min(m - 1, j + W);
        const int k = 31 - __builtin_clz((unsigned)(hi - lo + 1));
        const int h2 = hi - (1 << k) + 1;
        const float* xk = mx + k * md;
        const float* nk = mn + k * md;
        if (vec) {
            float4 x1[NCH], x2[NCH], n1[NCH], n2[NCH], cv[NCH];
#pragma unroll
            for (int t = 0; t < NCH; ++t) {
                if (t < D4) {
                    x1[t] = *reinterpret_cast<const float4*>(xk + (int64_t)lo * D + 4 * t);
                    x2[t] = *reinterpret_cast<const float4*>(xk + (int64_t)h2 * D + 4 * t);
                    n1[t] = *reinterpret_cast<const float4*>(nk + (int64_t)lo * D + 4 * t);
                    n2[t] = *reinterpret_cast<const float4*>(nk + (int64_t)h2 * D + 4 * t);
                    cv[t] = *reinterpret_cast<const float4*>(cs + (int64_t)j * D + 4 * t);
                }
            }
#pragma unroll
            for (int t = 0; t < NCH; ++t) {
                if (t < D4) {
                    float d;
                    d = mv_term(cv[t].x, __builtin_fmaxf(x1[t].x, x2[t].x), __builtin_fminf(n1[t].x, n2[t].x));
                    acc = __builtin_fmaf(d, d, acc);
                    d = mv_term(cv[t].y, __builtin_fmaxf(x1[t].y, x2[t].y), __builtin_fminf(n1[t].y, n2[t].y));
                    acc = __builtin_fmaf(d, d, acc);
                    d = mv_term(cv[t].z, __builtin_fmaxf(x1[t].z, x2[t].z), __builtin_fminf(n1[t].z, n2[t].z));
                    acc = __builtin_fmaf(d, d, acc);
                    d = mv_term(cv[t].w, __builtin_fmaxf(x1[t].w, x2[t].w), __builtin_fminf(n1[t].w, n2[t].w));
                    acc = __builtin_fmaf(d, d, acc);
                }
            }
        } else {
            for (int p = 0; p < D; ++p) {
                const float U = __builtin_fmaxf(xk[(int64_t)lo * D + p], xk[(int64_t)h2 * D + p]);
                const float Lw = __builtin_fminf(nk[(int64_t)lo * D + p], nk[(int64_t)h2 * D + p]);
                const float d = mv_term(cs[(int64_t)j * D + p], U, Lw);
                acc = __builtin_fmaf(d, d, acc);
            }
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
        const double N = (double)n * D + 6.0;
        a.lb[(int64_t)q * a.nc + c] = rdown_f((double)acc * (1.0 - (N + 3.0) / 16777216.0 * 1.001));
    }
}

// ----------------------------------------------------------------- DTW
// The DP of one item with K chunks of 4 dimensions (K <= the kernel's NCH).
template <int K>
__device__ __forceinline__ float rknn_pair(const RaggedKnnArgs& a, int q, int ref, int m, int n, int W, int D,
                                           int lane, const Abandon& ab, bool& aband, int& blocks) {
    if (a.abandon)
        return rows_core<float, K, false, true>(0, a.Q + a.q_off[q], a.C + a.c_off[ref], m, n, W, D, lane,
                                                nullptr, ab, aband, &blocks);
    return rows_core<float, K, false, false>(0, a.Q + a.q_off[q], a.C + a.c_off[ref], m, n, W, D, lane,
                                             nullptr, ab, aband, &blocks);
}

template <int K, int NCH>
__device__ __forceinline__ void rknn_pair_if(int nch, float& v, const RaggedKnnArgs& a, int q, int ref, int m,
                                             int n, int W, int D, int lane, const Abandon& ab, bool& aband,
                                             int& blocks) {
    if constexpr (K <= NCH)
        if (nch == K) v = rknn_pair<K>(a, q, ref, m, n, W, D, lane, ab, aband, blocks);
}

// Persistent one-wave blocks over the list items (one pair per item).
template <int NCH>
__global__ __launch_bounds__(64) void k_rknn_dtw(RaggedKnnArgs a) {
    const int lane = threadIdx.x;
    // the items of queries q0 .. q1-1 (every query when q1 is 0)
    const int first = __builtin_amdgcn_readfirstlane(a.q1 > 0 ? a.prefix[a.q0] : 0);
    const int total = __builtin_amdgcn_readfirstlane(a.prefix[a.q1 > 0 ? a.q1 : a.nq]);
    unsigned long long w_started = 0, w_aband = 0, w_cells = 0;
    for (;;) {
        const int item = first + wave_next_item(a.counter);
        if (item >= total) break;
        // every value that steers the loops below is read into a scalar register
        const int q = __builtin_amdgcn_readfirstlane(a.item_query[item]);
        const int e = item - __builtin_amdgcn_readfirstlane(a.prefix[q]);
        const int ref = __builtin_amdgcn_readfirstlane((int)a.list[(int64_t)q * a.cap + e]);
        if (ref < 0) {
            if (lane == 0) a.list_dist[(int64_t)q * a.cap + e] = __builtin_inff();
            continue;
        }
        const int m = __builtin_amdgcn_readfirstlane(a.q_len[q]);
        const int n = __builtin_amdgcn_readfirstlane(a.c_len[ref]);
        const int D = a.q_dim ? __builtin_amdgcn_readfirstlane(a.q_dim[q]) : a.D;
        const int nch = a.q_dim ? nch_pad(D) : NCH;
        const int W = weff_dev(m, n, a.window, a.num, a.den);
        const float gamma = dp_gamma_dev(m, n, nch);
        __syncthreads();
        Abandon ab{a.key + (int64_t)q * kKeyStride, gamma, ~0ull};
        bool aband = false;
        int blocks = 0;
        float v = __builtin_inff();
        if (nch == NCH) {
            v = rknn_pair<NCH>(a, q, ref, m, n, W, D, lane, ab, aband, blocks);
        } else {   // banks of several D: the item's own chunk count
            rknn_pair_if<1, NCH>(nch, v, a, q, ref, m, n, W, D, lane, ab, aband, blocks);
            rknn_pair_if<2, NCH>(nch, v, a, q, ref, m, n, W, D, lane, ab, aband, blocks);
            rknn_pair_if<3, NCH>(nch, v, a, q, ref, m, n, W, D, lane, ab, aband, blocks);
            rknn_pair_if<4, NCH>(nch, v, a, q, ref, m, n, W, D, lane, ab, aband, blocks);
            rknn_pair_if<6, NCH>(nch, v, a, q, ref, m, n, W, D, lane, ab, aband, blocks);
            rknn_pair_if<8, NCH>(nch, v, a, q, ref, m, n, W, D, lane, ab, aband, blocks);
            rknn_pair_if<12, NCH>(nch, v, a, q, ref, m, n, W, D, lane, ab, aband, blocks);
        }
        if (lane == (m - 1) % kRowBlock) {
            float out = __builtin_inff();
            if (!aband) {
                out = v;
                const float up = rup_f((double)v / (1.0 - (double)gamma));
                const unsigned long long k = ((unsigned long long)__float_as_uint(up) << 32) | (uint32_t)ref;
                atomicMin(&a.key[(int64_t)q * kKeyStride], k);
            }
            a.list_dist[(int64_t)q * a.cap + e] = out;
        }
        const int nb = (m + kRowBlock - 1) / kRowBlock;
        const long long cells = band_cells_dev(m, n, W);
        w_started += 1;
        w_aband += aband ? 1 : 0;
        w_cells += aband ? (unsigned long long)((double)cells * blocks / nb) : (unsigned long long)cells;
    }
    if (lane == 0 && w_started) {
        atomicAdd(&a.stats[kStDtwStarted], w_started);
        atomicAdd(&a.stats[kStDtwAbandoned], w_aband);
        atomicAdd(&a.stats[kStCells], w_cells);
    }
}

// ------------------------------------------------------------ finalize
// One wave per query: the smallest float32 DTW over the seeds and the
// survivors, then float64 re-scoring (row mapping) of every candidate
// within (1 + g) / (1 - g) of it, g the largest DP error bound of the
// query's pairs; the smallest float64 value wins, ties to the lowest index.
template <int K>
__device__ __forceinline__ double rknn_rescore(const RaggedKnnArgs& a, int q, int r, int m, int n, int W, int D,
                                               int lane) {
    Abandon ab{nullptr, 0.0f, 0};
    bool aband = false;
    return rows_core<double, K, false, false>(0, a.Q + a.q_off[q], a.C + a.c_off[r], m, n, W, D, lane, nullptr,
                                              ab, aband);
}

template <int K, int NCH>
__device__ __forceinline__ void rknn_rescore_if(int nch, double& v, const RaggedKnnArgs& a, int q, int r, int m,
                                                int n, int W, int D, int lane) {
    if constexpr (K <= NCH)
        if (nch == K) v = rknn_rescore<K>(a, q, r, m, n, W, D, lane);
}

template <int NCH>
__global__ __launch_bounds__(64) void k_rknn_finalize(RaggedKnnArgs a) {
    const int q = blockIdx.x, lane = threadIdx.x;
    const int m = __builtin_amdgcn_readfirstlane(a.q_len[q]);
    const int D = a.q_dim ? __builtin_amdgcn_readfirstlane(a.q_dim[q]) : a.D;
    const int nch = a.q_dim ? nch_pad(D) : NCH;
    float mn = __builtin_inff();
    const int ns = a.R, nl = a.list_cnt[q];
    for (int k = lane; k < ns; k += kWave)
        if (a.seeds[(int64_t)q * ns + k] >= 0) mn = __builtin_fminf(mn, a.seed_dist[(int64_t)q * ns + k]);
    for (int k = lane; k < nl; k += kWave) mn = __builtin_fminf(mn, a.list_dist[(int64_t)q * a.cap + k]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mn = __builtin_fminf(mn, __shfl_xor(mn, o));
    const double g = (double)dp_gamma_dev(m, a.maxn, nch);
    const double thr = (double)mn * ((1.0 + g) / (1.0 - g) * (1.0 + 1e-9));
    double best = __builtin_inf();
    int bestidx = 0x7fffffff;
    int rescored = 0;
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
                const int r = __builtin_amdgcn_readlane(ref, src);
                const int n = __builtin_amdgcn_readfirstlane(a.c_len[r]);
                const int W = weff_dev(m, n, a.window, a.num, a.den);
                __syncthreads();
                double v = __builtin_inf();
                if (nch == NCH) {
                    v = rknn_rescore<NCH>(a, q, r, m, n, W, D, lane);
                } else {
                    rknn_rescore_if<1, NCH>(nch, v, a, q, r, m, n, W, D, lane);
                    rknn_rescore_if<2, NCH>(nch, v, a, q, r, m, n, W, D, lane);
                    rknn_rescore_if<3, NCH>(nch, v, a, q, r, m, n, W, D, lane);
                    rknn_rescore_if<4, NCH>(nch, v, a, q, r, m, n, W, D, lane);
                    rknn_rescore_if<6, NCH>(nch, v, a, q, r, m, n, W, D, lane);
                    rknn_rescore_if<8, NCH>(nch, v, a, q, r, m, n, W, D, lane);
                    rknn_rescore_if<12, NCH>(nch, v, a, q, r, m, n, W, D, lane);
                }
                v = __shfl(v, (m - 1) % kRowBlock);
                ++rescored;
                if (v < best || (v == best && r < bestidx)) { best = v; bestidx = r; }
            }
        }
    }
    if (lane == 0) {
        const int qo = a.q_out ? a.q_out[q] : q;   // the caller's index of the query
        a.nn_idx[qo] = bestidx == 0x7fffffff ? -1 : bestidx;
        a.nn_dist[qo] = (float)best;
        atomicAdd(&a.stats[kStRescored], (unsigned long long)rescored);
        int nseeds = 0;
        for (int k = 0; k < ns; ++k) nseeds += a.seeds[(int64_t)q * ns + k] >= 0;
        const int bank = a.q_dim ? a.q_ce[q] - a.q_cb[q] : a.nc;
        const int pruned = bank - nseeds - nl;
        if (pruned > 0) atomicAdd(&a.stats[kStPrunedMv], (unsigned long long)pruned);
    }
}

// -------------------------------------------------------------- launch
hipError_t launch_rq_tables(const RaggedKnnArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_rq_tables, dim3(a.nq), dim3(256), 0, s, a);
    return hipGetLastError();
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if (blocks > 0) hipLaunchKernelGGL(k_fill_f32, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_rlb_mv(const RaggedKnnArgs& a, hipStream_t s) {
    const dim3 grid(((a.q_dim ? a.bank_max : a.nc) + 3) / 4, a.q1 > 0 ? a.q1 - a.q0 : a.nq);
    if (a.D % 4 != 0 && !a.q_dim) {
        hipLaunchKernelGGL((k_rlb_mv<1, false>), grid, dim3(256), 0, s, a);
    } else {
        switch (nch_pad(a.D)) {
            case 1: hipLaunchKernelGGL((k_rlb_mv<1, true>), grid, dim3(256), 0, s, a); break;
            case 2: hipLaunchKernelGGL((k_rlb_mv<2, true>), grid, dim3(256), 0, s, a); break;
            case 3: hipLaunchKernelGGL((k_rlb_mv<3, true>), grid, dim3(256), 0, s, a); break;
            case 4: hipLaunchKernelGGL((k_rlb_mv<4, true>), grid, dim3(256), 0, s, a); break;
            case 6: hipLaunchKernelGGL((k_rlb_mv<6, true>), grid, dim3(256), 0, s, a); break;
            case 8: hipLaunchKernelGGL((k_rlb_mv<8, true>), grid, dim3(256), 0, s, a); break;
            case 12: hipLaunchKernelGGL((k_rlb_mv<12, true>), grid, dim3(256), 0, s, a); break;
            default: hipLaunchKernelGGL((k_rlb_mv<16, true>), grid, dim3(256), 0, s, a); break;
        }
    }
    return hipGetLastError();
}

size_t rknn_dtw_lds_bytes(int maxn, int D) { return rows_core_lds(maxn, nch_pad(D), 4); }
size_t rknn_final_lds_bytes(int maxn, int D) { return rows_core_lds(maxn, nch_pad(D), 8); }

template <int NCH>
static hipError_t launch_r_nch(const RaggedKnnArgs& a, bool final, int nblocks, hipStream_t s) {
    if (final) {
        hipLaunchKernelGGL(k_rknn_finalize<NCH>, dim3(a.nq), dim3(64), rknn_final_lds_bytes(a.maxn, a.D), s, a);
    } else {
        hipLaunchKernelGGL(k_rknn_dtw<NCH>, dim3(nblocks), dim3(64), rknn_dtw_lds_bytes(a.maxn, a.D), s, a);
    }
    return hipGetLastError();
}

static hipError_t launch_r(const RaggedKnnArgs& a, bool final, int nblocks, hipStream_t s) {
    switch (nch_pad(a.D)) {
        case 1: return launch_r_nch<1>(a, final, nblocks, s);
        case 2: return launch_r_nch<2>(a, final, nblocks, s);
        case 3: return launch_r_nch<3>(a, final, nblocks, s);
        case 4: return launch_r_nch<4>(a, final, nblocks, s);
        case 6: return launch_r_nch<6>(a, final, nblocks, s);
        case 8: return launch_r_nch<8>(a, final, nblocks, s);
        case 12: return launch_r_nch<12>(a, final, nblocks, s);
        case 16: return launch_r_nch<16>(a, final, nblocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rknn_dtw(const RaggedKnnArgs& a, int nblocks, hipStream_t s) { return launch_r(a, false, nblocks, s); }
hipError_t launch_rknn_finalize(const RaggedKnnArgs& a, hipStream_t s) { return launch_r(a, true, 0, s); }

}  // namespace tcdtw
