// Banded DTW forward kernels for gfx950 (Sec. 2, Eq. 1 within the
// Sakoe-Chiba band |i-j| <= W_eff).
//
// Two mappings of the band onto a 64-lane wave; both evaluate the
// recurrence along anti-diagonals, one cell per lane per step, with
// neighbour values passed between lanes by DPP whole-wave shifts:
//
//  * diagonal pairs (W_eff <= 63): the band's 2 W_eff + 1 diagonals plus one
//    padding diagonal are split two per lane, W_eff + 1 lanes per pair, and
//    64 / (W_eff + 1) pairs share a wave.  At anti-diagonal s only the
//    diagonals with the parity of s are live, so each lane alternates
//    between its two diagonals (an "E" step for the even slot, an "O" step
//    for the odd one); the three live anti-diagonals are the lane's two
//    slot registers plus one neighbour value.  Each lane walks its two
//    diagonals one round (two cells) at a time and loads one new query
//    point and one new candidate point per round from LDS.
//  * row-systolic blocks (any W_eff, used above 63): lane l owns row
//    i0 + l of a block of 64 rows and sweeps the block's band columns; the
//    last row of a block is kept in an LDS row buffer for the next block,
//    and the candidate streams through a 128-position LDS ring refilled
//    every 64 steps (so LDS does not grow with the window).
//
// Diagonal pairs stage whole series in LDS as [chunk][t][4] floats
// (conflict-free 16-byte reads) with sentinel points outside the series
// (the ring of the row mapping uses the same sentinels): +inf on the query side,
// -inf on the candidate side, so a cell outside the matrix has cost +inf
// and no edge test is needed.  The single padding diagonal of each pair is
// forced to +inf.
//
// The virtual predecessor of (0,0) is a 0 placed on the slot of diagonal 0
// one round before the start.
#include "dtw_core.h"

namespace tcdtw {

size_t diag_lds_bytes(int m, int n, int W, int D, int P) {
    DiagGeom g;
    g.init(m, n, W);
    return (size_t)P * (size_t)(g.LQ + g.LC) * (size_t)nch_pad(D) * 16;
}

size_t rows_lds_bytes(int n, int W, int D, bool f64) {
    return rows_core_lds(n, nch_pad(D), f64 ? 8 : 4);
}

// ---------------------------------------------------------------------------
// Diagonal-pair mapping.
//
// With off = W + (W & 1) (even) lane l of a group owns the band offsets
// delta = 2l - off (even slot) and 2l + 1 - off (odd slot), so even slots are
// live at even anti-diagonals.  In round r the even slot holds cell
// (r + h - l, r - h + l) and the odd slot (r + h - l, r - h + l + 1),
// h = off / 2.  The padding diagonal is the top odd slot when W is even
// (delta = W + 1) and the bottom even slot when W is odd (delta = -W - 1).
// ---------------------------------------------------------------------------
template <typename T, int NCH, bool SAVE, bool WODD>
__device__ __forceinline__ void diag_item(const DtwFwdArgs& a, int item) {
    const int lane = threadIdx.x;
    int m, n, W, P, D;
    int64_t xoff0 = 0, yoff0 = 0, soff0 = 0;
    int out0;
    if (a.uniform) {
        m = a.m; n = a.n; W = a.W; P = a.P; D = a.D;
        out0 = item * P;
    } else {
        const PairDesc d = a.desc[item];
        m = d.m; n = d.n; W = d.W; P = 1; D = d.D;
        xoff0 = d.xoff; yoff0 = d.yoff; soff0 = d.saved_off; out0 = d.out;
    }
    DiagGeom g;
    g.init(m, n, W);
    const int G = g.G, h = g.h, R = g.R, LQ = g.LQ, LC = g.LC;
    const int per_pair = (LQ + LC) * NCH;   // float4 per staged pair

    int npair_here = P;
    if (a.uniform) npair_here = min(P, a.npairs - out0);
    for (int gg = 0; gg < npair_here; ++gg) {
        const float* xs = a.uniform ? a.x + (int64_t)(out0 + gg) * m * D : a.x + xoff0;
        const float* ys = a.uniform ? a.y + (int64_t)(out0 + gg) * n * D : a.y + yoff0;
        const int sq = gg * per_pair;
        stage_series<NCH>(sq, LQ, g.qfirst(), xs, m, D, __builtin_inff(), lane, kWave);
        stage_series<NCH>(sq + LQ * NCH, LC, g.cfirst(), ys, n, D, -__builtin_inff(), lane, kWave);
    }
    __syncthreads();

    const int grp = lane / G;
    const int lg = lane - grp * G;
    const bool spare = grp >= npair_here;          // lanes without a pair
    const int gsrc = spare ? 0 : grp;              // spare lanes read group 0's data
    const bool kill_e = WODD && (lg == 0 || spare);
    const bool kill_o = !WODD && (lg == G - 1);
    const int qb = gsrc * per_pair + (W - lg);
    const int cb = gsrc * per_pair + LQ * NCH + lg;

    const T INF = inf_v<T>();
    T vE = INF, vO = INF;
    if (!spare && lg == h) vE = T(0);              // virtual D(-1,-1)
    uint32_t* codes = nullptr;
    if (SAVE && !spare)
        codes = a.codes + (a.uniform ? (int64_t)(out0 + grp) * a.codes_stride : soff0);
    Abandon ab{nullptr, 0.0f, 0};
    bool aband = false;
    diag_core<T, NCH, SAVE, WODD, false>(qb, LQ, cb, LC, R, G, lg, kill_e, kill_o, vE, vO, codes, ab,
                                         aband, 0);

    const int sigma = (n - m) + 2 * h;             // cell (m-1, n-1) lies on diagonal n-m
    if (!spare && lg == (sigma >> 1)) {
        const T v = (sigma & 1) ? vO : vE;
        const int out = a.uniform ? out0 + grp : out0;
        a.dist[out] = (float)v;
        if (a.dist64) a.dist64[out] = (double)v;
    }
}

// One item per block, or persistent waves over a.nitems items.
template <typename T, int NCH, bool SAVE, bool WODD>
__global__ __launch_bounds__(64) void dtw_diag_kernel(DtwFwdArgs a) {
    if (!a.counter) {
        diag_item<T, NCH, SAVE, WODD>(a, blockIdx.x);
        return;
    }
    for (;;) {
        const int item = wave_next_item(a.counter);
        if (item >= a.nitems) break;
        __syncthreads();
        diag_item<T, NCH, SAVE, WODD>(a, item);
    }
}

// ---------------------------------------------------------------------------
// Row-systolic mapping: one pair per wave.  Block b holds rows
// i0 = 64 b .. i0 + 63; lane l owns row i0 + l and at step t evaluates
// column j = jlo + t - l.  up = lane l-1's previous value (lane 0: the
// row buffer), diag = the up value of the previous step, left = own
// previous value.  Lane 63 writes its row into the row buffer 63 columns
// behind lane 0's reads, so one buffer serves both.  The candidate streams
// through a ring (rows_core in dtw_core.h).
// ---------------------------------------------------------------------------
template <typename T, int NCH, bool SAVE>
__device__ __forceinline__ void rows_item(const DtwFwdArgs& a, int item) {
    const int lane = threadIdx.x;
    int m, n, W, out, D;
    int64_t xoff, yoff, soff;
    if (a.uniform) {
        m = a.m; n = a.n; W = a.W; D = a.D;
        out = item;
        xoff = (int64_t)out * m * D; yoff = (int64_t)out * n * D;
        soff = (int64_t)out * a.codes_stride;
    } else {
        const PairDesc d = a.desc[item];
        m = d.m; n = d.n; W = d.W; out = d.out; D = d.D;
        xoff = d.xoff; yoff = d.yoff; soff = d.saved_off;
    }
    Abandon ab{nullptr, 0.0f, 0};
    bool aband = false;
    const T v = rows_core<T, NCH, SAVE, false>(0, a.x + xoff, a.y + yoff, m, n, W, D, lane,
                                               SAVE ? a.codes + soff : nullptr, ab, aband);
    if (lane == (m - 1) % kRowBlock) {
        a.dist[out] = (float)v;
        if (a.dist64) a.dist64[out] = (double)v;
    }
}

template <typename T, int NCH, bool SAVE>
__global__ __launch_bounds__(64) void dtw_rows_kernel(DtwFwdArgs a) {
    if (!a.counter) {
        rows_item<T, NCH, SAVE>(a, blockIdx.x);
        return;
    }
    for (;;) {
        const int item = wave_next_item(a.counter);
        if (item >= a.nitems) break;
        __syncthreads();
        rows_item<T, NCH, SAVE>(a, item);
    }
}

// ---------------------------------------------------------------------------
// Diagonal pairs with the point costs formed ahead of the recurrence (float,
// uniform pairs).  A workgroup of sixteen waves takes one item (the P pairs
// of one wave of dtw_diag_kernel, same lane layout): after the pairs are
// staged and the costs of the first chunk of rounds formed, waves 1-15 form
// the costs of chunk c + 1 (cells of both slots of every lane, +inf on killed
// slots, spare lanes and cells outside the matrix) into one half of an LDS
// double buffer while wave 0 runs the recurrence over chunk c from the other
// half.  The serial chain of a round is then two cost reads, two 3-way
// minima, two adds and two lane shifts; the argmin codes (when saved) are
// written in diag_core's layout, so tc_dtw_backward reads them unchanged.
// This mapping is for batches too small to fill the chip with one wave per
// item, whose time is the latency of the serial chain (more cost waves keep
// the recurrence wave's SIMD freer: 41.7 us with eight waves, 38.4 us with
// sixteen, for 256 pairs of 512 at d = 12).
// ---------------------------------------------------------------------------
constexpr int kCoopRounds = 32;   // rounds per chunk (a multiple of 8: code words never straddle chunks)
constexpr int kCoopThreads = 1024; // one recurrence wave and fifteen cost waves

size_t diag_coop_lds_bytes(int m, int n, int W, int D, int P) {
    return diag_lds_bytes(m, n, W, D, P) + (size_t)2 * kCoopRounds * kWave * 8;
}

template <int NCH, bool SAVE, bool WODD>
__global__ __launch_bounds__(1024) void dtw_diag_coop_kernel(DtwFwdArgs a) {
    const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
    const int m = a.m, n = a.n, W = a.W, P = a.P, D = a.D;
    const int out0 = blockIdx.x * P;
    const int npair_here = min(P, a.npairs - out0);
    DiagGeom g;
    g.init(m, n, W);
    const int G = g.G, h = g.h, R = g.R, LQ = g.LQ, LC = g.LC;
    const int per_pair = (LQ + LC) * NCH;
    const float INF = __builtin_inff();
    for (int gg = 0; gg < npair_here; ++gg) {
        const float* xs = a.x + (int64_t)(out0 + gg) * m * D;
        const float* ys = a.y + (int64_t)(out0 + gg) * n * D;
        const int sq = gg * per_pair;
        stage_series<NCH>(sq, LQ, g.qfirst(), xs, m, D, INF, tid, blockDim.x);
        stage_series<NCH>(sq + LQ * NCH, LC, g.cfirst(), ys, n, D, -INF, tid, blockDim.x);
    }
    float2* cbuf = reinterpret_cast<float2*>(lds4 + P * per_pair);   // [2][kCoopRounds][64]
    const int nchunks = (R + kCoopRounds - 1) / kCoopRounds;
    // Costs of the E and O cells of lane `ln` for rounds [r0, r1) of chunk c: one thread walks
    // consecutive rounds, so the O step's candidate point is the next round's E point.
    auto produce = [&](int c, int ln, int r0, int r1) __attribute__((always_inline)) {
        float2* dst = cbuf + (c & 1) * kCoopRounds * kWave + ln;
        const int rbase = c * kCoopRounds;
        const int grp = ln / G, lg = ln - grp * G;
        if (grp >= npair_here) {
            for (int rr = r0; rr < r1; ++rr) dst[rr * kWave] = make_float2(INF, INF);
            return;
        }
        const int qpos = grp * per_pair + (W - lg) + rbase;
        const int cpos = grp * per_pair + LQ * NCH + lg + rbase;
        const bool ke = WODD && lg == 0, ko = !WODD && lg == G - 1;
        if (r0 >= r1) return;
        // the next round's points are read before this round's arithmetic
        float4 cc[NCH], qn[NCH], cnn[NCH];
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            cc[k] = lds4[cpos + k * LC + r0];
            qn[k] = lds4[qpos + k * LQ + r0];
            cnn[k] = lds4[cpos + k * LC + r0 + 1];
        }
        for (int rr = r0; rr < r1; ++rr) {
            float4 qv[NCH], cn[NCH];
#pragma unroll
            for (int k = 0; k < NCH; ++k) {
                qv[k] = qn[k];
                cn[k] = cnn[k];
            }
            if (rr + 1 < r1) {
#pragma unroll
                for (int k = 0; k < NCH; ++k) {
                    qn[k] = lds4[qpos + k * LQ + rr + 1];
                    cnn[k] = lds4[cpos + k * LC + rr + 2];
                }
            }
            float2 v;
            v.x = ke ? INF : point_cost<NCH>(qv, cc, 0.0f);
            v.y = ko ? INF : point_cost<NCH>(qv, cn, 0.0f);
            dst[rr * kWave] = v;
#pragma unroll
            for (int k = 0; k < NCH; ++k) cc[k] = cn[k];
        }
    };
    // the chunk's rounds split into nparts consecutive runs, part `part` of them
    auto produce_part = [&](int c, int ln, int part, int nparts) __attribute__((always_inline)) {
        const int rows = min(kCoopRounds, R - c * kCoopRounds);
        const int per = (rows + nparts - 1) / nparts;
        produce(c, ln, min(rows, part * per), min(rows, (part + 1) * per));
    };
    __syncthreads();
    const int nw = blockDim.x / kWave;
    produce_part(0, lane, wv, nw);
    __syncthreads();
    // recurrence state of wave 0
    const int grp = lane / G, lg = lane - grp * G;
    const bool spare = grp >= npair_here;
    float vE = INF, vO = INF;
    if (!spare && lg == h) vE = 0.0f;              // virtual D(-1,-1)
    uint32_t* codes = nullptr;
    if (SAVE && !spare) codes = a.codes + (int64_t)(out0 + grp) * a.codes_stride;
    // the recurrence's wave is first in issue arbitration: the producers fill its dependency gaps
    if (wv == 0) __builtin_amdgcn_s_setprio(3);
    for (int c = 0; c < nchunks; ++c) {
        if (wv == 0) {
            const float2* src = cbuf + (c & 1) * kCoopRounds * kWave + lane;
            const int rbase = c * kCoopRounds;
            const int rows = __builtin_amdgcn_readfirstlane(min(kCoopRounds, R - rbase));
            // groups of eight rounds; the next group's costs are read before this group's
            // recurrence so that the LDS latency is off the serial chain
            float2 cur[8], nxt[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) cur[u] = src[min(u, rows - 1) * kWave];
            for (int g0 = 0; g0 < rows; g0 += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) nxt[u] = src[min(g0 + 8 + u, rows - 1) * kWave];
                uint32_t cw = 0;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (g0 + u < rows) {
                        // neighbour values by whole-wave rotations: lane 0 receives lane 63's odd
                        // slot and lane 63 lane 0's even slot, which are +inf or feed a killed step
                        // (a killed or spare slot has cost +inf: lane 63's odd slot without WODD,
                        // lane 0's even slot with it)
                        {   // E step: diag = own even slot, up = own odd slot, left = lane-1's odd slot
                            const float left = __uint_as_float(wave_ror1(__float_as_uint(vO)));
                            float best;
                            if (SAVE) {
                                uint32_t code;
                                best = min3_code(vE, vO, left, code);
                                cw |= code << (u * 4);
                            } else {
                                best = __uint_as_float(umin3(__float_as_uint(vE), __float_as_uint(vO),
                                                             __float_as_uint(left)));
                            }
                            vE = cur[u].x + best;
                        }
                        {   // O step: diag = own odd slot, up = lane+1's even slot, left = own even slot
                            const float up = __uint_as_float(wave_rol1(__float_as_uint(vE)));
                            float best;
                            if (SAVE) {
                                uint32_t code;
                                best = min3_code(vO, up, vE, code);
                                cw |= code << (u * 4 + 2);
                            } else {
                                best = __uint_as_float(umin3(__float_as_uint(vO), __float_as_uint(up),
                                                             __float_as_uint(vE)));
                            }
                            vO = cur[u].y + best;
                        }
                    }
                }
                if (SAVE && codes) codes[(int64_t)((rbase + g0) >> 3) * G + lg] = cw;
#pragma unroll
                for (int u = 0; u < 8; ++u) cur[u] = nxt[u];
            }
        } else if (c + 1 < nchunks) {
            produce_part(c + 1, lane, wv - 1, nw - 1);
        }
        __syncthreads();
    }
    if (wv == 0) {
        const int sigma = (n - m) + 2 * h;             // cell (m-1, n-1) lies on diagonal n-m
        if (!spare && lg == (sigma >> 1)) a.dist[out0 + grp] = (sigma & 1) ? vO : vE;
    }
}

template <int NCH, bool SAVE>
static void launch_coop_nch(const DtwFwdArgs& a, int grid, size_t lds, hipStream_t s) {
    if (a.wodd) hipLaunchKernelGGL((dtw_diag_coop_kernel<NCH, SAVE, true>), dim3(grid), dim3(kCoopThreads), lds, s, a);
    else hipLaunchKernelGGL((dtw_diag_coop_kernel<NCH, SAVE, false>), dim3(grid), dim3(kCoopThreads), lds, s, a);
}

// Uniform pairs, W_eff <= 63, a.P pairs per item, float; one workgroup per item.
hipError_t launch_dtw_diag_coop(const DtwFwdArgs& a, bool save, int nitems, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const size_t lds = diag_coop_lds_bytes(a.m, a.n, a.W, a.D, a.P);
    switch (nch_pad(a.D)) {
#define TC_COOP_CASE(N) \
        case N: save ? launch_coop_nch<N, true>(a, nitems, lds, s) : launch_coop_nch<N, false>(a, nitems, lds, s); break;
        TC_COOP_CASE(1) TC_COOP_CASE(2) TC_COOP_CASE(3) TC_COOP_CASE(4)
        TC_COOP_CASE(6) TC_COOP_CASE(8) TC_COOP_CASE(12) TC_COOP_CASE(16)
#undef TC_COOP_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row mapping with K waves per pair (rows_core_pipe): persistent workgroups
// of 64 K threads take pairs from a device counter.  LDS: K candidate rings,
// the row buffer of the launch's longest candidate, K progress counters, the
// current item and a flag raised when a wait ran out (the pair's distance is
// then NaN).
// ---------------------------------------------------------------------------
template <typename T, int NCH, bool SAVE>
__global__ __launch_bounds__(512) void dtw_rows_pipe_kernel(DtwFwdArgs a) {
    const int K = blockDim.x / kWave;
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const T INF = inf_v<T>();
    T* rowbuf = reinterpret_cast<T*>(lds4 + K * kRowStride * NCH);
    const size_t rb_bytes = ((size_t)(a.n + 2 * kRowPad) * sizeof(T) + 15) & ~(size_t)15;
    int* prog = reinterpret_cast<int*>(reinterpret_cast<char*>(rowbuf) + rb_bytes);
    int* sitem = prog + K;
    int* sflag = sitem + 1;
    for (;;) {
        if (threadIdx.x == 0) *sitem = atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(*sitem);
        if (item >= a.nitems) break;
        const PairDesc d = a.desc[item];
        const int m = d.m, n = d.n, W = d.W, D = d.D;
        const int LB = n + 2 * kRowPad;
        for (int pos = threadIdx.x; pos < LB; pos += blockDim.x) rowbuf[pos] = (pos == kRowPad - 1) ? T(0) : INF;
        if (threadIdx.x < K) prog[threadIdx.x] = -1;
        if (threadIdx.x == 0) *sflag = 0;
        __syncthreads();
        bool late = false;
        const T v = rows_core_pipe<T, NCH, SAVE>(wv * kRowStride * NCH, rowbuf, prog, K, wv, a.x + d.xoff,
                                                 a.y + d.yoff, m, n, W, D, lane,
                                                 SAVE ? a.codes + d.saved_off : nullptr, late);
        if (late) *sflag = 1;
        __syncthreads();
        if (wv == ((m - 1) / kRowBlock) % K && lane == (m - 1) % kRowBlock) {
            const bool bad = *sflag != 0;
            a.dist[d.out] = bad ? __builtin_nanf("") : (float)v;
            if (a.dist64) a.dist64[d.out] = bad ? __builtin_nan("") : (double)v;
            if (bad && a.status) atomicOr(a.status, kStatusWaitExpired);
        }
        __syncthreads();
    }
}

template <typename T, int NCH, bool SAVE>
static hipError_t launch_pipe_nch(const DtwFwdArgs& a, int K, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((dtw_rows_pipe_kernel<T, NCH, SAVE>), dim3(grid), dim3(kWave * K), lds, s, a);
    return hipGetLastError();
}

template <typename T, bool SAVE>
static hipError_t launch_pipe_t(const DtwFwdArgs& a, int K, int grid, size_t lds, hipStream_t s) {
    switch (nch_pad(a.D)) {
        case 1: return launch_pipe_nch<T, 1, SAVE>(a, K, grid, lds, s);
        case 2: return launch_pipe_nch<T, 2, SAVE>(a, K, grid, lds, s);
        case 3: return launch_pipe_nch<T, 3, SAVE>(a, K, grid, lds, s);
        case 4: return launch_pipe_nch<T, 4, SAVE>(a, K, grid, lds, s);
        case 6: return launch_pipe_nch<T, 6, SAVE>(a, K, grid, lds, s);
        case 8: return launch_pipe_nch<T, 8, SAVE>(a, K, grid, lds, s);
        case 12: return launch_pipe_nch<T, 12, SAVE>(a, K, grid, lds, s);
        case 16: return launch_pipe_nch<T, 16, SAVE>(a, K, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

size_t pipe_lds_bytes(int maxn, int D, int K, bool f64) {
    return rows_pipe_lds(maxn, nch_pad(D), K, f64 ? 8 : 4);
}

// a.counter and a.desc set, a.n / a.D the launch's largest; `grid` workgroups of K waves.
hipError_t launch_dtw_rows_pipe(const DtwFwdArgs& a, bool f64, bool save, int K, int nitems, int grid,
                                hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (K < 2 || K > 8 || !a.counter) return hipErrorInvalidValue;
    DtwFwdArgs b = a;
    b.nitems = nitems;
    const size_t lds = pipe_lds_bytes(b.n, b.D, K, f64);
    if (f64) return save ? launch_pipe_t<double, true>(b, K, grid, lds, s) : launch_pipe_t<double, false>(b, K, grid, lds, s);
    return save ? launch_pipe_t<float, true>(b, K, grid, lds, s) : launch_pipe_t<float, false>(b, K, grid, lds, s);
}

// ---------------------------------------------------------------------------
// Launch: the mapping is chosen by the largest W_eff of the launch.
// ---------------------------------------------------------------------------

template <typename T, int NCH, bool SAVE>
static hipError_t launch_nch(const DtwFwdArgs& a, bool rows, int grid, size_t lds, hipStream_t s) {
    if (!rows) {
        // every item of a launch shares the parity of W (a ragged caller splits by parity)
        if (a.wodd) {
            hipLaunchKernelGGL((dtw_diag_kernel<T, NCH, SAVE, true>), dim3(grid), dim3(64), lds, s, a);
        } else {
            hipLaunchKernelGGL((dtw_diag_kernel<T, NCH, SAVE, false>), dim3(grid), dim3(64), lds, s, a);
        }
    } else {
        hipLaunchKernelGGL((dtw_rows_kernel<T, NCH, SAVE>), dim3(grid), dim3(64), lds, s, a);
    }
    return hipGetLastError();
}

template <typename T, bool SAVE>
static hipError_t launch_t(const DtwFwdArgs& a, bool rows, int grid, size_t lds, hipStream_t s) {
    switch (nch_pad(a.D)) {
        case 1: return launch_nch<T, 1, SAVE>(a, rows, grid, lds, s);
        case 2: return launch_nch<T, 2, SAVE>(a, rows, grid, lds, s);
        case 3: return launch_nch<T, 3, SAVE>(a, rows, grid, lds, s);
        case 4: return launch_nch<T, 4, SAVE>(a, rows, grid, lds, s);
        case 6: return launch_nch<T, 6, SAVE>(a, rows, grid, lds, s);
        case 8: return launch_nch<T, 8, SAVE>(a, rows, grid, lds, s);
        case 12: return launch_nch<T, 12, SAVE>(a, rows, grid, lds, s);
        case 16: return launch_nch<T, 16, SAVE>(a, rows, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

// Clears n counters with a kernel (a memset node misbehaves under graph replay).
__global__ void k_zero_i32(int32_t* p, int n) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) p[t] = 0;
}

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

size_t fwd_lds_bytes(const DtwFwdArgs& a, bool rows, bool f64) {
    return rows ? rows_lds_bytes(a.n, a.W, a.D, f64) : diag_lds_bytes(a.m, a.n, a.W, a.D, a.P);
}

// a.m, a.n, a.W, a.D: the largest of the launch (they size the LDS); with
// a.counter set, `grid` persistent waves share the a.nitems items.
hipError_t launch_dtw_fwd(const DtwFwdArgs& a, bool f64, bool save, bool rows, int nitems, int grid,
                          hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    DtwFwdArgs b = a;
    b.nitems = nitems;
    const int g = b.counter ? grid : nitems;
    const size_t lds = fwd_lds_bytes(b, rows, f64);
    if (f64) return save ? launch_t<double, true>(b, rows, g, lds, s) : launch_t<double, false>(b, rows, g, lds, s);
    return save ? launch_t<float, true>(b, rows, g, lds, s) : launch_t<float, false>(b, rows, g, lds, s);
}

}  // namespace tcdtw
