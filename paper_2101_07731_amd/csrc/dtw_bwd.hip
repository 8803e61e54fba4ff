// Banded DTW backward for gfx950: gradient of DTW(x, y) with respect to
// both series along the optimal warping path that the forward recorded
// as 2-bit argmin codes (0 = diagonal, 1 = (i-1,j), 2 = (i,j-1)).
//
// One block of 256 threads per pair:
//   1. the pair's codes, and both series when they fit, are copied to LDS
//      (eight loads in flight per thread);
//   2. wave 0 walks the path back from (m-1, n-1) to (0, 0) at a
//      wave-uniform position, its lanes holding the 64 code words around
//      it (consecutive steps mostly stay among them), each step reading its
//      word from the lane that holds it; a monotone path meets every row i in one run of columns
//      [rlo_i, rhi_i] and every column j in one run of rows [clo_j, chi_j],
//      which are kept in LDS;
//   3. threads over (row, dimension) form grad_x[i][p] = g * sum_{j in run}
//      2 (x_ip - y_jp), threads over (column, dimension) grad_y likewise,
//      accumulated in float64 in increasing j (i) and rounded once to
//      float32.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace tcdtw {

constexpr int kBwdCodeLdsWords = 12288;   // 48 KB of staged codes
constexpr int kBwdSeriesLdsFloats = 16384; // 64 KB of staged series (x then y)
constexpr int kBwdThreads = 256;


struct CodeMap {
    // diagonal layout
    int G, off;
    // row layout
    int W, nwb;
    bool diag;
    __device__ void init(int m, int n, int W_, bool rows) {
        W = W_;
        diag = !rows;
        G = W + 1;
        off = W + (W & 1);
        const int tmax = min(n, 2 * W + kRowBlock) + kRowBlock - 1;
        nwb = (tmax + 15) / 16;
        (void)m;
    }
    // The word of (i, j) as base + ln with 0 <= ln < 64: the words base .. base + 63 are one
    // round block of every band offset (diagonal) or one step block of every row of a 64-row
    // block (rows).
    __device__ __forceinline__ void locate64(int i, int j, int64_t& base, int& ln, int& shift) const {
        if (diag) {
            const int sigma = (j - i) + off;
            const int slot = sigma & 1;
            const int r = (i + j - slot) >> 1;
            ln = sigma >> 1;
            base = (int64_t)(r >> 3) * G;
            shift = (r & 7) * 4 + 2 * slot;
        } else {
            const int b = i / kRowBlock, l = i - b * kRowBlock;
            const int jlo = max(0, b * kRowBlock - W);
            const int t = j - jlo + l;
            ln = l;
            base = ((int64_t)b * nwb + (t >> 4)) * kWave;
            shift = (t & 15) * 2;
        }
    }
    __device__ __forceinline__ void locate(int i, int j, int64_t& word, int& shift) const {
        if (diag) {
            const int sigma = (j - i) + off;
            const int ln = sigma >> 1, slot = sigma & 1;
            const int r = (i + j - slot) >> 1;
            word = (int64_t)(r >> 3) * G + ln;
            shift = (r & 7) * 4 + 2 * slot;
        } else {
            const int b = i / kRowBlock, l = i - b * kRowBlock;
            const int jlo = max(0, b * kRowBlock - W);
            const int t = j - jlo + l;
            word = ((int64_t)b * nwb + (t >> 4)) * kWave + l;
            shift = (t & 15) * 2;
        }
    }
};

__device__ void bwd_item(const DtwBwdArgs& a, int item) {
    extern __shared__ int32_t sbw[];
    const int tid = threadIdx.x;
    int m, n, W, pid, D;
    bool rows;
    int64_t xoff, yoff, soff;
    if (a.uniform) {
        m = a.m; n = a.n; W = a.W; pid = item; D = a.D;
        rows = a.urows != 0;
        xoff = (int64_t)pid * m * a.D; yoff = (int64_t)pid * n * a.D;
        soff = (int64_t)pid * a.codes_stride;
    } else {
        const PairDesc d = a.desc[item];
        m = d.m; n = d.n; W = d.W; pid = d.out; D = d.D; rows = d.rows != 0;
        xoff = d.xoff; yoff = d.yoff; soff = d.saved_off;
    }
    int32_t* rlo = sbw;
    int32_t* rhi = rlo + m;
    int32_t* clo = rhi + m;
    int32_t* chi = clo + n;
    uint32_t* scodes = reinterpret_cast<uint32_t*>(sbw + a.runs_ints);
    float* sser = reinterpret_cast<float*>(scodes + a.stage_cap);
    CodeMap cm;
    cm.init(m, n, W, rows);
    const int64_t words = codes_words(m, n, W, rows);
    const bool staged = words <= a.stage_cap;
    const bool sstaged = (int64_t)(m + n) * D <= a.series_cap;
    const uint32_t* gcodes = a.codes + soff;
    const float* xs = a.x + xoff;
    const float* ys = a.y + yoff;
    if (staged) copy_to_lds(scodes, gcodes, words, tid, kBwdThreads);
    if (sstaged) {
        copy_to_lds(sser, xs, (int64_t)m * D, tid, kBwdThreads);
        copy_to_lds(sser + m * D, ys, (int64_t)n * D, tid, kBwdThreads);
    }
    __syncthreads();

    if (tid < kWave) {
        // wave 0 walks with wave-uniform (scalar) position: each lane holds one word of the
        // current block of 64 (reloaded when the path leaves it) and a step reads its word
        // from the lane that holds it, with no LDS round trip; lane 0 writes the runs
        const int lane = tid;
        int i = m - 1, j = n - 1;
        if (lane == 0) { rhi[i] = j; chi[j] = i; }
        int64_t cur = -1;
        uint32_t held = 0;
        while (i > 0 || j > 0) {
            int64_t base;
            int ln, sh;
            cm.locate64(i, j, base, ln, sh);
            if (base != cur) {
                const int64_t w = base + lane;
                held = w < words ? (staged ? scodes[w] : gcodes[w]) : 0u;
                cur = base;
            }
            const uint32_t word = (uint32_t)__builtin_amdgcn_readlane((int)held, ln);
            const int code = (word >> sh) & 3;
            int pi = i, pj = j;
            if (code == 0) { pi = i - 1; pj = j - 1; }
            else if (code == 1) { pi = i - 1; }
            else { pj = j - 1; }
            if (lane == 0) {
                if (pi != i) { rlo[i] = j; rhi[pi] = pj; }
                if (pj != j) { clo[j] = i; chi[pj] = pi; }
            }
            i = pi; j = pj;
        }
        if (lane == 0) { rlo[0] = 0; clo[0] = 0; }
    }
    __syncthreads();

    const float g2 = 2.0f * a.grad_dist[pid];
    const float* xv_src = sstaged ? sser : xs;
    const float* yv_src = sstaged ? sser + m * D : ys;
    float* gx = a.grad_x + xoff;
    float* gy = a.grad_y + yoff;
    for (int t = tid; t < m * D; t += kBwdThreads) {
        const int i = t / D, p = t - i * D;
        const int j0 = rlo[i], j1 = rhi[i];
        const double xv = xv_src[t];
        double acc = 0.0;
        for (int j = j0; j <= j1; ++j) acc += xv - (double)yv_src[j * D + p];
        gx[t] = (float)((double)g2 * acc);
    }
    for (int t = tid; t < n * D; t += kBwdThreads) {
        const int j = t / D, p = t - j * D;
        const int i0 = clo[j], i1 = chi[j];
        const double yv = yv_src[t];
        double acc = 0.0;
        for (int i = i0; i <= i1; ++i) acc += yv - (double)xv_src[i * D + p];
        gy[t] = (float)((double)g2 * acc);
    }
}

__global__ __launch_bounds__(kBwdThreads) void dtw_bwd_kernel(DtwBwdArgs a) {
    if (!a.counter) {
        bwd_item(a, blockIdx.x);
        return;
    }
    __shared__ int s_item;
    for (;;) {
        __syncthreads();   // the previous item's LDS is free, s_item may be rewritten
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= a.nitems) break;
        bwd_item(a, item);
    }
}

static int64_t bwd_series_cap(int maxm, int maxn, int maxd) {
    const int64_t f = (int64_t)(maxm + maxn) * maxd;
    return f <= kBwdSeriesLdsFloats ? f : 0;
}

size_t bwd_lds_bytes(int maxm, int maxn, int64_t max_words, int maxd) {
    const int64_t cap = max_words < kBwdCodeLdsWords ? max_words : kBwdCodeLdsWords;
    return (size_t)(2 * (maxm + maxn)) * 4 + (size_t)cap * 4 + (size_t)bwd_series_cap(maxm, maxn, maxd) * 4;
}

hipError_t launch_dtw_bwd(const DtwBwdArgs& a, int maxm, int maxn, int64_t max_words, int maxd, int nitems,
                          int grid, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    DtwBwdArgs b = a;
    b.runs_ints = 2 * (maxm + maxn);
    // the kernel stages a pair's codes (series) only when they fit the reserved words
    b.stage_cap = max_words < kBwdCodeLdsWords ? max_words : kBwdCodeLdsWords;
    b.series_cap = bwd_series_cap(maxm, maxn, maxd);
    b.nitems = nitems;
    const size_t lds = bwd_lds_bytes(maxm, maxn, max_words, maxd);
    const int blocks = b.counter ? std::max(1, std::min(grid, nitems)) : nitems;
    hipLaunchKernelGGL(dtw_bwd_kernel, dim3(blocks), dim3(kBwdThreads), lds, s, b);
    return hipGetLastError();
}

}  // namespace tcdtw
