// Banded DTW backward for gfx950: gradient of DTW(x, y) with respect to
// both series along the optimal warping path that the forward recorded
// as 2-bit argmin codes (0 = diagonal, 1 = (i-1,j), 2 = (i,j-1)).
//
// One wave per pair:
//   1. the pair's codes are copied to LDS when they fit;
//   2. lane 0 walks the path back from (m-1, n-1) to (0, 0); a monotone
//      path meets every row i in one run of columns [rlo_i, rhi_i] and
//      every column j in one run of rows [clo_j, chi_j], which are kept in
//      LDS;
//   3. lanes over rows form grad_x[i] = g * sum_{j in run} 2 (x_i - y_j),
//      lanes over columns grad_y[j] = g * sum_{i in run} 2 (y_j - x_i),
//      accumulated in float64 and rounded once to float32.
#include "device_common.h"
#include "internal.h"

namespace tcdtw {

constexpr int kBwdCodeLdsWords = 12288;   // 48 KB of staged codes


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
    const int lane = threadIdx.x;
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
    CodeMap cm;
    cm.init(m, n, W, rows);
    const int64_t words = codes_words(m, n, W, rows);
    const bool staged = words <= a.stage_cap;
    const uint32_t* gcodes = a.codes + soff;
    if (staged) {
        for (int64_t w = lane; w < words; w += kWave) scodes[w] = gcodes[w];
    }
    __syncthreads();

    if (lane == 0) {
        int i = m - 1, j = n - 1;
        rhi[i] = j;
        chi[j] = i;
        while (i > 0 || j > 0) {
            int64_t w;
            int sh;
            cm.locate(i, j, w, sh);
            const uint32_t word = staged ? scodes[w] : gcodes[w];
            const int code = (word >> sh) & 3;
            int pi = i, pj = j;
            if (code == 0) { pi = i - 1; pj = j - 1; }
            else if (code == 1) { pi = i - 1; }
            else { pj = j - 1; }
            if (pi != i) { rlo[i] = j; rhi[pi] = pj; }
            if (pj != j) { clo[j] = i; chi[pj] = pi; }
            i = pi; j = pj;
        }
        rlo[0] = 0;
        clo[0] = 0;
    }
    __syncthreads();

    const float g2 = 2.0f * a.grad_dist[pid];
    const float* xs = a.x + xoff;
    const float* ys = a.y + yoff;
    float* gx = a.grad_x + xoff;
    float* gy = a.grad_y + yoff;
    for (int i = lane; i < m; i += kWave) {
        const int j0 = rlo[i], j1 = rhi[i];
        for (int p = 0; p < D; ++p) {
            const double xv = xs[(int64_t)i * D + p];
            double acc = 0.0;
            for (int j = j0; j <= j1; ++j) acc += xv - (double)ys[(int64_t)j * D + p];
            gx[(int64_t)i * D + p] = (float)((double)g2 * acc);
        }
    }
    for (int j = lane; j < n; j += kWave) {
        const int i0 = clo[j], i1 = chi[j];
        for (int p = 0; p < D; ++p) {
            const double yv = ys[(int64_t)j * D + p];
            double acc = 0.0;
            for (int i = i0; i <= i1; ++i) acc += yv - (double)xs[(int64_t)i * D + p];
            gy[(int64_t)j * D + p] = (float)((double)g2 * acc);
        }
    }
}

__global__ __launch_bounds__(64) void dtw_bwd_kernel(DtwBwdArgs a) {
    if (!a.counter) {
        bwd_item(a, blockIdx.x);
        return;
    }
    for (;;) {
        const int item = wave_next_item(a.counter);
        if (item >= a.nitems) break;
        __syncthreads();
        bwd_item(a, item);
    }
}

size_t bwd_lds_bytes(int maxm, int maxn, int64_t max_words) {
    const int64_t cap = max_words < kBwdCodeLdsWords ? max_words : kBwdCodeLdsWords;
    return (size_t)(2 * (maxm + maxn)) * 4 + (size_t)cap * 4;
}

hipError_t launch_dtw_bwd(const DtwBwdArgs& a, int maxm, int maxn, int64_t max_words, int nitems,
                          int grid, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    DtwBwdArgs b = a;
    b.runs_ints = 2 * (maxm + maxn);
    // the kernel stages a pair's codes only when they fit the reserved words
    b.stage_cap = max_words < kBwdCodeLdsWords ? max_words : kBwdCodeLdsWords;
    b.nitems = nitems;
    const size_t lds = bwd_lds_bytes(maxm, maxn, max_words);
    hipLaunchKernelGGL(dtw_bwd_kernel, dim3(b.counter ? grid : nitems), dim3(64), lds, s, b);
    return hipGetLastError();
}

}  // namespace tcdtw
