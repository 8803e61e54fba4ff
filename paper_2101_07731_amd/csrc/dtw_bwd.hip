// Banded DTW backward for gfx950: gradient of DTW(x, y) with respect to
// both series along the optimal warping path that the forward recorded
// as 2-bit argmin codes (0 = diagonal, 1 = (i-1,j), 2 = (i,j-1)).
//
// One block of 256 threads per pair:
//   1. the pair's codes are copied to LDS (eight loads in flight per thread);
//   2. wave 0 walks the path back from (m-1, n-1) to (0, 0) at a
//      wave-uniform position, its lanes holding the 64 code words around
//      it (consecutive steps mostly stay among them; on the diagonal layout
//      the next block back is read ahead), each step reading its word from
//      the lane that holds it and appending its 2-bit step to a record in
//      LDS (one word per 16 steps; on the diagonal layout a run of diagonal
//      steps is read from one word at once, with no branch per step);
//      meanwhile waves 1-3 copy both series to LDS when they fit;
//   3. all threads decode the record: each takes a run of consecutive steps,
//      a block scan of the row and column decrements gives its starting
//      cell, and it writes the runs its steps close: a monotone path meets
//      every row i in one run of columns [rlo_i, rhi_i] and every column j
//      in one run of rows [clo_j, chi_j];
//   4. threads over (row, dimension) form grad_x[i][p] = g * sum_{j in run}
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

// The walk of wave 0 (all positions and codes wave-uniform, in scalar
// registers): from (m-1, n-1) back to (0, 0), each step's 2-bit code appended
// to `rec` (16 to a word, written by lane 0).  `codes` is the pair's code
// record, in LDS or global memory (one instantiation each, so that LDS reads
// are LDS instructions).  Each lane holds one word of the current block of
// 64; on the diagonal layout (32-bit index arithmetic) the block before it
// is read ahead, since a step never moves to a later block and moves back at
// most one.  Returns the number of steps.
// Diagonal layout: the walk keeps (sigma, r) of the current cell (sigma =
// j - i + off, its slot sigma & 1, r = (i + j - slot) / 2): a diagonal step
// lowers r; a step to (i-1, j) or (i, j-1) moves sigma by +1 or -1 (flipping
// the slot) and lowers r when the slot was 0.  The walk ends at (0, 0), the
// only cell with r = 0 and slot 0.  The word of a cell is block r / 8, lane
// sigma / 2, and holds the codes of rounds 8 (r / 8) .. 8 (r / 8) + 7 of both
// slots, so a run of diagonal steps is read from one word: the slot's codes
// of rounds r mod 8 down to 0, the run ending at the first nonzero code (or
// at round 0, after which the walk is in the block before).  A step never
// moves to a later block and moves back at most one, so the block before the
// current one is read ahead.  The loop is bounded by the longest path.
__device__ __forceinline__ int walk_diag(const CodeMap& cm, const uint32_t* codes, int words, int m, int n,
                                         uint32_t* rec, int lane) {
    int sigma = (n - m) + cm.off;
    int r = (m + n - 2 - (sigma & 1)) >> 1;
    int blk = r >> 3;
    auto load = [&](int b) __attribute__((always_inline)) {
        const int w = b * cm.G + lane;
        return (b >= 0 && w < words) ? codes[w] : 0u;
    };
    uint32_t held = load(blk), ahead = load(blk - 1);
    const int maxL = m + n - 2;
    int L = 0;          // steps recorded
    uint32_t acc = 0;   // the record word of step L (code 0 = diagonal)
    // Branch-free steps: each iteration takes one non-diagonal step or a run of diagonal ones,
    // stores the record word it wrote into (every lane the same value) and starts a new word
    // when the steps cross into the next.
    while ((r > 0 || (sigma & 1)) && L < maxL) {
        const int slot = sigma & 1, rr = r & 7;
        const uint32_t word = (uint32_t)__builtin_amdgcn_readlane((int)held, sigma >> 1);
        // this slot's codes of rounds 0 .. rr, round t at bits 4t and 4t + 1
        const uint32_t z = (word >> (2 * slot)) & 0x33333333u & (0xffffffffu >> (28 - 4 * rr));
        const uint32_t c = z >> (4 * rr);
        const bool diag = c == 0u;
        // diagonal steps down to the first nonzero code below round rr (the highest set bit
        // of z; none: through round 0); from r = 0 only slot 1 remains, which is never diagonal
        const int run = diag ? max(min(rr - ((31 - (int)__clz(z)) >> 2), r), 1) : 1;
        const uint32_t code = c == 3u ? 2u : c;
        acc |= code << (2 * (L & 15));
        rec[L >> 4] = acc;
        const int Ln = min(L + run, maxL);   // (a valid path ends at exactly maxL steps or fewer)
        acc = ((Ln ^ L) >> 4) != 0 ? 0u : acc;
        L = Ln;
        r -= diag ? run : (slot == 0 ? 1 : 0);
        sigma += diag ? 0 : (code == 1u ? 1 : -1);
        if ((r >> 3) != blk) {
            blk = r >> 3;
            held = ahead;
            ahead = load(blk - 1);
        }
    }
    if ((L & 15) != 0) rec[L >> 4] = acc;
    return L;
}

// Row layout: each lane holds one word of the current block of 64, reloaded
// when the path leaves it.
__device__ __forceinline__ int walk_rows(const CodeMap& cm, const uint32_t* codes, int words, int m, int n,
                                         uint32_t* rec, int lane) {
    int i = m - 1, j = n - 1;
    int cur = -1;
    uint32_t held = 0;
    int L = 0;
    while (i > 0 || j > 0) {
        uint32_t acc = 0;
        int k = 0;
        for (; k < 16 && (i > 0 || j > 0); ++k) {
            int64_t b64;
            int ln, sh;
            cm.locate64(i, j, b64, ln, sh);
            const int base = (int)b64;
            if (base != cur) {
                const int w = base + lane;
                held = w < words ? codes[w] : 0u;
                cur = base;
            }
            const uint32_t word = (uint32_t)__builtin_amdgcn_readlane((int)held, ln);
            uint32_t code = (word >> sh) & 3u;
            code = code == 3u ? 2u : code;
            i -= code != 2u;
            j -= code != 1u;
            acc |= code << (2 * k);
        }
        if (lane == 0) rec[L >> 4] = acc;
        L += k;
    }
    return L;
}

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
    uint32_t* rec = reinterpret_cast<uint32_t*>(chi + n);          // [(m + n) / 16 + 1] step record
    int32_t* scan = reinterpret_cast<int32_t*>(rec + (m + n) / 16 + 1);   // [kBwdThreads + 1]
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
    __syncthreads();

    if (tid < kWave) {
        const int lane = tid;
        int L;
        // the walk of wave 0, all positions and codes wave-uniform (scalar registers); the
        // codes from LDS or global memory (separate instantiations keep LDS reads LDS reads)
        if (staged)
            L = cm.diag ? walk_diag(cm, scodes, (int)words, m, n, rec, lane)
                        : walk_rows(cm, scodes, (int)words, m, n, rec, lane);
        else
            L = cm.diag ? walk_diag(cm, gcodes, (int)words, m, n, rec, lane)
                        : walk_rows(cm, gcodes, (int)words, m, n, rec, lane);
        if (lane == 0) scan[kBwdThreads] = L;
    } else if (sstaged) {
        copy_to_lds(sser, xs, (int64_t)m * D, tid - kWave, kBwdThreads - kWave);
        copy_to_lds(sser + m * D, ys, (int64_t)n * D, tid - kWave, kBwdThreads - kWave);
    }
    __syncthreads();

    {   // decode the record into the runs: thread t takes steps [s0, s1)
        const int L = scan[kBwdThreads];
        const int per = (L + kBwdThreads - 1) / kBwdThreads;
        const int s0 = min(L, tid * per), s1 = min(L, s0 + per);
        auto step_code = [&](int st) __attribute__((always_inline)) { return (rec[st >> 4] >> ((st & 15) * 2)) & 3u; };
        int di = 0, dj = 0;
        for (int st = s0; st < s1; ++st) {
            const uint32_t c = step_code(st);
            di += c != 2u;
            dj += c != 1u;
        }
        // exclusive block scan of the packed decrements (each below 2^16)
        scan[tid] = (di << 16) | dj;
        __syncthreads();
        for (int o = 1; o < kBwdThreads; o <<= 1) {
            const int add = tid >= o ? scan[tid - o] : 0;
            __syncthreads();
            scan[tid] += add;
            __syncthreads();
        }
        const int incl = scan[tid];
        const int excl = incl - ((di << 16) | dj);
        int i = m - 1 - (excl >> 16), j = n - 1 - (excl & 0xffff);
        for (int st = s0; st < s1; ++st) {
            const uint32_t c = step_code(st);
            const int pi = c != 2u ? i - 1 : i, pj = c != 1u ? j - 1 : j;
            if (pi != i) { rlo[i] = j; rhi[pi] = pj; }
            if (pj != j) { clo[j] = i; chi[pj] = pi; }
            i = pi; j = pj;
        }
        if (tid == 0) { rhi[m - 1] = n - 1; chi[n - 1] = m - 1; rlo[0] = 0; clo[0] = 0; }
    }
    __syncthreads();

    const float g2 = 2.0f * a.grad_dist[pid];
    const float* xv_src = sstaged ? sser : xs;
    const float* yv_src = sstaged ? sser + m * D : ys;
    float* gx = a.grad_x + xoff;
    float* gy = a.grad_y + yoff;
    // element t = i D + p; (i, p) advanced by kBwdThreads elements per iteration without a division
    const int si = kBwdThreads / D, sp = kBwdThreads - si * D;
    for (int t = tid, i = tid / D, p = tid - (tid / D) * D; t < m * D; t += kBwdThreads) {
        const int j0 = rlo[i], j1 = rhi[i];
        const double xv = xv_src[t];
        double acc = 0.0;
        for (int j = j0; j <= j1; ++j) acc += xv - (double)yv_src[j * D + p];
        gx[t] = (float)((double)g2 * acc);
        i += si;
        p += sp;
        if (p >= D) { p -= D; ++i; }
    }
    for (int t = tid, j = tid / D, p = tid - (tid / D) * D; t < n * D; t += kBwdThreads) {
        const int i0 = clo[j], i1 = chi[j];
        const double yv = yv_src[t];
        double acc = 0.0;
        for (int i = i0; i <= i1; ++i) acc += yv - (double)xv_src[i * D + p];
        gy[t] = (float)((double)g2 * acc);
        j += si;
        p += sp;
        if (p >= D) { p -= D; ++j; }
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

// LDS ints of the runs (rlo, rhi, clo, chi), the step record and the scan
static int bwd_runs_ints(int maxm, int maxn) {
    return 2 * (maxm + maxn) + (maxm + maxn) / 16 + 1 + kBwdThreads + 1;
}

size_t bwd_lds_bytes(int maxm, int maxn, int64_t max_words, int maxd) {
    const int64_t cap = max_words < kBwdCodeLdsWords ? max_words : kBwdCodeLdsWords;
    return (size_t)bwd_runs_ints(maxm, maxn) * 4 + (size_t)cap * 4 + (size_t)bwd_series_cap(maxm, maxn, maxd) * 4;
}

hipError_t launch_dtw_bwd(const DtwBwdArgs& a, int maxm, int maxn, int64_t max_words, int maxd, int nitems,
                          int grid, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    DtwBwdArgs b = a;
    b.runs_ints = bwd_runs_ints(maxm, maxn);
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
