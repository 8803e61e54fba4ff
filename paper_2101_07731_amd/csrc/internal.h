// Internal declarations shared by the host library and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tcdtw {

// Largest band half-width handled by the diagonal-pair mapping: W_eff + 1
// lanes per pair must fit one wave.
constexpr int kDiagMaxW = 63;
constexpr int kWave = 64;
constexpr int kRowBlock = 64;  // rows per block of the row-systolic mapping

// One DTW pair of a ragged batch.
struct PairDesc {
    int64_t xoff, yoff;   // float offsets of the two series
    int64_t saved_off;    // u32-word offset of the pair's argmin codes
    int32_t m, n, W;      // lengths and W_eff
    int32_t out;          // output slot
};

// Arguments of the forward DTW kernels.
struct DtwFwdArgs {
    const float* x;
    const float* y;
    const PairDesc* desc;    // ragged: one descriptor per work item (then P = 1)
    int32_t uniform;         // 1: every pair has lengths (m, n), window W, pair b at b*m*D / b*n*D
    int32_t m, n, W;
    int32_t D;
    int32_t npairs;
    int32_t P;               // pairs per wave (uniform diagonal mapping)
    int32_t wodd;            // diagonal mapping: W_eff of every item is odd
    float* dist;
    double* dist64;          // optional
    uint32_t* codes;         // optional argmin codes
    int64_t codes_stride;    // uniform: u32 words per pair
};

// Arguments of the backward kernel.
struct DtwBwdArgs {
    const float* x;
    const float* y;
    const PairDesc* desc;
    int32_t uniform;
    int32_t m, n, W;
    int32_t D;
    int32_t npairs;
    const uint32_t* codes;
    int64_t codes_stride;
    const float* grad_dist;
    float* grad_x;
    float* grad_y;
    int32_t runs_ints;       // LDS ints reserved for the row/column runs (>= 2*(m+n) of every pair)
    int64_t stage_cap;       // u32 words of LDS available for staging a pair's codes
};

// Size of the argmin-code record of one pair (u32 words).  Diagonal
// mapping: 4 bits per lane per round, 8 rounds per word, (W+1) lanes.
// Row mapping: 2 bits per lane per step, 16 steps per word, per 64-row block.
__host__ __device__ inline int64_t codes_words(int m, int n, int W) {
    if (W <= kDiagMaxW) {
        const int R = (m + n) / 2;
        return (int64_t)((R + 7) / 8) * (W + 1);
    }
    const int nb = (m + kRowBlock - 1) / kRowBlock;
    const int band = n < 2 * W + kRowBlock ? n : 2 * W + kRowBlock;
    const int tmax = band + kRowBlock - 1;
    const int nwb = (tmax + 15) / 16;
    return (int64_t)nb * nwb * kWave;
}
// LDS bytes of the forward kernels.
size_t diag_lds_bytes(int m, int n, int W, int D, int P);
size_t rows_lds_bytes(int n, int W, int D, bool f64);

hipError_t launch_dtw_fwd(const DtwFwdArgs& a, bool f64, bool save, int maxW, int nitems,
                          hipStream_t s);
hipError_t launch_dtw_bwd(const DtwBwdArgs& a, int maxm, int maxn, int maxW, int nitems,
                          hipStream_t s);

inline int nchunks(int D) { return (D + 3) / 4; }
// Supported chunk counts (template instantiations); D is padded up to one of them.
inline int nch_pad(int D) {
    int c = nchunks(D);
    if (c <= 4) return c;
    if (c <= 6) return 6;
    if (c <= 8) return 8;
    if (c <= 12) return 12;
    return 16;
}

}  // namespace tcdtw
