// Internal declarations shared by the host library and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tcdtw {

// Bits of the device status word (one per device; kernels OR conditions into
// it, tc_dtw_sync_status reads and clears it).
enum : uint32_t {
    kStatusNonFiniteRef = 1u,     // a reference value is not finite (index build)
    kStatusNonFiniteQuery = 2u,   // a query value is not finite (search preparation)
    kStatusWaitExpired = 4u       // a bounded wait between the waves of a pair ran out (distance NaN)
};
// The current device's status word (null if it cannot be located).
uint32_t* status_word();

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
    int32_t D;            // dimensions of both series
    int32_t rows;         // 1: row-systolic mapping (code layout follows the mapping)
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
    int32_t* counter;        // non-null: persistent waves take items 0..nitems-1 from it
    int32_t nitems;
    uint32_t* status;        // device status word (or null)
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
    int64_t series_cap;      // floats of LDS available for staging a pair's x and y (0: read them from HBM)
    int32_t* counter;        // non-null: persistent waves take items 0..nitems-1 from it
    int32_t nitems;
    int32_t urows;           // uniform: the pairs ran on the row mapping
};

// Size of the argmin-code record of one pair (u32 words).  Diagonal
// mapping: 4 bits per lane per round, 8 rounds per word, (W+1) lanes.
// Row mapping: 2 bits per lane per step, 16 steps per word, per 64-row block.
__host__ __device__ inline int64_t codes_words(int m, int n, int W, bool rows) {
    if (!rows) {
        const int R = (m + n) / 2;
        return (int64_t)((R + 7) / 8) * (W + 1);
    }
    const int nb = (m + kRowBlock - 1) / kRowBlock;
    const int band = n < 2 * W + kRowBlock ? n : 2 * W + kRowBlock;
    const int tmax = band + kRowBlock - 1;
    const int nwb = (tmax + 15) / 16;
    return (int64_t)nb * nwb * kWave;
}
__host__ __device__ inline int64_t codes_words(int m, int n, int W) {
    return codes_words(m, n, W, W > kDiagMaxW);
}
// LDS bytes of the forward kernels.
size_t diag_lds_bytes(int m, int n, int W, int D, int P);
size_t rows_lds_bytes(int n, int W, int D, bool f64);

hipError_t launch_dtw_fwd(const DtwFwdArgs& a, bool f64, bool save, bool rows, int nitems, int grid,
                          hipStream_t s);
size_t fwd_lds_bytes(const DtwFwdArgs& a, bool rows, bool f64);
// Row mapping with K (2..8) waves per pair, persistent workgroups over a.nitems items.
hipError_t launch_dtw_rows_pipe(const DtwFwdArgs& a, bool f64, bool save, int K, int nitems, int grid,
                                hipStream_t s);
size_t pipe_lds_bytes(int maxn, int D, int K, bool f64);
hipError_t launch_dtw_bwd(const DtwBwdArgs& a, int maxm, int maxn, int64_t max_words, int maxd, int nitems,
                          int grid, hipStream_t s);
size_t bwd_lds_bytes(int maxm, int maxn, int64_t max_words, int maxd);
hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t s);
// Diagonal pairs with the point costs formed ahead of the recurrence by three more waves per item
// (uniform pairs, float, W_eff <= 63): for batches of at most kCoopMaxItems items.
constexpr int kCoopMaxItems = 1024;
size_t diag_coop_lds_bytes(int m, int n, int W, int D, int P);
hipError_t launch_dtw_diag_coop(const DtwFwdArgs& a, bool save, int nitems, hipStream_t s);

// ------------------------------------------------------------- index build
struct IndexBuildArgs {
    const float* src;         // candidate data as given
    const int64_t* src_off;   // ragged: device copy of the given offsets
    const int64_t* dst_off;   // ragged: offsets inside `series`
    const int32_t* lens;      // ragged: lengths
    const int64_t* gamma_off; // ragged: offsets inside `gamma`
    const int32_t* dims;      // per-series D (banks of several dims), or null: D for every series
    int32_t count, ulen, D, maxlen, ntiles;
    int64_t total_len;
    float* series;
    float* tiles;
    float* gamma;
    uint32_t* range_keys;     // 2 words, become float min / max
    uint32_t* status;         // device status word (or null)
};
hipError_t launch_index_build(const IndexBuildArgs& a, hipStream_t s);

// ------------------------------------------------------------------- 1-NN
// Best-so-far keys of the queries sit 128 bytes apart: every query's key
// is its own cache line, so the atomic updates and coherent reads of
// different queries do not queue on shared lines.
constexpr int kKeyStride = 16;   // u64 words
constexpr int kQT = 8;           // queries per LB_MV tile
constexpr int kMaxSeeds = 32;
constexpr int kMaxK = 32;           // largest k of a k-nearest-neighbour search
constexpr int kNumCounters = 24;   // 1 + two stages x one persistent launch per bank (8 at most)
constexpr int kNumStats = 16;
enum {
    kStPrunedMv = 0, kStPrunedPc, kStPrunedTi, kStDtwStarted, kStDtwAbandoned, kStRescored,
    kStCells, kStEvalPc, kStEvalTi
};

// Device pointers of one search (uniform lengths).
struct KnnPlanDev {
    const float* Q;       // queries [nq][m][D]
    const float* C;       // index series [nc][n][D]
    const float* tiles;   // index tiles
    int32_t nq, nc, m, n, D, W, ntiles, R, cap;
    float* env;
    float* lb;
    int32_t* seeds;
    float* seed_dist;
    uint32_t* list;
    float* list_dist;
    int32_t* cnt;
    uint32_t* glist;
    int32_t* gcnt;
    int32_t* prefix;
    int32_t* item_query;
    int32_t* counters;
    unsigned long long* key;
    unsigned long long* stats;
    int32_t* clear[3];    // optional extra per-query counters zeroed with the others
    float* part;          // LB_MV partial sums [nseg][nq][nc] when nseg > 1, else null
    int32_t nseg;
    unsigned long long* topk;   // [nq][k] keys of the k best candidates so far (k > 1), else null
    int32_t k;
    uint32_t* status;     // device status word (or null)
    const int32_t* q_cb;  // banks of several dims: [nq] candidate range of each query, else null
    const int32_t* q_ce;
};
// Element segments of the LB_MV launch (more when few query tiles would leave HBM idle).
int lb_mv_segments(int ntiles, int nq, int E);

// Persistent DTW over per-query candidate lists.
struct KnnDtwArgs {
    const float* Q;
    const float* C;
    int32_t nq, m, n, D, W, P;
    int32_t gs;                // lanes per pair group (knn_lane_stride)
    unsigned long long* topk;  // [nq][k] keys of the k best so far (k > 1); key[] then holds their largest
    int32_t k;
    int32_t indep;             // 1: independent DTW (sum of per-dimension DTWs)
    const uint32_t* list;      // [nq][cap] candidate indices (negative: none)
    float* list_dist;          // [nq][cap] float32 DTW, +inf when abandoned
    const int32_t* cnt;        // [nq] list lengths (unless cnt_uniform > 0)
    int32_t cnt_uniform;
    int32_t cap;
    const int32_t* prefix;     // [nq+1] work items per query, prefix sums
    const int32_t* item_query; // [items] query of each work item
    int32_t* counter;          // work counter
    unsigned long long* key;   // [nq] packed best-so-far
    unsigned long long* stats;
    float gamma;               // float DP relative error bound
    int32_t abandon;
    int64_t band_cells;        // cells of one pair's band (statistics)
};

struct KnnFinalArgs {
    const float* Q;
    const float* C;
    int32_t nq, m, n, D, W, R, cap;
    const int32_t* seeds;
    const float* seed_dist;
    const uint32_t* list;
    const float* list_dist;
    const int32_t* cnt;
    const int32_t* gcnt;       // gated pairs (advanced bounds)
    const int32_t* cnt_mv;     // DTW-list length right after the LB_MV compaction (null: cnt)
    const int32_t* pruned_pc;  // [nq] or null
    const int32_t* pruned_ti;  // [nq] or null
    int32_t nc;
    double ratio;              // finalists: float32 DTW <= (bound of the k-th smallest) * ratio
    const unsigned long long* key;   // [nq] threshold keys after the DTW stage (k-th best key)
    int32_t k;                 // neighbours per query; nn_idx / nn_dist are [nq][k]
    int32_t indep;             // 1: independent DTW
    int32_t* nn_idx;
    float* nn_dist;
    unsigned long long* stats;
};

// 1-NN over a bank of uneven lengths (knn_ragged.hip).
struct RaggedKnnArgs {
    const float* Q;
    const int64_t* q_off;      // [nq] float offsets of the queries
    const int32_t* q_len;      // [nq]
    const int32_t* q_dim;      // [nq] D of each query (banks of several D), or null: D for all
    const int32_t* q_cb;       // [nq] first candidate of the query's bank (with q_dim)
    const int32_t* q_ce;       // [nq] one past its last candidate
    int32_t bank_max;          // the largest bank (with q_dim; of this launch's bank with a query range)
    const int32_t* q_out;      // [nq] the caller's index of each query (queries grouped by bank), or null
    int32_t q0, q1;            // the queries of this launch: DTW items of queries q0 .. q1-1, LB_MV rows
                               // q0 + blockIdx.y (q1 = 0: every query)
    const float* C;            // index series
    const int64_t* c_off;      // [nc] float offsets inside the index series
    const int32_t* c_len;      // [nc]
    int32_t nq, nc, D, maxm, maxn;  // D: the largest D (with banks)
    int32_t window, num, den;  // window specification (per pair W_eff)
    float* tab;                // query sparse tables
    const int64_t* t_off;      // [nq] float offsets of each query's tables
    float* lb;                 // [nq][nc]
    const uint32_t* list;      // DTW list (seeds or survivors) [nq][cap]
    float* list_dist;
    int32_t cap;
    const int32_t* prefix;
    const int32_t* item_query;
    int32_t* counter;
    unsigned long long* key;
    unsigned long long* stats;
    int32_t abandon;
    // finalize
    const int32_t* seeds;
    const float* seed_dist;
    int32_t R;
    const int32_t* list_cnt;
    int32_t* nn_idx;
    float* nn_dist;
    uint32_t* status;          // device status word (or null)
};
hipError_t launch_rq_tables(const RaggedKnnArgs& a, hipStream_t s);
// p[0 .. n) = v
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_rlb_mv(const RaggedKnnArgs& a, hipStream_t s);
hipError_t launch_rknn_dtw(const RaggedKnnArgs& a, int nblocks, hipStream_t s);
hipError_t launch_rknn_finalize(const RaggedKnnArgs& a, hipStream_t s);
size_t rknn_dtw_lds_bytes(int maxn, int D);
size_t rknn_final_lds_bytes(int maxn, int D);

// Query envelope; with init also the
// per-query search state (best-so-far keys, list counts, counters, stats).
hipError_t launch_knn_prep(const KnnPlanDev& p, hipStream_t s, bool init = true);
hipError_t launch_lb_mv(const KnnPlanDev& p, float* lb, hipStream_t s);
hipError_t launch_topr(const KnnPlanDev& p, hipStream_t s);
hipError_t launch_compact(const KnnPlanDev& p, double keep, double gate_e2, int use_gate, hipStream_t s);
hipError_t launch_chunk_scan(const KnnDtwArgs& a, hipStream_t s);
hipError_t launch_dtw_lists(const KnnDtwArgs& a, int nblocks, hipStream_t s);
int64_t band_cells(int m, int n, int W);
hipError_t launch_knn_finalize(const KnnFinalArgs& a, hipStream_t s);
size_t knn_dtw_lds_bytes(int m, int n, int W, int D, int P);
int knn_ring_max_passes(int nch);
int knn_dtw_max_pairs(int W, int D, bool indep);
// Ring size of the diagonal 1-NN kernel: the live window W + 5 plus one
// refill of RS / 4 positions must fit.
inline int ring_size(int W) { return W <= 27 ? 64 : 128; }
// Lanes per pair in the 1-NN diagonal kernel: the W + 1 band offsets of a
// pair, padded to a power of two when that keeps as many pairs per wave.
// Each 16-lane quarter of the wave then reads 16 consecutive positions of
// one series, which the LDS serves without bank conflicts; two pairs in
// one quarter read positions 16 apart, which share banks.
inline int knn_lane_stride(int W, bool pow2 = false) {
    const int G = W + 1;
    int p2 = 1;
    while (p2 < G) p2 <<= 1;
    return (pow2 || 64 / p2 >= 64 / G) ? p2 : G;
}
size_t knn_final_lds_bytes(int m, int n, int W, int D);

// --------------------------------------------------------- advanced bounds
struct PcArgs {
    const float* Q;            // queries [nq][m][D]
    const float* C;            // candidates [nc][n][D]
    int32_t nq, nc, m, n, D, W;
    int32_t Lv, K, w, ngroups, max_pts;
    float floor_len;           // <= 0: 1e-5 * (range[1] - range[0])
    const float* range;        // index value range (min, max)
    float* boxes;              // [nq][ngroups][K][D][2] (cand: [nc][ngroups][K][D][2])
    int32_t* nbox;             // [nq][ngroups] (cand: [nc][ngroups])
    int32_t cand;              // 1: the boxes are the candidates' (over query-position groups) and
                               // the query's points are evaluated against them
    // list evaluation
    const uint32_t* in_list;   // [nq][cap] or null (every candidate)
    const int32_t* in_cnt;
    int32_t in_uniform;        // > 0: every query lists this many entries
    int32_t cap;
    float* out_lb;             // [nq][cap]
    const int32_t* prefix;
    const int32_t* item_query;
    int32_t* counter;
    const unsigned long long* key;   // null: dense mode (no gate, no early stop)
    const float* lb_mv;        // [nq][nc] (search mode)
    double e2, keep;
    unsigned long long* evaluated;   // null, or a count of the pairs whose bound was evaluated
};

struct TiArgs {
    const float* Q;
    const float* C;
    const float* qstep;        // [nq][m] query steps
    const float* gamma;        // [nc][n] candidate steps (index)
    int32_t nq, nc, m, n, D, W, P, top;
    const uint32_t* in_list;
    int32_t cap;
    float* out_lb;
    const float* lb_in;        // [nq][cap] bound so far of each listed pair (search mode)
    const int32_t* prefix;
    const int32_t* item_query;
    int32_t* counter;
    const unsigned long long* key;
    double e2;
    unsigned long long* evaluated;   // null, or a count of the pairs whose bound was evaluated
};

struct RouteArgs {
    int32_t nq, nc, cap;
    const uint32_t* in_list;
    const int32_t* in_cnt;
    const float* lb_prev;      // [nq][cap] or null: take LB_MV from lb_mv
    const float* lb_mv;        // [nq][nc]
    const float* lb_new;       // [nq][cap], < 0 when not evaluated
    const unsigned long long* key;
    double keep, next_e2;
    uint32_t* dtw_list;
    int32_t* dtw_cnt;
    uint32_t* next_list;       // null: no further bound
    float* next_lb;
    int32_t* next_cnt;
    int32_t* pruned;           // [nq]
};

hipError_t launch_query_steps(const float* Q, int nq, int m, int D, float* delta, hipStream_t s);
size_t pc_boxes_lds_bytes(int max_pts, int K, int D);
hipError_t launch_pc_boxes(const PcArgs& a, hipStream_t s);
hipError_t launch_lb_pc(const PcArgs& a, int nblocks, hipStream_t s);
// query-side boxes only; items are chunks of 64 list entries of one query
hipError_t launch_lb_pc_lanes(const PcArgs& a, int nblocks, hipStream_t s);
hipError_t launch_lb_ti(const TiArgs& a, int nblocks, hipStream_t s);
// Exact rows of LB_TIP: row 0 and, with P > 0, every multiple of P.
__host__ __device__ inline int ti_exact_rows(int m, int P) { return P > 0 ? (m - 1) / P + 1 : 1; }
// LDS of the LB_TI launch for a pair of lengths (m, n) and band half-width W
size_t ti_lds_bytes(int m, int n, int D, int P, int W);
size_t ti_cols_lds_bytes(int m);
hipError_t launch_lb_ti_cols(const TiArgs& a, int nblocks, hipStream_t s);
hipError_t launch_route(const RouteArgs& a, int max_in, hipStream_t s);
hipError_t launch_list_items(const int32_t* cnt, int cnt_uniform, int nq, int per, int32_t* prefix,
                             int32_t* item_query, int32_t* counter, hipStream_t s);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int n, hipStream_t s);

__host__ __device__ inline int nchunks(int D) { return (D + 3) / 4; }
// Supported chunk counts (template instantiations); D is padded up to one of them.
__host__ __device__ inline int nch_pad(int D) {
    int c = nchunks(D);
    if (c <= 4) return c;
    if (c <= 6) return 6;
    if (c <= 8) return 8;
    if (c <= 12) return 12;
    return 16;
}

}  // namespace tcdtw
