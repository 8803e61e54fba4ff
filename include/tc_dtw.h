/*
 * tc_dtw.h -- C ABI of an MI355X (gfx950) library for multivariate (dependent)
 * DTW nearest-neighbour search with lower-bound filtering, after TC-DTW
 * (Shen & Chi, arXiv 2101.07731).
 *
 * The calls follow the paper's problem statement (Sec. 3, Definition 1):
 * given a query set Q and a candidate set C of D-dimensional series, find
 * for every query the candidate with the smallest windowed DTW distance,
 * using lower bounds LB <= DTW to skip DTW computations.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Plain C, no C++ or framework types.  Every pointer is documented as
 *    DEVICE (memory of the current HIP device) or HOST.
 *  - Point cost: squared Euclidean distance of two D-vectors (dependent DTW,
 *    Sec. 2).  Every distance and bound is reported in that squared space;
 *    no square root is ever taken of a DTW value.
 *  - Window: Sakoe-Chiba band |i - j| <= W_eff (Sec. 2, "Window DTW") with
 *    W = floor(max(m,n) * frac_num / frac_den) when frac_den > 0, else
 *    W = window, and W_eff = max(W, |m - n|) so the end cell stays
 *    reachable for unequal lengths m, n.
 *  - All device memory is owned by the caller: inputs, outputs, the index
 *    buffer, the saved-state buffer and the workspace.  The library never
 *    allocates or frees device memory (its only device memory of its own
 *    is the static scratch array of tc_dtw_banded_noalloc); sizes come from
 *    the *_bytes() queries.  Workspace contents need no initialisation and are
 *    meaningless after a call.
 *  - Every call that takes a stream enqueues its work on that stream and
 *    returns without waiting (unless a HOST output such as stats is
 *    requested, which is documented per call).  Calls that share a
 *    workspace must not overlap.
 *  - Arguments are validated on the host before any HIP call; on error
 *    nothing is enqueued, outputs are untouched, and tc_dtw_last_error()
 *    returns a message (thread-local).
 *  - Input values must be finite.  Limits: 1 <= D <= 64, 1 <= length.
 */
#ifndef TC_DTW_H
#define TC_DTW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TC_DTW_ABI_VERSION 7

typedef struct ihipStream_t* tc_dtw_stream; /* same type as hipStream_t; NULL = default stream */

typedef enum {
    TC_DTW_OK = 0,
    TC_DTW_ERR_INVALID = 1,     /* bad argument (null pointer, count, length, window, mismatch) */
    TC_DTW_ERR_WORKSPACE = 2,   /* a caller buffer is smaller than its *_bytes() query */
    TC_DTW_ERR_UNSUPPORTED = 3, /* valid but not supported (D > 64, k != 1, key overflow) */
    TC_DTW_ERR_DEVICE = 4       /* no usable gfx950 device, or a HIP call failed */
} tc_dtw_status;

/* A set of float32 series.
 *   data    DEVICE  series s occupies data[offset[s] .. offset[s] + len[s]*D_s),
 *                   row-major [t][d] (a torch [B, T, D] tensor when uniform).
 *   offset  HOST    per-series start in floats, or NULL: the series packed
 *                   back to back in order (s * uniform_len * dim when uniform).
 *   len     HOST    per-series length, or NULL: every series has uniform_len.
 *   count   number of series (>= 1).
 *   dim     D of every series (1..64) when dims == NULL, else ignored.
 *   uniform_len  length of every series when len == NULL, else ignored.
 *   dims    HOST    per-series D_s (1..64), or NULL: every series has dim.
 *                   Accepted by the pair calls (banded, backward, pairs
 *                   plans); the search calls need one D per set. */
typedef struct {
    const float* data;
    const int64_t* offset;
    const int32_t* len;
    int32_t count;
    int32_t dim;
    int32_t uniform_len;
    const int32_t* dims;
} tc_dtw_batch;

/* Window specification (see conventions above). */
typedef struct {
    int32_t window;
    int32_t frac_num;
    int32_t frac_den;
} tc_dtw_window;

/* ------------------------------------------------------------------ misc */

int tc_dtw_abi_version(void);
const char* tc_dtw_last_error(void);
const char* tc_dtw_status_string(tc_dtw_status s);

/* tc_dtw_sync_status: waits for `stream`, then reads and clears the
 * device's status word, into which kernels record conditions they detect
 * but cannot return (the calls are asynchronous): a reference value that
 * is not finite (tc_dtw_build_index), a query value that is not finite
 * (the searches and the bound matrices), and a bounded wait between the
 * waves sharing a long pair that ran out (tc_dtw_banded / _run: that
 * pair's distance is NaN).  The word is one per device and accumulates
 * over all calls since it was last read.  Returns TC_DTW_OK if it was
 * clear, else TC_DTW_ERR_DEVICE with the conditions in tc_dtw_last_error();
 * TC_DTW_ERR_DEVICE also when there is no usable device.  For tests, the
 * environment variable TC_DTW_FAKE_NO_DEVICE (set, not "0") makes every
 * call behave as on a machine without a usable device. */
tc_dtw_status tc_dtw_sync_status(tc_dtw_stream stream);

/* --------------------------------------------------------- banded DTW ---
 * tc_dtw_banded: DTW of x->count pairs (x_b, y_b), b = 0..count-1
 * (Sec. 2, Eq. 1 within the Sakoe-Chiba band).
 *   x, y    sets of equal count and dim.
 *   win     window per pair (W_eff from the pair's lengths).
 *   flags   TC_DTW_F64: the recurrence is evaluated in float64 (point
 *           costs from the float32 inputs, each product and sum rounded
 *           once in increasing-dimension order), which reproduces an FP64
 *           reference bit for bit.  Default: float32 arithmetic.
 *   dist    DEVICE float[count], squared-cost DTW of each pair.
 *   saved   DEVICE buffer of tc_dtw_saved_bytes() bytes, or NULL.  When
 *           given, the forward also records, per band cell, which
 *           predecessor attained the minimum (ties: diagonal, then
 *           (i-1,j), then (i,j-1)); tc_dtw_backward reads it.
 *   ws      DEVICE workspace of tc_dtw_banded_workspace_bytes() bytes.
 * Errors: INVALID (null data/dist, count < 1, length < 1, dims differ,
 * negative window, frac_den < 0), UNSUPPORTED (dim > 64), WORKSPACE,
 * DEVICE. */
#define TC_DTW_F64 1u

size_t tc_dtw_banded_workspace_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y,
                                     tc_dtw_window win, uint32_t flags);
size_t tc_dtw_saved_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win);
tc_dtw_status tc_dtw_banded(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                            uint32_t flags, float* dist, void* saved,
                            void* ws, size_t ws_bytes, tc_dtw_stream stream);

/* ----------------------------------------------------------- backward ---
 * tc_dtw_backward: gradient of dist_b = DTW(x_b, y_b) with respect to both
 * series along the optimal warping path recorded by tc_dtw_banded (the
 * paper cites DTW as a loss, Sec. 1 and Sec. 9; this is the adjoint of
 * Eq. 1 on a fixed path):
 *   grad_x[b][i] = g_b * sum_{j: (i,j) on path} 2 (x_b[i] - y_b[j])
 *   grad_y[b][j] = g_b * sum_{i: (i,j) on path} 2 (y_b[j] - x_b[i])
 *   saved      DEVICE, written by tc_dtw_banded with the same x, y, win.
 *   grad_dist  DEVICE float[count] (g_b).
 *   grad_x, grad_y  DEVICE, same layout and offsets as x->data, y->data;
 *              every element of every series is written.
 * Errors: as tc_dtw_banded, plus INVALID for a NULL saved pointer. */
size_t tc_dtw_backward_workspace_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y,
                                       tc_dtw_window win);
tc_dtw_status tc_dtw_backward(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                              const void* saved, const float* grad_dist,
                              float* grad_x, float* grad_y,
                              void* ws, size_t ws_bytes, tc_dtw_stream stream);

/* ------------------------------------------- banded DTW, no allocation ---
 * tc_dtw_banded_noalloc: tc_dtw_banded for callers that cannot allocate
 * device memory or pass a workspace (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * results as tc_dtw_banded without ws / ws_bytes: the scratch that
 * tc_dtw_banded plans into for pairs of uneven shapes (32 class counters
 * and a 48-byte descriptor per pair, about tc_dtw_banded_workspace_bytes())
 * lives in a static device array of tc_dtw_noalloc_scratch_bytes() bytes
 * (8 MiB, about 170 000 pairs), one per GPU, held until the process ends.
 * The call allocates no device memory and creates no streams or events: the
 * plan's classes run one after another on `stream` (tc_dtw_banded runs them
 * concurrently on library streams).  Pair descriptors are copied from host
 * memory with hipMemcpyAsync.
 * Concurrency: every call on one GPU uses that GPU's one array; calls that
 * overlap on a GPU (from other streams or threads) race and must be
 * serialised by the caller.
 * Errors: as tc_dtw_banded, and UNSUPPORTED (checked on the host, before
 * any HIP call) when the batch's plan exceeds the static scratch. */
size_t tc_dtw_noalloc_scratch_bytes(void);
tc_dtw_status tc_dtw_banded_noalloc(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                                    uint32_t flags, float* dist, void* saved, tc_dtw_stream stream);

/* ------------------------------------------------- reusable pair plans ---
 * A plan fixes the shapes of a batch of pairs once: lengths, dims, W_eff,
 * which wave mapping evaluates each pair (diagonal pairs for narrow bands,
 * row-systolic blocks otherwise), and the order of the work.  The pairs are
 * grouped into classes of one mapping and one dimension class, each run by
 * one persistent launch whose waves take pairs, longest first, from a
 * device counter.  tc_dtw_banded_run and tc_dtw_backward_run then only
 * enqueue kernels (no host-to-device copies, no allocation), so a caller
 * can capture them in a HIP graph and replay them with new data laid out
 * like the planned batch.  This is the batched form of Sec. 2, Eq. 1 over
 * many pairs of uneven lengths and dims; results equal tc_dtw_banded's.
 *
 * tc_dtw_tuning (HOST, may be NULL for the defaults):
 *   diag_max_w    pairs with W_eff <= diag_max_w (and whose two series fit
 *                 32 KB of LDS) use the diagonal mapping, the others the
 *                 row mapping; -1..63, default 63.
 *   waves_per_cu  resident waves per CU of the persistent launches, 1..32;
 *                 0 means 16.  Fewer when a class's LDS does not allow them.
 *   waves_per_pair  largest number of waves that share one pair on the row
 *                 mapping, 1, 2, 4 or 8 (0 means 8).  A pair gets K > 1
 *                 waves only when one wave alone would take longer than the
 *                 whole batch spread over 256 wave slots (K = that ratio
 *                 rounded up to 2, 4 or 8), capped here and by LDS; the K
 *                 waves pipeline its 64-row blocks through a shared row
 *                 buffer.
 * tc_dtw_pairs_plan_bytes: size of the DEVICE plan buffer (0 on invalid
 *   arguments).  x->data and y->data are not read by the plan calls.
 * tc_dtw_pairs_plan_build: fills `plan` (HOST) and copies the pair
 *   descriptors into `buf` (DEVICE, caller-owned, must outlive every run)
 *   on `stream`, then waits for that copy.  Errors: as tc_dtw_banded, and
 *   UNSUPPORTED when the batch needs more than TC_DTW_PLAN_MAX_CLASSES
 *   classes.
 * tc_dtw_banded_run: as tc_dtw_banded on x, y (DEVICE base pointers; the
 *   planned offsets are relative to them); `saved` (DEVICE, or NULL) must
 *   hold plan->saved_bytes.  A run resets the plan's counters itself; runs
 *   of one plan must not overlap (they share the counters).  The classes
 *   run concurrently: the run forks from `stream` to TC_DTW_RUN_STREAMS
 *   streams the library creates once per device (default priority) and
 *   joins back with events, so the work is ordered after everything
 *   already on `stream` and everything enqueued later waits for it (also
 *   when `stream` is being captured into a graph).
 * tc_dtw_backward_run: as tc_dtw_backward, with `saved` written by a
 *   tc_dtw_banded_run of the same plan. */
typedef struct {
    int32_t diag_max_w;
    int32_t waves_per_cu;
    int32_t waves_per_pair;
} tc_dtw_tuning;

#define TC_DTW_PLAN_MAX_CLASSES 32
#define TC_DTW_RUN_STREAMS 4

typedef struct {
    int32_t rows;        /* 1: row mapping, 0: diagonal mapping */
    int32_t wodd;        /* diagonal mapping: W_eff of every pair of the class is odd */
    int32_t dim;         /* largest D of the class */
    int32_t nitems;      /* pairs in the class */
    int32_t maxm, maxn, maxw;
    int32_t waves_per_pair; /* row mapping: waves sharing each pair (1: one wave per pair) */
    int64_t max_words;   /* largest argmin-code record of the class (u32 words) */
    int64_t desc_off;    /* byte offset of the class's descriptors in the plan buffer */
    double work;         /* band cells x (2 D + 2) summed over the class: balances the streams */
    int32_t stream;      /* which of the library's streams runs the class */
    int32_t reserved;
} tc_dtw_plan_class;

typedef struct {
    void* buf;           /* DEVICE plan buffer */
    size_t bytes;
    int32_t npairs;
    int32_t nclasses;
    int32_t waves_per_cu;
    int32_t reserved;
    int64_t saved_bytes; /* bytes of the `saved` buffer of a recording forward */
    tc_dtw_plan_class cls[TC_DTW_PLAN_MAX_CLASSES];
} tc_dtw_pairs_plan;

size_t tc_dtw_pairs_plan_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                               const tc_dtw_tuning* tune);
tc_dtw_status tc_dtw_pairs_plan_build(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                                      const tc_dtw_tuning* tune, void* buf, size_t bytes,
                                      tc_dtw_pairs_plan* plan, tc_dtw_stream stream);
tc_dtw_status tc_dtw_banded_run(const tc_dtw_pairs_plan* plan, const float* x, const float* y,
                                uint32_t flags, float* dist, void* saved, tc_dtw_stream stream);
tc_dtw_status tc_dtw_backward_run(const tc_dtw_pairs_plan* plan, const float* x, const float* y,
                                  const void* saved, const float* grad_dist, float* grad_x,
                                  float* grad_y, tc_dtw_stream stream);

/* -------------------------------------------------------------- index ---
 * tc_dtw_build_index: prepares a candidate (reference) set for repeated
 * searches: a copy of the series, an element-major copy in tiles of 64
 * references (uniform lengths only; float[tile][e/4][64][e%4], elements
 * padded with zeros to a multiple of 4) for the envelope bound, the candidate
 * neighbour distances d(c_{j-1}, c_j) of the basic triangle bound (Sec. 4.1,
 * Eqs. 9-10, computed ahead of time and reused by every query), and the
 * value range (min, max over all values) that sets LB_PC's smallest cell
 * (Sec. 5).
 *   refs   the candidate set; its device data may be freed once the call
 *          has completed on `stream`.
 *   buf    DEVICE buffer of tc_dtw_index_bytes(refs) bytes, owned by the
 *          caller and read by every later call that takes the index; it
 *          must stay alive and unmodified while the index is used.
 *   out    HOST: receives the index description (plain data; copy freely).
 * Banks of several dimensions: with refs->dims given, the references may
 * have different D, each dimension forming one contiguous run of the set
 * (a bank; at most TC_DTW_MAX_BANKS of them).  A search then compares each
 * query only with the bank of its own D (DTW between series of different
 * D is undefined); the bank table is in `out`.
 * The index is immutable after the build, so searches on different streams
 * may share it.  Errors: INVALID, UNSUPPORTED (a dimension in two runs,
 * more than TC_DTW_MAX_BANKS banks), WORKSPACE (buf too small), DEVICE. */
#define TC_DTW_MAX_BANKS 8

typedef struct {
    void* buf;
    size_t bytes;
    int32_t count;        /* number of candidate series */
    int32_t dim;          /* D of every candidate; with banks, the largest D */
    int32_t uniform_len;  /* > 0 when every candidate has this length, else 0 */
    int32_t max_len;
    int32_t ntiles;       /* 64-candidate tiles of the element-major copy (uniform only) */
    int32_t nbanks;       /* 0: one D for all candidates; else the bank table below */
    int64_t off_series;   /* byte offsets of the sections inside buf */
    int64_t off_tiles;
    int64_t off_gamma;
    int64_t off_meta;     /* int64 offsets[count], then int32 lengths[count] */
    int64_t off_range;    /* float[2]: smallest and largest value */
    int64_t total_len;    /* sum of the candidate lengths */
    int64_t off_dims;     /* banks: int32 dims[count] */
    int64_t reserved[2];
    int32_t bank_dim[TC_DTW_MAX_BANKS];    /* D of bank b */
    int32_t bank_first[TC_DTW_MAX_BANKS];  /* its first candidate */
    int32_t bank_count[TC_DTW_MAX_BANKS];  /* its number of candidates */
} tc_dtw_index;

size_t tc_dtw_index_bytes(const tc_dtw_batch* refs);
tc_dtw_status tc_dtw_build_index(const tc_dtw_batch* refs, void* buf, size_t bytes,
                                 tc_dtw_index* out, tc_dtw_stream stream);

/* ---------------------------------------------------- search parameters ---
 * Lower-bound cascade of the 1-NN search (Sec. 6, selective deployment):
 * LB_MV (Sec. 3) for every pair; LB_PC (Sec. 5) and then LB_TI (Sec. 4,
 * LB_TIP_TOP by default) only for pairs whose LB_MV exceeds e^2 times the
 * best-so-far (the squared-cost form of e < LB_MV / d_best; the paper's e
 * applies to distances, Sec. 6); DTW with early abandoning (Sec. 7.1) for
 * the survivors.  Defaults are the paper's settings (Sec. 7.1): P = 5 with
 * TOP, K = w = 6, Lv = 2, e in its grids. */
#define TC_DTW_LB_MV 1u
#define TC_DTW_LB_PC 2u
#define TC_DTW_LB_TI 4u

typedef struct {
    tc_dtw_window window;
    uint32_t bounds;        /* OR of TC_DTW_LB_*; 0 = plain exhaustive DTW (no bounds, no abandoning) */
    int32_t early_abandon;  /* 1: abandon a DTW once it provably exceeds the best so far */
    int32_t ti_period;      /* P of LB_TIP; <= 0: only row 0 is exact (basic LB_TI) */
    int32_t ti_top;         /* 1: exact distance at the top cell of every row's window */
    int32_t pc_levels;      /* quantisation levels per dimension, Lv */
    int32_t pc_clusters;    /* boxes per expanded window, K */
    int32_t pc_group;       /* window expansion factor, w */
    float pc_min_cell;      /* smallest cell length; <= 0: 1e-5 * (max - min) of the index */
    float trigger_ti;       /* triggering threshold e of LB_TI */
    float trigger_pc;       /* triggering threshold e of LB_PC */
    float prune_margin;     /* extra relative margin of every prune test (>= 0) */
    int32_t seed_r;         /* smallest-LB_MV candidates per query whose DTW seeds the best-so-far; 0: 4 */
    int32_t k;              /* neighbours per query, 1..32 (k > 1: uniform lengths only) */
    int32_t independent;    /* 0: dependent DTW (one warping path for all dimensions, Sec. 2 DTW_D,
                               the paper's subject); 1: independent DTW (Sec. 2 DTW_I, the sum of
                               the dimensions' univariate DTWs), with LB_MV or no bounds, uniform
                               lengths, W_eff <= 63 and up to 16 dimensions */
    const struct tc_dtw_cand_boxes* pc_cand;  /* HOST pointer or NULL.  NULL: LB_PC boxes the
                               query's points when the query arrives (Sec. 5).  Otherwise LB_PC, in
                               tc_dtw_knn and tc_dtw_lower_bounds, uses these boxes of the candidates'
                               points, built ahead of time (Sec. 8; see tc_dtw_build_cand_boxes) */
    int32_t reuse_query_meta; /* searches of queries of uneven lengths or dims copy per-query
                               metadata (offsets, lengths, dims, table offsets) from host memory
                               into the workspace.  1: the workspace already holds that metadata
                               from a previous call with the same queries shapes, params and index,
                               so the call enqueues kernels only (and may be captured in a HIP
                               graph); 0: copy it (default). */
} tc_dtw_knn_params;

void tc_dtw_knn_params_default(tc_dtw_knn_params* p);

/* ------------------------------------------------ candidate-side boxes ---
 * LB_PC with the roles of query and candidate swapped (Sec. 8: the boxes of
 * the candidate series are computed once, when the database is set up,
 * instead of the query's boxes each time a query arrives).  For every
 * candidate c and every group g of w = p->pc_group consecutive QUERY
 * positions, the boxes of c's points in the expanded window
 * [g*w - W, g*w + w - 1 + W] (Sec. 5's quantisation-based clustering
 * applied to c, with p->pc_levels, pc_clusters and pc_min_cell).  The bound
 * of a pair is then the sum over the query's points of the smallest squared
 * distance to a box of the point's group; it bounds the same banded DTW
 * because the band is symmetric and DTW(q, c) = DTW(c, q) (Sec. 2, Eq. 1).
 * The boxes depend on the query length, the window and those parameters; a
 * search checks them against the descriptor (ERR_INVALID on a mismatch).
 *   ix         index with uniform candidate lengths (ERR_UNSUPPORTED otherwise)
 *   query_len  the length of the queries the boxes will serve (>= 1)
 *   buf        DEVICE, at least tc_dtw_cand_boxes_bytes() bytes, caller-owned
 *              and kept alive while searches use it; receives
 *              float boxes[count][groups][K][dim][2] (lo, hi; unused boxes
 *              +inf, -inf) and, at byte offset off_nbox, int32 nbox[count][groups]
 *   out        HOST descriptor, filled on success (pass it as p->pc_cand)
 * tc_dtw_cand_boxes_bytes returns 0 for invalid arguments.  Errors:
 * ERR_INVALID (bad index, length, parameters, null or short buffer),
 * ERR_UNSUPPORTED (ragged index, pc_levels^dim >= 2^63), ERR_HIP. */
typedef struct tc_dtw_cand_boxes {
    void* buf;            /* DEVICE */
    int64_t off_nbox;     /* byte offset of nbox inside buf */
    int32_t count, dim, query_len, cand_len;
    int32_t weff;         /* band half-width the boxes were built for */
    int32_t groups;       /* ceil(query_len / pc_group) */
    int32_t levels, clusters, group;
    float min_cell;
} tc_dtw_cand_boxes;

size_t tc_dtw_cand_boxes_bytes(const tc_dtw_index* ix, int32_t query_len, const tc_dtw_knn_params* p);
tc_dtw_status tc_dtw_build_cand_boxes(const tc_dtw_index* ix, int32_t query_len, const tc_dtw_knn_params* p,
                                      void* buf, size_t bytes, tc_dtw_cand_boxes* out, tc_dtw_stream stream);

/* ------------------------------------------------------- lower bounds ---
 * tc_dtw_lower_bounds: the dense bound matrix lb[q][c] (squared cost) of one
 * kind: TC_DTW_LB_MV (Sec. 3), TC_DTW_LB_PC (Sec. 5) or TC_DTW_LB_TI
 * (Sec. 4) with the parameters of `p`.  Every value is rounded so that it
 * never exceeds the exact bound of the float32 inputs, so it is safe to
 * prune with.  Uniform query and candidate lengths.
 *   lb   DEVICE float[queries->count * ix->count], row-major by query. */
size_t tc_dtw_lower_bounds_workspace_bytes(const tc_dtw_index* ix, const tc_dtw_batch* queries,
                                           const tc_dtw_knn_params* p, uint32_t kind);
tc_dtw_status tc_dtw_lower_bounds(const tc_dtw_index* ix, const tc_dtw_batch* queries,
                                  const tc_dtw_knn_params* p, uint32_t kind, float* lb,
                                  void* ws, size_t ws_bytes, tc_dtw_stream stream);

/* ---------------------------------------------------------------- k-NN ---
 * tc_dtw_knn: for every query, the indices of the p->k candidates with the
 * smallest banded DTW (dependent, or independent with p->independent; LB_MV
 * bounds both, being a sum of per-dimension envelope bounds, Sec. 3),
 * ordered by (distance, index) so that ties go to the
 * lower index, and those distances (Sec. 2 DTW-NN; Sec. 3 Definition 1;
 * k = 1 is the paper's nearest neighbour).  The result equals an exhaustive
 * float64 search: pruning and abandoning compare against an upper bound of
 * the k-th smallest distance with rigorous float32 error bounds, and every
 * candidate whose float32 DTW lies within those bounds of the k-th smallest
 * is re-scored in float64.
 * With an index of several banks (see tc_dtw_build_index) the queries may
 * have different D (queries->dims): each is searched against the bank of
 * its D in the same launches (every stage is one launch over all queries,
 * the work items of all banks mixed); nn_idx is the index in the whole
 * reference set; pairs counts query-bank pairs only.  (LB_MV bounds; k = 1.)
 *   nn_idx   DEVICE int32[queries->count * k], row-major by query
 *   nn_dist  DEVICE float[queries->count * k] (float64 DTW rounded to float32)
 *   stats    HOST or NULL.  When given, the call waits for the stream and
 *            fills the counters and per-stage times.
 * Errors: INVALID (dims differ, a query D with no bank, k < 1 or k >
 * candidates, bad parameters), UNSUPPORTED (k > 32; k > 1 with uneven
 * lengths or banks; independent DTW outside its limits or with LB_PC /
 * LB_TI), WORKSPACE, DEVICE. */
typedef struct {
    uint64_t pairs;          /* query-candidate pairs */
    uint64_t pruned_mv;      /* pairs skipped by LB_MV */
    uint64_t pruned_pc;      /* pairs skipped by LB_PC */
    uint64_t pruned_ti;      /* pairs skipped by LB_TI */
    uint64_t dtw_started;    /* pairs whose DTW was started (seeds included) */
    uint64_t dtw_abandoned;  /* of those, abandoned early */
    uint64_t dtw_completed;
    uint64_t cells;          /* DTW cells evaluated (abandoned pairs counted up to the abandoning step) */
    uint64_t rescored;       /* float64 re-scorings */
    float stage_ms[8];       /* prep, lb_mv, seed, compact, lb_pc+lb_ti, dtw, finalize, total */
    uint64_t evaluated_pc;   /* pairs whose LB_PC was evaluated (uniform searches) */
    uint64_t evaluated_ti;   /* pairs whose LB_TI was evaluated (uniform searches) */
    float lb_ti_ms;          /* the LB_TI launch's share of stage_ms[4] */
} tc_dtw_knn_stats;

size_t tc_dtw_knn_workspace_bytes(const tc_dtw_index* ix, const tc_dtw_batch* queries,
                                  const tc_dtw_knn_params* p);
tc_dtw_status tc_dtw_knn(const tc_dtw_index* ix, const tc_dtw_batch* queries,
                         const tc_dtw_knn_params* p, int32_t* nn_idx, float* nn_dist,
                         tc_dtw_knn_stats* stats, void* ws, size_t ws_bytes,
                         tc_dtw_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* TC_DTW_H */
