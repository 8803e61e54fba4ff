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
 *    allocates or frees device memory; sizes come from the *_bytes()
 *    queries.  Workspace contents need no initialisation and are
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

#define TC_DTW_ABI_VERSION 1

typedef struct ihipStream_t* tc_dtw_stream; /* same type as hipStream_t; NULL = default stream */

typedef enum {
    TC_DTW_OK = 0,
    TC_DTW_ERR_INVALID = 1,     /* bad argument (null pointer, count, length, window, mismatch) */
    TC_DTW_ERR_WORKSPACE = 2,   /* a caller buffer is smaller than its *_bytes() query */
    TC_DTW_ERR_UNSUPPORTED = 3, /* valid but not supported (D > 64, k != 1, key overflow) */
    TC_DTW_ERR_DEVICE = 4       /* no usable gfx950 device, or a HIP call failed */
} tc_dtw_status;

/* A set of D-dimensional float32 series.
 *   data    DEVICE  series s occupies data[offset[s] .. offset[s] + len[s]*dim),
 *                   row-major [t][d] (a torch [B, T, D] tensor when uniform).
 *   offset  HOST    per-series start in floats, or NULL: s * uniform_len * dim.
 *   len     HOST    per-series length, or NULL: every series has uniform_len.
 *   count   number of series (>= 1).
 *   dim     D, shared by all series of the set (1..64).
 *   uniform_len  length of every series when len == NULL, else ignored. */
typedef struct {
    const float* data;
    const int64_t* offset;
    const int32_t* len;
    int32_t count;
    int32_t dim;
    int32_t uniform_len;
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

#ifdef __cplusplus
}
#endif
#endif /* TC_DTW_H */
