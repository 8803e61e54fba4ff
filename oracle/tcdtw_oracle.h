/*
 * Reference oracle for multivariate (dependent) DTW nearest-neighbour search
 * with lower-bound filtering (TC-DTW, arXiv 2101.07731).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU restatement of
 * what the GPU path computes.  Only the test-suite, the package smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the GPU library and the GPU library never
 * calls it.
 *
 * Conventions (all functions):
 *   - series are row-major [t][d] arrays of doubles (the caller promotes the
 *     float32 inputs exactly);
 *   - indices are 0-based (the paper counts from 1);
 *   - the point cost is the squared Euclidean distance between two
 *     D-vectors, summed in increasing dimension order; every distance and
 *     every bound lives in that squared space and no square root is taken
 *     of a DTW value;
 *   - `weff` is the effective Sakoe-Chiba half-width max(W, |m-n|), which
 *     keeps the end cell reachable when the lengths differ
 *     (orc_window_eff computes it).
 */
#ifndef TCDTW_ORACLE_H
#define TCDTW_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Effective window for one pair of lengths (Sec. 2, "Window DTW").
 * W = floor(max(m,n) * num / den) when den > 0, else W = window;
 * the result is max(W, |m-n|). */
int orc_window_eff(int m, int n, int window, int num, int den);

/* Banded DTW (Sec. 2, Eq. 1, with the Sakoe-Chiba constraint |i-j| <= W). */
double orc_dtw(const double* q, int m, const double* c, int n, int D, int weff);

/* Same recurrence with row-wise early abandoning (Sec. 7.1): returns +inf
 * as soon as a whole band row has a minimum >= bsf; *abandoned is set to 1
 * in that case.  With bsf = +inf it equals orc_dtw. */
double orc_dtw_ea(const double* q, int m, const double* c, int n, int D,
                  int weff, double bsf, int* abandoned);

/* DTW for many pairs: pair k is (x + xoff[k], xlen[k]) against
 * (y + yoff[k], ylen[k]); offsets are in doubles.  Window per pair from
 * (window, num, den).  OpenMP over pairs with `threads` threads. */
void orc_dtw_pairs(const double* x, const int64_t* xoff, const int32_t* xlen,
                   const double* y, const int64_t* yoff, const int32_t* ylen,
                   int npairs, int D, int window, int num, int den,
                   int threads, double* out);

/* Gradient of DTW along one optimal warping path.  The full band DP is
 * kept; the path is traced back from (m-1,n-1) taking the smallest
 * predecessor with tie priority diagonal, then (i-1,j), then (i,j-1).
 * gq[i] = gbar * sum_{j:(i,j) on path} 2(q_i - c_j), gc likewise with the
 * sign flipped.  path (optional, 2*(m+n) ints) receives (i,j) pairs from
 * the end cell back to (0,0); *plen its length.  Returns the DTW value. */
double orc_dtw_path_grad(const double* q, int m, const double* c, int n, int D,
                         int weff, double gbar, double* gq, double* gc,
                         int32_t* path, int32_t* plen);

/* Query envelope (Sec. 3, LB_MV): for every candidate position j in
 * [0,n) the max / min of each query dimension over the query window
 * [j-weff, j+weff] clipped to [0,m).  U, L are [n][D]. */
void orc_envelope(const double* q, int m, int n, int D, int weff, double* U, double* L);

/* LB_MV (Sec. 3), squared form (no outer square root). */
double orc_lb_mv(const double* q, int m, const double* c, int n, int D, int weff);

/* LB_AD (Sec. 3): per candidate point, the smallest true point cost over
 * its query window; summed over candidate points. */
double orc_lb_ad(const double* q, int m, const double* c, int n, int D, int weff);

/* LB_TI family (Sec. 4.1, Eqs. 7-10; Sec. 4.2).  P > 0: rows i with
 * i mod P == 0 are computed exactly (LB_TIP); P <= 0: only row 0 (basic
 * LB_TI).  top != 0: the top cell of each row's window is computed exactly
 * (LB_TI_TOP).  The default of the paper's experiments is P = 5, top = 1. */
double orc_lb_ti(const double* q, int m, const double* c, int n, int D, int weff,
                 int P, int top);

/* Per-cell triangle bounds of the LB_TI recursion, for invariant checks:
 * Lo, Hi are [m][n]; cells outside the band are set to NaN. */
void orc_ti_cells(const double* q, int m, const double* c, int n, int D, int weff,
                  int P, int top, double* Lo, double* Hi);

/* LB_PC clustering stage (Sec. 5, quantisation-based clustering with
 * uniform window grouping).  For group g (candidate positions
 * [g*w, min(n,(g+1)*w)) ), the query points of the expanded window are
 * quantised with Lv levels per dimension in float32 arithmetic, distinct
 * cells are ordered lexicographically (dimension 0 most significant), the
 * first K-1 cells form one box each and all later cells share box K, and
 * each box is the tight [min,max] of its member points.
 * box_lo, box_hi: [ngroups][K][D]; nbox: [ngroups]; ngroups = ceil(n/w).
 * floor_len is the smallest cell length.  Returns ngroups, or -1 if
 * Lv^D does not fit 63 bits. */
int orc_pc_boxes(const double* q, int m, int n, int D, int weff, int Lv, int K,
                 int w, float floor_len, double* box_lo, double* box_hi,
                 int32_t* nbox);

/* LB_PC (Sec. 5): sum over candidate points of the smallest squared
 * distance to a box of the point's group. */
double orc_lb_pc(const double* q, int m, const double* c, int n, int D, int weff,
                 int Lv, int K, int w, float floor_len);

/* Exhaustive 1-NN (the "default windowed DTW", Sec. 2 DTW-NN and Sec. 7.2):
 * nn_idx[q] = argmin_k DTW(Q_q, C_k), ties to the lowest k.
 * Series s of a set occupies data[off[s] .. off[s] + len[s]*D). */
void orc_knn_exhaustive(const double* Q, const int64_t* qoff, const int32_t* qlen, int nq,
                        const double* C, const int64_t* coff, const int32_t* clen, int nc,
                        int D, int window, int num, int den, int threads,
                        int32_t* nn_idx, double* nn_dist);

/* Counters of the sequential cascade, per query. */
typedef struct {
    int64_t pairs, pruned_mv, pruned_pc, pruned_ti, dtw_started, dtw_abandoned;
} orc_cascade_stats;

/* The paper's filtering cascade, sequential per query in index order
 * (Sec. 2 DTW-NN, Sec. 6 selective deployment, Sec. 7.1 early abandoning):
 * LB_MV first; LB_PC and then LB_TI are applied only when
 * LB_MV > e^2 * bsf (the squared-space form of e < LB_MV/d_best); a
 * candidate is skipped once a bound reaches bsf; otherwise DTW with
 * row-wise early abandoning.  bounds bit 1 = PC, bit 2 = TI.
 * Returns the same (nn_idx, nn_dist) as orc_knn_exhaustive. */
void orc_knn_cascade(const double* Q, const int64_t* qoff, const int32_t* qlen, int nq,
                     const double* C, const int64_t* coff, const int32_t* clen, int nc,
                     int D, int window, int num, int den, uint32_t bounds,
                     int ti_P, int ti_top, int pc_Lv, int pc_K, int pc_w, float pc_floor,
                     double e_ti, double e_pc, int threads,
                     int32_t* nn_idx, double* nn_dist, orc_cascade_stats* stats);

#ifdef __cplusplus
}
#endif
#endif
