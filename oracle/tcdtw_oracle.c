/*
 * Reference oracle for multivariate (dependent) DTW nearest-neighbour search
 * with lower-bound filtering (TC-DTW, arXiv 2101.07731).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark; never by the GPU library.
 *
 * Plain FP64 C, written for readability rather than speed.  Built with
 * -ffp-contract=off so every product and sum is rounded separately, in the
 * order written.  Parallelism is limited to independent queries / pairs
 * (OpenMP), which does not change any result.
 *
 * Parity notes:
 *   - orc_knn_exhaustive is the plain definition of the 1-NN result;
 *   - the bounds follow the paper's steps, with the readings of the
 *     ambiguous points listed in each function's comment.
 */
#include "tcdtw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define INF HUGE_VAL

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* Squared Euclidean distance of two D-vectors, dimensions in increasing
 * order (dependent DTW point cost, Sec. 2 "Multivariate DTW"). */
static double point_cost(const double* a, const double* b, int D)
{
    double s = 0.0;
    for (int p = 0; p < D; ++p) {
        double d = a[p] - b[p];
        s += d * d;
    }
    return s;
}

/* Euclidean (not squared) point distance e(a,b): the metric on which the
 * triangle inequality of Sec. 4 holds. */
static double point_dist(const double* a, const double* b, int D)
{
    return sqrt(point_cost(a, b, D));
}

int orc_window_eff(int m, int n, int window, int num, int den)
{
    int longer = imax(m, n);
    long long W = den > 0 ? ((long long)longer * num) / den : window;
    int diff = abs(m - n);
    return W > diff ? (int)W : diff;
}

/* ---------------------------------------------------------------- DTW --- */

/* Sec. 2, Eq. 1: D(i,j) = cost(i,j) + min(D(i-1,j), D(i,j-1), D(i-1,j-1)),
 * D(0,0) = cost(0,0), restricted to the Sakoe-Chiba band |i-j| <= weff.
 * Cells outside the band or outside the matrix are +inf.  Two rows are
 * kept.  Row-wise early abandoning (Sec. 7.1): every warping path visits
 * every row and path prefixes only grow, so once the minimum of a
 * completed row reaches bsf the final value cannot be below bsf. */
double orc_dtw_ea(const double* q, int m, const double* c, int n, int D,
                  int weff, double bsf, int* abandoned)
{
    double* prev = (double*)malloc(sizeof(double) * (size_t)n);
    double* cur = (double*)malloc(sizeof(double) * (size_t)n);
    if (abandoned) *abandoned = 0;
    for (int j = 0; j < n; ++j) prev[j] = INF;
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) cur[j] = INF;
        int jlo = imax(0, i - weff), jhi = imin(n - 1, i + weff);
        double rowmin = INF;
        for (int j = jlo; j <= jhi; ++j) {
            double best;
            if (i == 0 && j == 0) {
                best = 0.0;
            } else {
                best = INF;
                if (i > 0 && j - (i - 1) <= weff) best = dmin(best, prev[j]);       /* (i-1, j)   */
                if (j > 0 && i - (j - 1) <= weff) best = dmin(best, cur[j - 1]);    /* (i,   j-1) */
                if (i > 0 && j > 0) best = dmin(best, prev[j - 1]);                 /* (i-1, j-1) */
            }
            cur[j] = point_cost(q + (size_t)i * D, c + (size_t)j * D, D) + best;
            rowmin = dmin(rowmin, cur[j]);
        }
        double* t = prev; prev = cur; cur = t;
        if (bsf < INF && rowmin >= bsf) {
            free(prev); free(cur);
            if (abandoned) *abandoned = 1;
            return INF;
        }
    }
    double r = prev[n - 1];
    free(prev); free(cur);
    return r;
}

double orc_dtw(const double* q, int m, const double* c, int n, int D, int weff)
{
    return orc_dtw_ea(q, m, c, n, D, weff, INF, NULL);
}

void orc_dtw_pairs(const double* x, const int64_t* xoff, const int32_t* xlen,
                   const double* y, const int64_t* yoff, const int32_t* ylen,
                   int npairs, int D, int window, int num, int den,
                   int threads, double* out)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
    for (int k = 0; k < npairs; ++k) {
        int m = xlen[k], n = ylen[k];
        int weff = orc_window_eff(m, n, window, num, den);
        out[k] = orc_dtw(x + xoff[k], m, y + yoff[k], n, D, weff);
    }
}

/* Path gradient of DTW.  The paper uses DTW as a loss only as motivation
 * (Sec. 1, Sec. 9); the derivative of the banded DTW value along a fixed
 * optimal path is the sum of the derivatives of the point costs on it. */
double orc_dtw_path_grad(const double* q, int m, const double* c, int n, int D,
                         int weff, double gbar, double* gq, double* gc,
                         int32_t* path, int32_t* plen)
{
    double* A = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n);
    for (size_t t = 0; t < (size_t)m * (size_t)n; ++t) A[t] = INF;
#define CELL(i, j) A[(size_t)(i) * (size_t)n + (size_t)(j)]
    for (int i = 0; i < m; ++i) {
        int jlo = imax(0, i - weff), jhi = imin(n - 1, i + weff);
        for (int j = jlo; j <= jhi; ++j) {
            double best;
            if (i == 0 && j == 0) {
                best = 0.0;
            } else {
                best = INF;
                if (i > 0 && j - (i - 1) <= weff) best = dmin(best, CELL(i - 1, j));
                if (j > 0 && i - (j - 1) <= weff) best = dmin(best, CELL(i, j - 1));
                if (i > 0 && j > 0) best = dmin(best, CELL(i - 1, j - 1));
            }
            CELL(i, j) = point_cost(q + (size_t)i * D, c + (size_t)j * D, D) + best;
        }
    }
    double value = CELL(m - 1, n - 1);
    for (size_t t = 0; t < (size_t)m * D; ++t) gq[t] = 0.0;
    for (size_t t = 0; t < (size_t)n * D; ++t) gc[t] = 0.0;
    int i = m - 1, j = n - 1, len = 0;
    for (;;) {
        if (path) { path[2 * len] = i; path[2 * len + 1] = j; }
        ++len;
        for (int p = 0; p < D; ++p) {
            double d = q[(size_t)i * D + p] - c[(size_t)j * D + p];
            gq[(size_t)i * D + p] += gbar * 2.0 * d;
            gc[(size_t)j * D + p] -= gbar * 2.0 * d;
        }
        if (i == 0 && j == 0) break;
        /* predecessor with the smallest value; ties: diagonal, up, left */
        int bi = -1, bj = -1;
        double bv = INF;
        if (i > 0 && j > 0) { bi = i - 1; bj = j - 1; bv = CELL(i - 1, j - 1); }
        if (i > 0 && j - (i - 1) <= weff && CELL(i - 1, j) < bv) { bi = i - 1; bj = j; bv = CELL(i - 1, j); }
        if (j > 0 && i - (j - 1) <= weff && CELL(i, j - 1) < bv) { bi = i; bj = j - 1; bv = CELL(i, j - 1); }
        i = bi; j = bj;
    }
#undef CELL
    if (plen) *plen = len;
    free(A);
    return value;
}

/* --------------------------------------------------------- lower bounds --- */

/* Every bound below is computed per candidate point c_j against the query
 * points of its window I(j) = [j-weff, j+weff] clipped to [0,m), and summed
 * over j.  It is sound because every warping path visits every column j at
 * some row i in I(j) and all point costs are non-negative. */

void orc_envelope(const double* q, int m, int n, int D, int weff, double* U, double* L)
{
    for (int j = 0; j < n; ++j) {
        int ilo = imax(0, j - weff), ihi = imin(m - 1, j + weff);
        for (int p = 0; p < D; ++p) {
            double u = -INF, l = INF;
            for (int i = ilo; i <= ihi; ++i) {
                u = dmax(u, q[(size_t)i * D + p]);
                l = dmin(l, q[(size_t)i * D + p]);
            }
            U[(size_t)j * D + p] = u;
            L[(size_t)j * D + p] = l;
        }
    }
}

/* Sec. 3, LB_MV: squared excess of each candidate coordinate over the
 * query envelope, summed over points and dimensions. */
double orc_lb_mv(const double* q, int m, const double* c, int n, int D, int weff)
{
    double* U = (double*)malloc(sizeof(double) * (size_t)n * D);
    double* L = (double*)malloc(sizeof(double) * (size_t)n * D);
    orc_envelope(q, m, n, D, weff, U, L);
    double lb = 0.0;
    for (int j = 0; j < n; ++j) {
        for (int p = 0; p < D; ++p) {
            double x = c[(size_t)j * D + p];
            double u = U[(size_t)j * D + p], l = L[(size_t)j * D + p];
            if (x > u) lb += (x - u) * (x - u);
            else if (x < l) lb += (l - x) * (l - x);
        }
    }
    free(U); free(L);
    return lb;
}

/* Sec. 3, LB_AD: the smallest true point cost in each candidate point's
 * window. */
double orc_lb_ad(const double* q, int m, const double* c, int n, int D, int weff)
{
    double lb = 0.0;
    for (int j = 0; j < n; ++j) {
        int ilo = imax(0, j - weff), ihi = imin(m - 1, j + weff);
        double best = INF;
        for (int i = ilo; i <= ihi; ++i)
            best = dmin(best, point_cost(q + (size_t)i * D, c + (size_t)j * D, D));
        lb += best;
    }
    return lb;
}

/* Sec. 4.1 / 4.2: triangle bounds L(i,j) <= e(q_i,c_j) <= U(i,j).
 * Rows are processed in order; within row i the window is
 * J(i) = [i-weff, i+weff] clipped to [0,n).
 *   - row 0, and rows with i mod P == 0 when P > 0: exact distances
 *     (initialisation of Sec. 4.1; periodic rows of LB_TIP, Sec. 4.2);
 *   - cells whose (i-1,j) lies in the band: Eqs. 7-8 with the query step
 *     delta_i = e(q_{i-1}, q_i);
 *   - the top cell j = i+weff: exact under LB_TI_TOP, else Eqs. 9-10 from
 *     (i,j-1) with the candidate step gamma_j = e(c_{j-1}, c_j); exact if
 *     (i,j-1) is not in the band (only when weff = 0).
 * The recursion is applied literally (no clamping); a negative lower bound
 * is clamped to 0 only where it is used.  Lo/Hi receive every band cell. */
static void ti_core(const double* q, int m, const double* c, int n, int D, int weff,
                    int P, int top, double* colmin, double* Lo, double* Hi)
{
    double* delta = (double*)malloc(sizeof(double) * (size_t)m);
    double* gamma = (double*)malloc(sizeof(double) * (size_t)n);
    double* Lp = (double*)malloc(sizeof(double) * (size_t)n);
    double* Up = (double*)malloc(sizeof(double) * (size_t)n);
    double* Lc = (double*)malloc(sizeof(double) * (size_t)n);
    double* Uc = (double*)malloc(sizeof(double) * (size_t)n);
    delta[0] = 0.0;
    for (int i = 1; i < m; ++i) delta[i] = point_dist(q + (size_t)(i - 1) * D, q + (size_t)i * D, D);
    gamma[0] = 0.0;
    for (int j = 1; j < n; ++j) gamma[j] = point_dist(c + (size_t)(j - 1) * D, c + (size_t)j * D, D);
    for (int j = 0; j < n; ++j) colmin[j] = INF;
    for (int i = 0; i < m; ++i) {
        int exact_row = (i == 0) || (P > 0 && i % P == 0);
        int jlo = imax(0, i - weff), jhi = imin(n - 1, i + weff);
        for (int j = jlo; j <= jhi; ++j) {
            double lo, hi;
            if (exact_row) {
                lo = hi = point_dist(q + (size_t)i * D, c + (size_t)j * D, D);
            } else if (j <= i - 1 + weff) {
                /* triangle (q_{i-1}, q_i, c_j) */
                lo = dmax(Lp[j] - delta[i], delta[i] - Up[j]);
                hi = Up[j] + delta[i];
            } else if (top) {
                lo = hi = point_dist(q + (size_t)i * D, c + (size_t)j * D, D);
            } else if (j - 1 >= jlo) {
                /* triangle (c_{j-1}, c_j, q_i) at the top of the window */
                lo = dmax(Lc[j - 1] - gamma[j], gamma[j] - Uc[j - 1]);
                hi = Uc[j - 1] + gamma[j];
            } else {
                lo = hi = point_dist(q + (size_t)i * D, c + (size_t)j * D, D);
            }
            Lc[j] = lo;
            Uc[j] = hi;
            if (Lo) { Lo[(size_t)i * n + j] = lo; Hi[(size_t)i * n + j] = hi; }
            colmin[j] = dmin(colmin[j], dmax(0.0, lo));
        }
        double* t;
        t = Lp; Lp = Lc; Lc = t;
        t = Up; Up = Uc; Uc = t;
    }
    free(delta); free(gamma); free(Lp); free(Up); free(Lc); free(Uc);
}

/* Fig. 3 / Sec. 4.1: per candidate point the smallest of its lower bounds
 * over its window, squared (the bounds are on the Euclidean distance, the
 * DTW is in squared cost), summed over candidate points. */
double orc_lb_ti(const double* q, int m, const double* c, int n, int D, int weff,
                 int P, int top)
{
    double* colmin = (double*)malloc(sizeof(double) * (size_t)n);
    ti_core(q, m, c, n, D, weff, P, top, colmin, NULL, NULL);
    double lb = 0.0;
    for (int j = 0; j < n; ++j) lb += colmin[j] * colmin[j];
    free(colmin);
    return lb;
}

void orc_ti_cells(const double* q, int m, const double* c, int n, int D, int weff,
                  int P, int top, double* Lo, double* Hi)
{
    for (size_t t = 0; t < (size_t)m * (size_t)n; ++t) { Lo[t] = NAN; Hi[t] = NAN; }
    double* colmin = (double*)malloc(sizeof(double) * (size_t)n);
    ti_core(q, m, c, n, D, weff, P, top, colmin, Lo, Hi);
    free(colmin);
}

/* Sec. 5: quantisation-based clustering of the query points of each
 * expanded window (uniform window grouping with expansion factor w).
 * Cell assignment is done in float32 so that another float32
 * implementation can reproduce it bit for bit:
 *   lo_p, hi_p   = min / max of dimension p over the window's points,
 *   len_p        = max((hi_p - lo_p) / Lv, floor_len),
 *   digit_p(x)   = min(Lv-1, floor((x_p - lo_p) / len_p)),
 *   cell key     = sum_p digit_p * Lv^(D-1-p)   (lexicographic order).
 * The distinct keys sorted ascending are k_1 < ... < k_M.  Keys k_1..k_{K-1}
 * are one box each; if M > K every key >= k_K joins box K ("the last ...
 * extra boxes are combined").  A box is the tight bounding box of its
 * member points (the bounding box to which LB_MV is applied per group). */
static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int orc_pc_boxes(const double* q, int m, int n, int D, int weff, int Lv, int K,
                 int w, float floor_len, double* box_lo, double* box_hi,
                 int32_t* nbox)
{
    /* Lv^D must fit in 63 bits */
    uint64_t pw = 1;
    for (int p = 0; p < D; ++p) {
        if (pw > (UINT64_C(1) << 62) / (uint64_t)Lv) return -1;
        pw *= (uint64_t)Lv;
    }
    int ngroups = (n + w - 1) / w;
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)m);
    uint64_t* sorted = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)m);
    float* lo = (float*)malloc(sizeof(float) * (size_t)D);
    float* len = (float*)malloc(sizeof(float) * (size_t)D);
    for (int g = 0; g < ngroups; ++g) {
        int jfirst = g * w, jlast = imin(n - 1, g * w + w - 1);
        int ilo = imax(0, jfirst - weff), ihi = imin(m - 1, jlast + weff);
        int npts = ihi - ilo + 1;
        for (int p = 0; p < D; ++p) {
            float a = (float)q[(size_t)ilo * D + p], b = a;
            for (int i = ilo; i <= ihi; ++i) {
                float x = (float)q[(size_t)i * D + p];
                if (x < a) a = x;
                if (x > b) b = x;
            }
            float l = (b - a) / (float)Lv;
            if (l < floor_len) l = floor_len;
            lo[p] = a;
            len[p] = l;
        }
        for (int i = ilo; i <= ihi; ++i) {
            uint64_t key = 0;
            for (int p = 0; p < D; ++p) {
                float x = (float)q[(size_t)i * D + p];
                /* len_p >= (hi_p - lo_p) / Lv, so r stays within [0, Lv] */
                int dgt = 0;
                if (len[p] > 0.0f) {
                    float r = (x - lo[p]) / len[p];
                    dgt = (int)floorf(r);
                }
                if (dgt > Lv - 1) dgt = Lv - 1;
                key = key * (uint64_t)Lv + (uint64_t)dgt;
            }
            keys[i - ilo] = key;
            sorted[i - ilo] = key;
        }
        qsort(sorted, (size_t)npts, sizeof(uint64_t), cmp_u64);
        int M = 0;
        for (int t = 0; t < npts; ++t)
            if (t == 0 || sorted[t] != sorted[t - 1]) sorted[M++] = sorted[t];
        int nb = M < K ? M : K;
        nbox[g] = nb;
        double* blo = box_lo + (size_t)g * K * D;
        double* bhi = box_hi + (size_t)g * K * D;
        for (int t = 0; t < K * D; ++t) { blo[t] = INF; bhi[t] = -INF; }
        for (int i = ilo; i <= ihi; ++i) {
            /* rank of this point's key among the distinct keys */
            int rank = 0;
            while (sorted[rank] != keys[i - ilo]) ++rank;
            int b = rank < K - 1 ? rank : K - 1;
            for (int p = 0; p < D; ++p) {
                double x = q[(size_t)i * D + p];
                blo[(size_t)b * D + p] = dmin(blo[(size_t)b * D + p], x);
                bhi[(size_t)b * D + p] = dmax(bhi[(size_t)b * D + p], x);
            }
        }
    }
    free(keys); free(sorted); free(lo); free(len);
    return ngroups;
}

/* Sec. 5: LB_MV applied per box; a candidate point takes the smallest
 * squared distance to any box of its group. */
double orc_lb_pc(const double* q, int m, const double* c, int n, int D, int weff,
                 int Lv, int K, int w, float floor_len)
{
    int ngroups = (n + w - 1) / w;
    double* blo = (double*)malloc(sizeof(double) * (size_t)ngroups * K * D);
    double* bhi = (double*)malloc(sizeof(double) * (size_t)ngroups * K * D);
    int32_t* nb = (int32_t*)malloc(sizeof(int32_t) * (size_t)ngroups);
    if (orc_pc_boxes(q, m, n, D, weff, Lv, K, w, floor_len, blo, bhi, nb) < 0) {
        free(blo); free(bhi); free(nb);
        return NAN;
    }
    double lb = 0.0;
    for (int j = 0; j < n; ++j) {
        int g = j / w;
        double best = INF;
        for (int b = 0; b < nb[g]; ++b) {
            const double* lo = blo + ((size_t)g * K + b) * D;
            const double* hi = bhi + ((size_t)g * K + b) * D;
            double s = 0.0;
            for (int p = 0; p < D; ++p) {
                double x = c[(size_t)j * D + p];
                double e = 0.0;
                if (x < lo[p]) e = lo[p] - x;
                else if (x > hi[p]) e = x - hi[p];
                s += e * e;
            }
            best = dmin(best, s);
        }
        lb += best;
    }
    free(blo); free(bhi); free(nb);
    return lb;
}

/* ----------------------------------------------------------------- 1-NN --- */

void orc_knn_exhaustive(const double* Q, const int64_t* qoff, const int32_t* qlen, int nq,
                        const double* C, const int64_t* coff, const int32_t* clen, int nc,
                        int D, int window, int num, int den, int threads,
                        int32_t* nn_idx, double* nn_dist)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
    for (int a = 0; a < nq; ++a) {
        double best = INF;
        int arg = -1;
        for (int k = 0; k < nc; ++k) {
            int weff = orc_window_eff(qlen[a], clen[k], window, num, den);
            double d = orc_dtw(Q + qoff[a], qlen[a], C + coff[k], clen[k], D, weff);
            if (d < best) { best = d; arg = k; }
        }
        nn_idx[a] = arg;
        nn_dist[a] = best;
    }
}

void orc_knn_cascade(const double* Q, const int64_t* qoff, const int32_t* qlen, int nq,
                     const double* C, const int64_t* coff, const int32_t* clen, int nc,
                     int D, int window, int num, int den, uint32_t bounds,
                     int ti_P, int ti_top, int pc_Lv, int pc_K, int pc_w, float pc_floor,
                     double e_ti, double e_pc, int threads,
                     int32_t* nn_idx, double* nn_dist, orc_cascade_stats* stats)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : 1)
    for (int a = 0; a < nq; ++a) {
        const double* q = Q + qoff[a];
        int m = qlen[a];
        orc_cascade_stats st;
        memset(&st, 0, sizeof st);
        double bsf = INF;
        int arg = -1;
        for (int k = 0; k < nc; ++k) {
            const double* c = C + coff[k];
            int n = clen[k];
            int weff = orc_window_eff(m, n, window, num, den);
            ++st.pairs;
            double lb = orc_lb_mv(q, m, c, n, D, weff);
            if (lb >= bsf) { ++st.pruned_mv; continue; }
            if ((bounds & 2u) && lb > e_pc * e_pc * bsf) {
                lb = dmax(lb, orc_lb_pc(q, m, c, n, D, weff, pc_Lv, pc_K, pc_w, pc_floor));
                if (lb >= bsf) { ++st.pruned_pc; continue; }
            }
            if ((bounds & 4u) && lb > e_ti * e_ti * bsf) {
                lb = dmax(lb, orc_lb_ti(q, m, c, n, D, weff, ti_P, ti_top));
                if (lb >= bsf) { ++st.pruned_ti; continue; }
            }
            ++st.dtw_started;
            int ab = 0;
            double d = orc_dtw_ea(q, m, c, n, D, weff, bsf, &ab);
            if (ab) { ++st.dtw_abandoned; continue; }
            if (d < bsf) { bsf = d; arg = k; }
        }
        nn_idx[a] = arg;
        nn_dist[a] = bsf;
        if (stats) stats[a] = st;
    }
}
