// Device-side DTW cores shared by the pair kernels and the 1-NN kernels.
//
// Both cores evaluate the DTW recurrence (Sec. 2, Eq. 1) inside the
// Sakoe-Chiba band along anti-diagonals, one cell per lane per step, with
// neighbour values passed by DPP whole-wave shifts.  See dtw_fwd.hip for
// the lane layouts.
#pragma once
#include "device_common.h"
#include "internal.h"

namespace tcdtw {

// The dynamic LDS of every kernel of the library, addressed by float4 index
// so that every access is known to be an LDS access.
extern __shared__ float4 lds4[];

// ------------------------------------------------------------------ staging
// Copies series `src` (row-major [len][D]) into LDS as [k][L][4] chunks for
// positions pos = 0..L-1 holding series index t = pos + first; positions
// outside [0, len) get `sentinel` in every component.
template <int NCH>
__device__ __forceinline__ void stage_series(int dst, int L, int first, const float* src, int len,
                                             int D, float sentinel, int lane, int nlanes) {
    for (int pos = lane; pos < L; pos += nlanes) {
        const int t = pos + first;
        const bool in = (t >= 0 && t < len);
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = 4 * k + e;
                v[e] = in ? (p < D ? src[(int64_t)t * D + p] : 0.0f) : sentinel;
            }
            lds4[dst + k * L + pos] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

// Dimension p of series `src` ([len][D]) as single-chunk points (v, 0, 0, 0)
// at positions pos = 0..L-1 (t = pos + first); `sentinel` outside [0, len).
__device__ __forceinline__ void stage_dim(int dst, int L, int first, const float* src, int len, int D,
                                          int p, float sentinel, int lane, int nlanes) {
    for (int pos = lane; pos < L; pos += nlanes) {
        const int t = pos + first;
        const bool in = (t >= 0 && t < len);
        lds4[dst + pos] = in ? make_float4(src[(int64_t)t * D + p], 0.0f, 0.0f, 0.0f)
                             : make_float4(sentinel, sentinel, sentinel, sentinel);
    }
}

// ---------------------------------------------------------- diagonal pairs
struct DiagGeom {
    int m, n, W, G, h, R, LQ, LC;
    __host__ __device__ void init(int m_, int n_, int W_) {
        m = m_; n = n_; W = W_;
        G = W + 1;
        h = (W + (W & 1)) / 2;
        R = (m + n) / 2;           // rounds: anti-diagonals 0 .. m+n-2
        LQ = R + W + 1;            // query positions, index i = pos + h - W
        LC = R + W + 2;            // candidate positions, index j = pos - h
    }
    __host__ __device__ int qfirst() const { return h - W; }
    __host__ __device__ int cfirst() const { return -h; }
};

// Early-abandon context of a wave (1-NN mode): every `every` rounds the
// groups whose cells on two consecutive anti-diagonals all exceed `thr`
// are abandoned; the loop ends when every live group is.
struct Abandon {
    const unsigned long long* key;   // packed best-so-far of the wave's query
    float gamma;                     // relative error bound of the float DP
    uint64_t valid_mask;             // lanes of groups with a pair
};

__device__ __forceinline__ float bsf_from_key(unsigned long long k) {
    return __uint_as_float((uint32_t)(k >> 32));
}

// Abandon threshold: a cell value v (float DP) proves DTW > bsf when
// v / (1 + gamma) > bsf; computed in double and rounded up.
__device__ __forceinline__ float abandon_threshold(float bsf, float gamma) {
    const double t = (double)bsf * (1.0 + (double)gamma) * (1.0 + 1e-6);
    float f = (float)t;
    if ((double)f < t) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

// One round of the diagonal mapping: E step on anti-diagonal 2r with the
// candidate point cin, O step on 2r+1 with the candidate point loaded into
// cout (which the next round uses as its cin).
// Smallest of (diag, up, left) and its 2-bit code (0 diagonal, 1 up, 2 left;
// ties go to the earlier of that order).  The minimum comes from one 3-way
// min, so the DP recurrence does not wait on the comparisons that form the code.
template <typename T>
__device__ __forceinline__ T min3_code(T diag, T up, T left, uint32_t& code) {
    const T best = vmin3(diag, up, left);
    code = best == diag ? 0u : (best == up ? 1u : 2u);
    return best;
}

template <typename T, int NCH, bool SAVE, bool WODD>
__device__ __forceinline__ void diag_round(const int (&qk)[NCH], const int (&ck)[NCH],
                                           int off, const float4 (&cin)[NCH], float4 (&cout)[NCH],
                                           bool kill_e, bool kill_o, T& vE, T& vO, uint32_t& cw,
                                           int shift) {
    const T INF = inf_v<T>();
    float4 qv[NCH];
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        qv[k] = lds4[qk[k] + off];
        cout[k] = lds4[ck[k] + off + 1];
    }
    {   // E step: up = own odd slot, left = lane-1's odd slot, diag = own even slot
        const T cost = point_cost<NCH>(qv, cin, T(0));
        const T up = vO;
        const T left = wave_shr1(INF, vO);
        T best;
        if (SAVE) {
            uint32_t code;
            best = min3_code(vE, up, left, code);
            cw |= code << shift;
        } else {
            best = vmin3(vE, up, left);
        }
        T v = add_cost(cost, best);
        if (WODD && kill_e) v = INF;
        vE = v;
    }
    {   // O step: up = lane+1's even slot, left = own even slot, diag = own odd slot
        const T cost = point_cost<NCH>(qv, cout, T(0));
        const T up = wave_shl1(INF, vE);
        const T left = vE;
        T best;
        if (SAVE) {
            uint32_t code;
            best = min3_code(vO, up, left, code);
            cw |= code << (shift + 2);
        } else {
            best = vmin3(vO, up, left);
        }
        T v = add_cost(cost, best);
        if (!WODD && kill_o) v = INF;
        vO = v;
    }
}

// The round of diag_round for float values without argmin codes, with the
// neighbour values passed by whole-wave rotations and the minimum taken on
// the bit patterns (every DP value is >= +0 or +inf, never NaN).  Rotations
// give lane 0 the value of lane 63 and lane 63 that of lane 0, so they need
// the caller's layout to hold +inf there: with WODD lane 0's even slot (its
// E step is killed), otherwise lane 63's odd slot (lane 63 is a padding
// lane or belongs to no pair, and its O step is killed).
// The two steps of a round on points already in registers.
template <int NCH, bool WODD>
__device__ __forceinline__ void diag_steps_rot(const float4 (&qv)[NCH], const float4 (&cin)[NCH],
                                               const float4 (&cout)[NCH], bool kill_e, bool kill_o,
                                               float& vE, float& vO) {
    {   // E step: up = own odd slot, left = lane-1's odd slot, diag = own even slot
        const float cost = point_cost<NCH>(qv, cin, 0.0f);
        const uint32_t o = __float_as_uint(vO);
        float v = cost + __uint_as_float(umin3(__float_as_uint(vE), o, wave_ror1(o)));
        if (WODD && kill_e) v = __builtin_inff();
        vE = v;
    }
    {   // O step: up = lane+1's even slot, left = own even slot, diag = own odd slot
        const float cost = point_cost<NCH>(qv, cout, 0.0f);
        const uint32_t e = __float_as_uint(vE);
        float v = cost + __uint_as_float(umin3(__float_as_uint(vO), wave_rol1(e), e));
        if (!WODD && kill_o) v = __builtin_inff();
        vO = v;
    }
}

// Component p (0 .. 4 NCH - 1) of a point held as NCH float4 chunks.
template <int NCH>
__device__ __forceinline__ float comp(const float4 (&v)[NCH], int p) {
    const float4 x = v[p >> 2];
    return (p & 3) == 0 ? x.x : (p & 3) == 1 ? x.y : (p & 3) == 2 ? x.z : x.w;
}

// Independent DTW (DTW_I): the steps of diag_steps_rot for every dimension
// p with its own DP values vE[p], vO[p] and the univariate cost
// (q_p - c_p)^2; the kills and neighbour exchanges are those of the
// dependent case, per dimension.
template <int NCH, bool WODD>
__device__ __forceinline__ void diag_steps_indep(const float4 (&qv)[NCH], const float4 (&cin)[NCH],
                                                 const float4 (&cout)[NCH], bool kill_e, bool kill_o,
                                                 float (&vE)[4 * NCH], float (&vO)[4 * NCH]) {
#pragma unroll
    for (int p = 0; p < 4 * NCH; ++p) {
        const float d = comp<NCH>(qv, p) - comp<NCH>(cin, p);
        const uint32_t o = __float_as_uint(vO[p]);
        float v = d * d + __uint_as_float(umin3(__float_as_uint(vE[p]), o, wave_ror1(o)));
        if (WODD && kill_e) v = __builtin_inff();
        vE[p] = v;
    }
#pragma unroll
    for (int p = 0; p < 4 * NCH; ++p) {
        const float d = comp<NCH>(qv, p) - comp<NCH>(cout, p);
        const uint32_t e = __float_as_uint(vE[p]);
        float v = d * d + __uint_as_float(umin3(__float_as_uint(vO[p]), wave_rol1(e), e));
        if (!WODD && kill_o) v = __builtin_inff();
        vO[p] = v;
    }
}

template <int NCH, bool WODD>
__device__ __forceinline__ void diag_round_rot(const int (&qk)[NCH], const int (&ck)[NCH], int off,
                                               const float4 (&cin)[NCH], float4 (&cout)[NCH],
                                               bool kill_e, bool kill_o, float& vE, float& vO) {
    float4 qv[NCH];
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        qv[k] = lds4[qk[k] + off];
        cout[k] = lds4[ck[k] + off + 1];
    }
    diag_steps_rot<NCH, WODD>(qv, cin, cout, kill_e, kill_o, vE, vO);
}

// One wave, groups of G lanes each evaluating one pair.  qb / cb: this
// lane's LDS float4 indices (position offsets already applied, see
// dtw_fwd.hip); chunk k of the query lies LQ float4 further, of the
// candidate LC.
// Runs rounds 0..R-1 (fewer when every group is abandoned) and returns the
// number of rounds run; vE / vO hold the lane's slot values afterwards and
// `aband` is set for lanes of abandoned groups.  Four rounds per iteration
// alternate two candidate buffers, so no point is copied between rounds.
template <typename T, int NCH, bool SAVE, bool WODD, bool ABANDON>
__device__ __forceinline__ int diag_core(int qb, int LQ, int cb, int LC, int R,
                                          int G, int lg, bool kill_e, bool kill_o, T& vE, T& vO,
                                          uint32_t* codes, const Abandon& ab, bool& aband,
                                          uint64_t grp_mask) {
    int qk[NCH];
    int ck[NCH];
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        qk[k] = qb + k * LQ;
        ck[k] = cb + k * LC;
    }
    float4 cA[NCH], cB[NCH];
#pragma unroll
    for (int k = 0; k < NCH; ++k) cA[k] = lds4[ck[k]];
    uint32_t cw = 0;
    float thr = __builtin_inff();
    unsigned long long pend = 0;
    if (ABANDON) {
        thr = abandon_threshold(bsf_from_key(__hip_atomic_load(ab.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)),
                                ab.gamma);
        pend = __hip_atomic_load(ab.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int r = 0;
    for (; r + 4 <= R; r += 4) {
        const int sh = (r & 4) * 4;
        diag_round<T, NCH, SAVE, WODD>(qk, ck, 0, cA, cB, kill_e, kill_o, vE, vO, cw, sh + 0);
        diag_round<T, NCH, SAVE, WODD>(qk, ck, 1, cB, cA, kill_e, kill_o, vE, vO, cw, sh + 4);
        diag_round<T, NCH, SAVE, WODD>(qk, ck, 2, cA, cB, kill_e, kill_o, vE, vO, cw, sh + 8);
        diag_round<T, NCH, SAVE, WODD>(qk, ck, 3, cB, cA, kill_e, kill_o, vE, vO, cw, sh + 12);
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            qk[k] += 4;
            ck[k] += 4;
        }
        if (SAVE && (r & 4)) {
            if (codes) codes[(int64_t)(r >> 3) * G + lg] = cw;
            cw = 0;
        }
        if (ABANDON && ((r + 4) & 15) == 0 && r + 4 < R) {
            // every warping path crosses anti-diagonal 2r+6 or 2r+7 (steps advance i+j by 1 or 2)
            const bool over = (float)vmin(vE, vO) > thr;
            const uint64_t bal = __ballot(over);
            if ((bal & grp_mask) == grp_mask) aband = true;
            if ((bal & ab.valid_mask) == ab.valid_mask) {
                r += 4;
                return __builtin_amdgcn_readfirstlane(r);
            }
            // the key read at the previous check (a best-so-far only decreases)
            thr = abandon_threshold(bsf_from_key(pend), ab.gamma);
            pend = __hip_atomic_load(ab.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    for (; r < R; ++r) {
        diag_round<T, NCH, SAVE, WODD>(qk, ck, 0, cA, cB, kill_e, kill_o, vE, vO, cw, (r & 7) * 4);
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            qk[k] += 1;
            ck[k] += 1;
            cA[k] = cB[k];
        }
        if (SAVE && ((r & 7) == 7 || r == R - 1)) {
            if (codes) codes[(int64_t)(r >> 3) * G + lg] = cw;
            cw = 0;
        }
    }
    if (SAVE && (R & 3) == 0 && (R & 4)) {
        // R = 8k + 4 with no single-round tail: rounds 8k .. 8k+3 are not stored yet
        if (codes) codes[(int64_t)((R - 1) >> 3) * G + lg] = cw;
    }
    return R;
}

// ------------------------------------------------------------- row-systolic
constexpr int kRowPad = 65;   // row-buffer positions left of column 0

// Point t of a series (row-major [len][D]) as NCH float4 chunks; `sentinel`
// in every component outside [0, len), 0 in padded dimensions.
template <int NCH>
__device__ __forceinline__ void load_point(const float* src, int len, int D, int t, float sentinel,
                                           float4 (&out)[NCH]) {
    if (t < 0 || t >= len) {
#pragma unroll
        for (int k = 0; k < NCH; ++k) out[k] = make_float4(sentinel, sentinel, sentinel, sentinel);
        return;
    }
    const float* p = src + (int64_t)t * D;
    if ((D & 3) == 0) {
#pragma unroll
        for (int k = 0; k < NCH; ++k)
            out[k] = (4 * k < D) ? *reinterpret_cast<const float4*>(p + 4 * k) : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (4 * k + e < D) ? p[4 * k + e] : 0.0f;
            out[k] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

// Row-systolic mapping: lane l owns row i0 + l of a block of 64 rows and
// sweeps the block's band columns, lane l reading column jlo - l + t at
// step t; up and diag come from lane l - 1 by a DPP shift (lane 0 from the
// row buffer), left from the lane itself.
//
// LDS at float4 index `ring`: a ring of 128 candidate positions plus 8
// mirrored slots ([k][136] float4, column j at slot (j + 64) mod 128; slots
// 0..7 are repeated at 128..135 so that up to 8 consecutive steps read at
// fixed offsets from one base), and the row buffer (T[n + 2 kRowPad],
// column j at j + kRowPad) holding the last row of the previous block.  At
// step t the wave reads columns jlo + t - 63 .. jlo + t, so 128 positions
// hold everything live: at the start of a block columns jlo - 63 .. jlo + 64
// are loaded, and every 64 steps the next 64 columns (prefetched into
// registers during the previous 64 steps) replace the 64 no lane reads any
// more.  LDS therefore does not grow with the window.  Candidate positions
// outside [0, n) hold -inf, query rows past m hold +inf, so cells outside
// the matrix cost +inf.  Steps run in groups of U (8 / chunks, at least 1):
// the group's candidate points and row-buffer values are read first, then
// the U cells are evaluated, then lane 63 stores its U values.  The last
// block stops at the step that evaluates cell (m-1, n-1).
constexpr int kRowRing = 2 * kRowBlock;
constexpr int kRowMirror = 8;
constexpr int kRowStride = kRowRing + kRowMirror;   // float4 per chunk of a ring

template <int NCH>
__device__ __forceinline__ void ring_put(int ring, int j, const float4 (&v)[NCH]) {
    const int slot = (j + kRowBlock) & (kRowRing - 1);
#pragma unroll
    for (int k = 0; k < NCH; ++k) lds4[ring + slot + k * kRowStride] = v[k];
    if (slot < kRowMirror) {
#pragma unroll
        for (int k = 0; k < NCH; ++k) lds4[ring + kRowRing + slot + k * kRowStride] = v[k];
    }
}

// State of one wave in one row block.
template <typename T, int NCH>
struct RowBlock {
    float4 qv[NCH];
    int i0, jlo, jhi, T_b, T_end;   // T_end: steps actually run (the last block stops at the end cell)
    int k0, cs0, rb, wb;
    T cur, prevup;
    uint32_t cw;
    uint32_t* cp;
};

// Steps [ta, tb) of block B (tb - ta <= 64, no refill in between).
template <typename T, int NCH, bool SAVE>
__device__ __forceinline__ void rows_steps(int ring, const T* rowbuf, T* rowbuf_w, int W, int lane,
                                           RowBlock<T, NCH>& B, int ta, int tb) {
    constexpr int U = NCH >= 8 ? 1 : NCH >= 4 ? 2 : NCH >= 2 ? 4 : 8;
    const T INF = inf_v<T>();
    const unsigned W2 = (unsigned)(2 * W);
    auto step = [&](int t, const float4 (&cv)[NCH], T upin) -> T {
        const T up = wave_shr1(upin, B.cur);
        const T diag = B.prevup;
        B.prevup = up;
        const T left = B.cur;
        const T cost = point_cost<NCH>(B.qv, cv, T(0));
        T best;
        if (SAVE) {
            uint32_t code;
            best = min3_code(diag, up, left, code);
            B.cw |= code << ((t & 15) * 2);
        } else {
            best = vmin3(diag, up, left);
        }
        T v = add_cost(cost, best);
        v = ((unsigned)(t + B.k0) <= W2) ? v : INF;
        B.cur = v;
        return v;
    };
    // A code word (16 steps) is stored once its last step is done, or at the
    // block's last step.  ta is a multiple of 16 (the callers step by 64), so
    // no word ends inside an unrolled group of U steps (U divides 16) and the
    // group's steps run without a branch between them.
    auto store_word = [&](int t_last) __attribute__((always_inline)) {
        B.cp[(int64_t)(t_last >> 4) * kWave] = B.cw;
        B.cw = 0;
    };
    int t = ta;
    for (; t + U <= tb; t += U) {
        const int sb = ring + ((B.cs0 + t) & (kRowRing - 1));
        float4 cv[U][NCH];
        T upv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int k = 0; k < NCH; ++k) cv[u][k] = lds4[sb + u + k * kRowStride];
            upv[u] = rowbuf[B.rb + t + u];
        }
        T out[U];
#pragma unroll
        for (int u = 0; u < U; ++u) out[u] = step(t + u, cv[u], upv[u]);
        if (lane == kRowBlock - 1) {
#pragma unroll
            for (int u = 0; u < U; ++u) rowbuf_w[B.wb + t + u] = out[u];
        }
        if (SAVE && (((t + U) & 15) == 0 || t + U == B.T_end)) store_word(t + U - 1);
    }
    for (; t < tb; ++t) {
        const int sb = ring + ((B.cs0 + t) & (kRowRing - 1));
        float4 cv[NCH];
#pragma unroll
        for (int k = 0; k < NCH; ++k) cv[k] = lds4[sb + k * kRowStride];
        const T v = step(t, cv, rowbuf[B.rb + t]);
        if (lane == kRowBlock - 1) rowbuf_w[B.wb + t] = v;
        if (SAVE && ((t & 15) == 15 || t == B.T_end - 1)) store_word(t);
    }
}

// Sets up block b: query rows into registers, the ring's first 128 columns.
template <typename T, int NCH, bool SAVE>
__device__ __forceinline__ void rows_block_begin(int ring, const T* rowbuf, const float* xs, const float* ys,
                                                 int m, int n, int W, int D, int lane, int b, int nwb,
                                                 uint32_t* codes, RowBlock<T, NCH>& B) {
    const T INF = inf_v<T>();
    B.i0 = b * kRowBlock;
    const int i = B.i0 + lane;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int p = 4 * k + e;
            v[e] = (i < m) ? (p < D ? xs[(int64_t)i * D + p] : 0.0f) : __builtin_inff();
        }
        B.qv[k] = make_float4(v[0], v[1], v[2], v[3]);
    }
    B.jlo = max(0, B.i0 - W);
    B.jhi = min(n - 1, B.i0 + kRowBlock - 1 + W);
    {   // columns jlo - 63 .. jlo + 64
        float4 v0[NCH], v1[NCH];
        load_point<NCH>(ys, n, D, B.jlo - (kRowBlock - 1) + lane, -__builtin_inff(), v0);
        load_point<NCH>(ys, n, D, B.jlo + 1 + lane, -__builtin_inff(), v1);
        ring_put<NCH>(ring, B.jlo - (kRowBlock - 1) + lane, v0);
        ring_put<NCH>(ring, B.jlo + 1 + lane, v1);
    }
    B.T_b = B.jhi - B.jlo + kRowBlock;
    const int nb = (m + kRowBlock - 1) / kRowBlock;
    // the last block stops after lane m-1-i0 has evaluated column n-1
    B.T_end = (b == nb - 1) ? min(B.T_b, (n - 1) - B.jlo + (m - 1 - B.i0) + 1) : B.T_b;
    B.k0 = B.jlo - B.i0 + W - 2 * lane;           // band offset k = t + k0 must lie in [0, 2W]
    B.cs0 = B.jlo - lane + kRowBlock;              // ring slot of step t: (cs0 + t) mod 128
    B.rb = B.jlo + kRowPad;                        // rowbuf index of lane 0's up value: rb + t
    B.wb = B.jlo - (kRowBlock - 1) + kRowPad;      // lane 63 writes rowbuf[wb + t]
    B.cur = INF;
    B.prevup = INF;
    B.cw = 0;
    B.cp = SAVE ? codes + (int64_t)b * nwb * kWave + lane : nullptr;
}

// One wave per pair.  sc: LDS float4 index of the ring; the row buffer follows it.
// Returns the DTW value in the lane (m - 1) mod 64 (others undefined).
template <typename T, int NCH, bool SAVE, bool ABANDON>
__device__ __forceinline__ T rows_core(int sc, const float* xs, const float* ys, int m,
                                       int n, int W, int D, int lane, uint32_t* codes,
                                       const Abandon& ab, bool& aband, int* blocks_done = nullptr) {
    const T INF = inf_v<T>();
    T* rowbuf = reinterpret_cast<T*>(lds4 + sc + kRowStride * NCH);
    const int LB = n + 2 * kRowPad;
    for (int pos = lane; pos < LB; pos += kWave) rowbuf[pos] = (pos - kRowPad == -1) ? T(0) : INF;
    const int nb = (m + kRowBlock - 1) / kRowBlock;
    const int band = min(n, 2 * W + kRowBlock);
    const int nwb = (band + kRowBlock - 1 + 15) / 16;
    T result = INF;
    if (blocks_done) *blocks_done = nb;
    unsigned long long pend = 0;
    for (int b = 0; b < nb; ++b) {
        // the best-so-far for this block's check, loaded a block ahead of its use: the
        // coherent load is slow, and the block's own loads would otherwise wait for it
        if (ABANDON) pend = __hip_atomic_load(ab.key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        RowBlock<T, NCH> B;
        rows_block_begin<T, NCH, SAVE>(sc, rowbuf, xs, ys, m, n, W, D, lane, b, nwb, codes, B);
        __syncthreads();
        if (lane == 0) B.prevup = rowbuf[B.jlo - 1 + kRowPad];
        for (int t0 = 0; t0 < B.T_end; t0 += kRowBlock) {
            const bool refill = t0 + kRowBlock < B.T_end;
            float4 nx[NCH];
            if (refill) load_point<NCH>(ys, n, D, B.jlo + t0 + kRowBlock + 1 + lane, -__builtin_inff(), nx);
            rows_steps<T, NCH, SAVE>(sc, rowbuf, rowbuf, W, lane, B, t0, min(B.T_end, t0 + kRowBlock));
            if (refill) ring_put<NCH>(sc, B.jlo + t0 + kRowBlock + 1 + lane, nx);
        }
        if (b == nb - 1) result = B.cur;
        __syncthreads();
        if (ABANDON && b + 1 < nb) {
            // every path crosses row i0+63: its minimum bounds the final value from below
            const int i0 = B.i0;
            const int r0 = max(0, i0 + kRowBlock - 1 - W), r1 = min(n - 1, i0 + kRowBlock - 1 + W);
            T mn = INF;
            for (int j = r0 + lane; j <= r1; j += kWave) mn = vmin(mn, rowbuf[j + kRowPad]);
            const float thr = abandon_threshold(bsf_from_key(pend), ab.gamma);
            const bool over = (float)mn > thr;
            if (__ballot(over) == ~0ull) {
                aband = true;
                if (blocks_done) *blocks_done = b + 1;
                break;
            }
        }
    }
    return result;
}

// LDS bytes of rows_core for candidate length n (tbytes = sizeof(T)).
__host__ __device__ inline size_t rows_core_lds(int n, int nch, int tbytes) {
    return (size_t)kRowStride * nch * 16 + (size_t)(n + 2 * kRowPad) * tbytes;
}

// Row mapping with K waves per pair (one workgroup of 64 K threads): wave
// v runs row blocks v, v + K, v + 2K, ... of the pair, each exactly as in
// rows_core, with its own candidate ring.  All blocks share one row buffer:
// block b reads row i0 - 1 at column c (lane 0, step c - jlo) and writes
// row i0 + 63 there 63 steps later, and block b + 1 may read column c only
// after block b has written it.  Each wave publishes its progress
// (block * kProgStride + steps done) in LDS after every 64 steps; before a
// chunk of 64 steps a block waits until its predecessor has done the steps
// that write the columns the chunk reads.  A block waits only on the block
// before it, so the chain always ends at block 0 and cannot deadlock; the
// wait is also bounded (kSpinLimit sleeps), after which `late` is set, the
// wave waits no more, and the caller reports the pair as NaN instead of
// hanging.
constexpr int kProgStride = 1 << 20;
constexpr int kSpinLimit = 1 << 17;   // x s_sleep 2 (128 clocks): ~7 ms, several times the longest legitimate wait

template <typename T, int NCH, bool SAVE>
__device__ __forceinline__ T rows_core_pipe(int ring, T* rowbuf, int* prog, int K, int wv,
                                            const float* xs, const float* ys, int m, int n, int W,
                                            int D, int lane, uint32_t* codes, bool& late) {
    const T INF = inf_v<T>();
    const int nb = (m + kRowBlock - 1) / kRowBlock;
    const int band = min(n, 2 * W + kRowBlock);
    const int nwb = (band + kRowBlock - 1 + 15) / 16;
    const int pw = wv == 0 ? K - 1 : wv - 1;   // wave of the previous block
    T result = INF;
    for (int b = wv; b < nb; b += K) {
        RowBlock<T, NCH> B;
        rows_block_begin<T, NCH, SAVE>(ring, rowbuf, xs, ys, m, n, W, D, lane, b, nwb, codes, B);
        // the previous block: its first column and its step count
        const int pjlo = max(0, B.i0 - kRowBlock - W);
        const int pT = b > 0 ? min(n - 1, B.i0 - 1 + W) - pjlo + kRowBlock : 0;
        for (int t0 = 0; t0 < B.T_end; t0 += kRowBlock) {
            if (b > 0 && K > 1 && !late) {
                // columns up to jlo + t0 + 63 are written by the previous block's step
                // (column - pjlo + 63); it must have completed that many steps
                const int need = min(pT, B.jlo - pjlo + t0 + 2 * kRowBlock - 1);
                const int target = (b - 1) * kProgStride + need;
                int spins = 0;
                for (;;) {
                    const int p = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(prog + pw, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
                    if (p >= target) break;
                    if (++spins > kSpinLimit) {
                        late = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            if (t0 == 0 && lane == 0) B.prevup = rowbuf[B.jlo - 1 + kRowPad];
            const bool refill = t0 + kRowBlock < B.T_end;
            float4 nx[NCH];
            if (refill) load_point<NCH>(ys, n, D, B.jlo + t0 + kRowBlock + 1 + lane, -__builtin_inff(), nx);
            const int t1 = min(B.T_end, t0 + kRowBlock);
            rows_steps<T, NCH, SAVE>(ring, rowbuf, rowbuf, W, lane, B, t0, t1);
            if (refill) ring_put<NCH>(ring, B.jlo + t0 + kRowBlock + 1 + lane, nx);
            // this block has completed t1 steps, its row-buffer writes included
            if (K > 1 && lane == 0)
                __hip_atomic_store(prog + wv, b * kProgStride + t1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (b == nb - 1) result = B.cur;
    }
    return result;
}

// LDS bytes of the K-wave row kernel: K rings, the row buffer, K progress
// counters, the work item and a status flag.
__host__ __device__ inline size_t rows_pipe_lds(int n, int nch, int K, int tbytes) {
    const size_t rings = (size_t)K * kRowStride * nch * 16;
    const size_t rowbuf = ((size_t)(n + 2 * kRowPad) * tbytes + 15) & ~(size_t)15;
    return rings + rowbuf + (size_t)(K + 2) * 4;
}

}  // namespace tcdtw
