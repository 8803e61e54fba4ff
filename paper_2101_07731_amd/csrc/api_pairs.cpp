// C ABI: banded DTW of pairs, its backward, and reusable pair plans.
//
// A uniform batch (one length pair, one D, packed densely) is launched
// directly: one block per pair or per P pairs.  Every other batch is
// planned: each pair gets a descriptor (offsets, lengths, W_eff, D, wave
// mapping, offset of its argmin codes), pairs are grouped into classes of
// one mapping and one dimension class, sorted longest first, and each class
// runs as one persistent launch whose waves take pairs from a device
// counter.  tc_dtw_banded / tc_dtw_backward plan into their workspace on
// every call; the tc_dtw_pairs_plan_* calls keep the plan for many runs.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

#include "api_common.h"

namespace tcdtw {

// The diagonal mapping stages both series of a pair in LDS; beyond this
// many bytes a pair runs on the row mapping, whose LDS stays small.
constexpr size_t kDiagLdsBudget = 32768;
constexpr size_t kLdsPerWorkgroup = 163840;   // gfx950: 160 KB of LDS per workgroup
constexpr int kDefaultWavesPerCu = 16;

struct PairClass {
    bool rows = false, wodd = false;
    int nch = 1;
    int K = 1;                // row mapping: waves per pair
    int maxm = 0, maxn = 0, maxW = 0;
    int64_t max_words = 0;
    double work = 0;
    std::vector<PairDesc> items;
};

struct PairsPlan {
    bool uniform = false;
    bool urows = false;       // uniform: row mapping
    int m = 0, n = 0, W = 0, D = 0, npairs = 0;
    int waves_per_cu = kDefaultWavesPerCu;
    int waves_per_pair = 8;
    std::vector<PairClass> classes;
    int64_t saved_words = 0;
    int64_t codes_stride = 0;   // uniform
};

// LDS per block of the current device, queried once per device (runs may
// be captured in a graph, so they make no property queries).
static size_t lds_limit() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    static std::mutex mu;
    static std::map<int, size_t> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    hipDeviceProp_t p;
    const size_t v = hipGetDeviceProperties(&p, dev) == hipSuccess ? p.sharedMemPerBlock : 65536;
    cache[dev] = v;
    return v;
}

static bool use_rows(int m, int n, int W, int D, int diag_max) {
    return W > diag_max || diag_lds_bytes(m, n, W, D, 1) > kDiagLdsBudget;
}

// Steps x lane-operations of one wave running a pair on the row mapping:
// its 64-row blocks each sweep the block's band columns plus 63.
static double rows_wave_cost(int m, int n, int W, int D) {
    const int nb = (m + kRowBlock - 1) / kRowBlock;
    double steps = 0;
    for (int b = 0; b < nb; ++b) {
        const int i0 = b * kRowBlock;
        steps += std::min(n - 1, i0 + kRowBlock - 1 + W) - std::max(0, i0 - W) + kRowBlock;
    }
    return steps * (2.0 * D + 14.0);
}

// Waves sharing a pair on the row mapping.  One wave per pair keeps every
// wave busy (waiting waves of a pipelined pair cost throughput), but a pair
// whose single-wave time exceeds the time the whole batch needs would be
// the critical path: it gets K = that ratio, rounded up to 2, 4 or 8,
// capped by the tuning and by LDS (sized for a float64 row buffer).  The
// batch time is estimated as its work spread over 256 wave slots (the
// 1024 SIMDs at the quarter of peak issue that row kernels reach with
// mixed shapes).  A pair of at most two row blocks has nothing to pipeline.
static int waves_for(int m, int n, int W, int D, double spread, int cap) {
    const int nb = (m + kRowBlock - 1) / kRowBlock;
    if (nb <= 2 || spread <= 0) return 1;
    const double ratio = rows_wave_cost(m, n, W, D) / spread;
    int K = ratio <= 1.0 ? 1 : ratio <= 2.0 ? 2 : ratio <= 4.0 ? 4 : 8;
    K = std::min(K, cap);
    while (K > 1 && pipe_lds_bytes(n, D, K, true) > 163840) K /= 2;
    return std::max(K, 1);
}

// force_plan: plan even a uniform batch (the reusable plans always do).
static tc_dtw_status make_plan(const tc_dtw_batch* xb, const tc_dtw_batch* yb, tc_dtw_window w,
                               const tc_dtw_tuning* tune, bool force_plan, PairsPlan& P, HostSet& X,
                               HostSet& Y) {
    tc_dtw_status st;
    if ((st = read_set(xb, "x", X)) != TC_DTW_OK) return st;
    if ((st = read_set(yb, "y", Y)) != TC_DTW_OK) return st;
    if ((st = check_window(w)) != TC_DTW_OK) return st;
    if (X.count != Y.count) return fail(TC_DTW_ERR_INVALID, "x and y must hold the same number of series");
    for (int b = 0; b < X.count; ++b)
        if (X.dimension(b) != Y.dimension(b))
            return fail(TC_DTW_ERR_INVALID, "x and y must have the same dim in every pair");
    int diag_max = kDiagMaxW;
    P = PairsPlan();
    if (tune) {
        if (tune->diag_max_w < -1 || tune->diag_max_w > kDiagMaxW)
            return fail(TC_DTW_ERR_INVALID, "tuning.diag_max_w must lie in -1..63");
        if (tune->waves_per_cu < 0 || tune->waves_per_cu > 32)
            return fail(TC_DTW_ERR_INVALID, "tuning.waves_per_cu must lie in 0..32");
        const int wp = tune->waves_per_pair;
        if (wp != 0 && wp != 1 && wp != 2 && wp != 4 && wp != 8)
            return fail(TC_DTW_ERR_INVALID, "tuning.waves_per_pair must be 0, 1, 2, 4 or 8");
        diag_max = tune->diag_max_w;
        if (tune->waves_per_cu > 0) P.waves_per_cu = tune->waves_per_cu;
        if (wp > 0) P.waves_per_pair = wp;
    }
    P.D = X.dim;
    P.npairs = X.count;
    if (X.uniform && Y.uniform && !force_plan) {
        P.uniform = true;
        P.m = X.ulen;
        P.n = Y.ulen;
        P.W = window_eff(P.m, P.n, w);
        P.urows = use_rows(P.m, P.n, P.W, P.D, diag_max);
        // a batch too small to fill the chip with one wave per pair runs the cooperative
        // diagonal kernel (float32), whose time is the serial chain, not occupancy: it keeps
        // the diagonal mapping wherever its LDS fits (the codes layout follows the mapping)
        if (P.urows && P.W <= diag_max && P.npairs <= kCoopMaxItems &&
            diag_coop_lds_bytes(P.m, P.n, P.W, P.D, 1) <= kLdsPerWorkgroup)
            P.urows = false;
        P.codes_stride = codes_words(P.m, P.n, P.W, P.urows);
        P.saved_words = P.codes_stride * P.npairs;
        return TC_DTW_OK;
    }
    // the batch's row-mapping work spread over the chip's SIMDs
    double spread = 0;
    for (int b = 0; b < P.npairs; ++b) {
        const int m = X.length(b), n = Y.length(b), W = window_eff(m, n, w), D = X.dimension(b);
        if (use_rows(m, n, W, D, diag_max)) spread += rows_wave_cost(m, n, W, 4 * nch_pad(D));
    }
    spread /= 256.0;
    // class key: mapping kind (diag even, diag odd, rows) x dimension class x waves per pair
    int index[3][17][9];
    for (auto& r : index)
        for (auto& q : r) std::fill(q, q + 9, -1);
    int64_t soff = 0;
    for (int b = 0; b < P.npairs; ++b) {
        PairDesc d;
        std::memset(&d, 0, sizeof d);
        d.m = X.length(b);
        d.n = Y.length(b);
        d.W = window_eff(d.m, d.n, w);
        d.D = X.dimension(b);
        d.rows = use_rows(d.m, d.n, d.W, d.D, diag_max) ? 1 : 0;
        d.xoff = X.offset(b);
        d.yoff = Y.offset(b);
        d.out = b;
        d.saved_off = soff;
        const int64_t words = codes_words(d.m, d.n, d.W, d.rows != 0);
        soff += words;
        const int kind = d.rows ? 2 : (d.W & 1);
        const int nch = nch_pad(d.D);
        const int K = d.rows ? waves_for(d.m, d.n, d.W, 4 * nch, spread, P.waves_per_pair) : 1;
        int& ci = index[kind][nch][K];
        if (ci < 0) {
            if ((int)P.classes.size() == TC_DTW_PLAN_MAX_CLASSES)
                return fail(TC_DTW_ERR_UNSUPPORTED, "too many pair classes");
            ci = (int)P.classes.size();
            P.classes.emplace_back();
            P.classes.back().rows = d.rows != 0;
            P.classes.back().wodd = kind == 1;
            P.classes.back().nch = nch;
            P.classes.back().K = K;
        }
        PairClass& c = P.classes[ci];
        c.maxm = std::max(c.maxm, d.m);
        c.maxn = std::max(c.maxn, d.n);
        c.maxW = std::max(c.maxW, d.W);
        c.max_words = std::max(c.max_words, words);
        c.work += (double)band_cells(d.m, d.n, d.W) * (2.0 * d.D + 2.0);
        c.items.push_back(d);
    }
    P.saved_words = soff;
    // longest pairs (most band cells) first inside a class, heaviest class first
    for (auto& c : P.classes) {
        std::vector<std::pair<int64_t, int>> key(c.items.size());
        for (size_t k = 0; k < c.items.size(); ++k)
            key[k] = {band_cells(c.items[k].m, c.items[k].n, c.items[k].W), (int)k};
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<int64_t, int>& a, const std::pair<int64_t, int>& b) {
                             return a.first > b.first;
                         });
        std::vector<PairDesc> sorted(c.items.size());
        for (size_t k = 0; k < key.size(); ++k) sorted[k] = c.items[key[k].second];
        c.items.swap(sorted);
    }
    std::stable_sort(P.classes.begin(), P.classes.end(),
                     [](const PairClass& a, const PairClass& b) { return a.work > b.work; });
    return TC_DTW_OK;
}

// Plan buffer: class counters, then each class's descriptors.
static size_t plan_layout(const PairsPlan& P, std::vector<size_t>* desc_off) {
    if (P.uniform) return 0;
    Carve c(nullptr, 0);
    c.take<int32_t>(TC_DTW_PLAN_MAX_CLASSES);
    for (auto& cl : P.classes) {
        c.used = (c.used + 255) & ~(size_t)255;
        if (desc_off) desc_off->push_back(c.used);
        c.used += cl.items.size() * sizeof(PairDesc);
    }
    return c.need();
}

static void to_public(const PairsPlan& P, const std::vector<size_t>& off, void* buf, size_t bytes,
                      tc_dtw_pairs_plan* out) {
    std::memset(out, 0, sizeof *out);
    out->buf = buf;
    out->bytes = bytes;
    out->npairs = P.npairs;
    out->nclasses = (int32_t)P.classes.size();
    out->waves_per_cu = P.waves_per_cu;
    out->saved_bytes = P.saved_words * 4;
    for (size_t k = 0; k < P.classes.size(); ++k) {
        const PairClass& c = P.classes[k];
        tc_dtw_plan_class& o = out->cls[k];
        o.rows = c.rows;
        o.wodd = c.wodd;
        o.dim = 4 * c.nch;
        o.nitems = (int32_t)c.items.size();
        o.maxm = c.maxm;
        o.maxn = c.maxn;
        o.maxw = c.maxW;
        o.waves_per_pair = c.K;
        o.max_words = c.max_words;
        o.desc_off = (int64_t)off[k];
        o.work = c.work;
    }
    // classes to streams, heaviest first onto the least loaded stream
    double load[TC_DTW_RUN_STREAMS] = {0};
    for (size_t k = 0; k < P.classes.size(); ++k) {
        int best = 0;
        for (int i = 1; i < TC_DTW_RUN_STREAMS; ++i)
            if (load[i] < load[best]) best = i;
        out->cls[k].stream = best;
        load[best] += P.classes[k].work;
    }
}

// The streams a run forks to, created once per device, with the events of
// the fork and the join.  One run at a time enqueues on them (mutex); the
// work itself overlaps freely.
struct RunStreams {
    hipStream_t s[TC_DTW_RUN_STREAMS];
    hipEvent_t fork;
    hipEvent_t done[TC_DTW_RUN_STREAMS];
    std::mutex mu;
};

static RunStreams* run_streams(hipError_t& err) {
    int dev = 0;
    err = hipGetDevice(&dev);
    if (err != hipSuccess) return nullptr;
    static std::mutex mu;
    static std::map<int, RunStreams*> pools;
    std::lock_guard<std::mutex> lk(mu);
    auto it = pools.find(dev);
    if (it != pools.end()) return it->second;
    RunStreams* r = new RunStreams();
    for (int i = 0; i < TC_DTW_RUN_STREAMS && err == hipSuccess; ++i)
        err = hipStreamCreateWithFlags(&r->s[i], hipStreamNonBlocking);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&r->fork, hipEventDisableTiming);
    for (int i = 0; i < TC_DTW_RUN_STREAMS && err == hipSuccess; ++i)
        err = hipEventCreateWithFlags(&r->done[i], hipEventDisableTiming);
    if (err != hipSuccess) return nullptr;   // kept nothing: the next call tries again
    pools[dev] = r;
    return r;
}

// Fork: the library streams wait for everything enqueued on `s` so far.
static hipError_t fork_from(RunStreams* r, hipStream_t s) {
    hipError_t e = hipEventRecord(r->fork, s);
    for (int i = 0; i < TC_DTW_RUN_STREAMS && e == hipSuccess; ++i) e = hipStreamWaitEvent(r->s[i], r->fork, 0);
    return e;
}

// Join: `s` waits for everything the run put on the library streams.
static hipError_t join_into(RunStreams* r, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int i = 0; i < TC_DTW_RUN_STREAMS && e == hipSuccess; ++i) {
        e = hipEventRecord(r->done[i], r->s[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, r->done[i], 0);
    }
    return e;
}

static tc_dtw_status upload(const PairsPlan& P, const std::vector<size_t>& off, void* buf, hipStream_t s) {
    char* base = static_cast<char*>(buf);
    for (size_t k = 0; k < P.classes.size(); ++k) {
        const auto& L = P.classes[k].items;
        const hipError_t e =
            hipMemcpyAsync(base + off[k], L.data(), L.size() * sizeof(PairDesc), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    }
    return TC_DTW_OK;
}

static int persistent_grid(size_t lds, int waves_per_cu, int nitems) {
    const size_t lim = 163840;
    const int by_lds = (int)std::max<size_t>(1, lim / std::max<size_t>(lds, 1));
    const int per_cu = std::max(1, std::min(waves_per_cu, by_lds));
    return std::max(1, std::min(nitems, 256 * per_cu));
}

static tc_dtw_status check_plan(const tc_dtw_pairs_plan* p) {
    if (!p || !p->buf) return fail(TC_DTW_ERR_INVALID, "null plan");
    if (p->nclasses < 0 || p->nclasses > TC_DTW_PLAN_MAX_CLASSES)
        return fail(TC_DTW_ERR_INVALID, "corrupt plan");
    return TC_DTW_OK;
}

// With `fork` the classes run concurrently on the library's streams (forked
// from and joined back into s0); without it every class runs on s0 in turn,
// and the call creates no streams or events.
static tc_dtw_status run_fwd(const tc_dtw_pairs_plan* p, const float* x, const float* y, uint32_t flags,
                             float* dist, void* saved, hipStream_t s0, bool fork = true) {
    const bool f64 = (flags & TC_DTW_F64) != 0;
    char* base = static_cast<char*>(p->buf);
    int32_t* counters = reinterpret_cast<int32_t*>(base);
    hipError_t e = launch_zero_i32(counters, TC_DTW_PLAN_MAX_CLASSES, s0);
    if (e != hipSuccess) return hip_fail(e, "counter reset");
    const size_t lim = lds_limit();
    RunStreams* rs = nullptr;
    std::unique_lock<std::mutex> lk;
    if (fork) {
        rs = run_streams(e);
        if (!rs) return hip_fail(e, "run streams");
        lk = std::unique_lock<std::mutex>(rs->mu);
        if ((e = fork_from(rs, s0)) != hipSuccess) return hip_fail(e, "stream fork");
    }
    auto join = [&]() { return rs ? join_into(rs, s0) : hipSuccess; };
    for (int k = 0; k < p->nclasses; ++k) {
        hipStream_t s = rs ? rs->s[p->cls[k].stream % TC_DTW_RUN_STREAMS] : s0;
        const tc_dtw_plan_class& c = p->cls[k];
        DtwFwdArgs a;
        std::memset(&a, 0, sizeof a);
        a.x = x;
        a.y = y;
        a.desc = reinterpret_cast<const PairDesc*>(base + c.desc_off);
        a.uniform = 0;
        a.m = c.maxm; a.n = c.maxn; a.W = c.maxw; a.D = c.dim;
        a.P = 1;
        a.wodd = c.wodd;
        a.npairs = p->npairs;
        a.dist = dist;
        a.codes = static_cast<uint32_t*>(saved);
        a.counter = counters + k;
        a.status = status_word();
        const int K = c.rows ? c.waves_per_pair : 1;
        if (K > 1) {
            const size_t lds = pipe_lds_bytes(c.maxn, c.dim, K, f64);
            if (lds > lim) { (void)join(); return fail(TC_DTW_ERR_UNSUPPORTED, "series too long for the LDS staging of one pair"); }
            const int per_cu = std::max(1, std::min(p->waves_per_cu / K, (int)(lim / lds)));
            const int grid = std::max(1, std::min(c.nitems, 256 * per_cu));
            e = launch_dtw_rows_pipe(a, f64, saved != nullptr, K, c.nitems, grid, s);
        } else {
            const size_t lds = fwd_lds_bytes(a, c.rows != 0, f64);
            if (lds > lim) { (void)join(); return fail(TC_DTW_ERR_UNSUPPORTED, "series too long for the LDS staging of one pair"); }
            e = launch_dtw_fwd(a, f64, saved != nullptr, c.rows != 0, c.nitems,
                               persistent_grid(lds, p->waves_per_cu, c.nitems), s);
        }
        if (e != hipSuccess) { (void)join(); return hip_fail(e, "dtw forward launch"); }
    }
    if ((e = join()) != hipSuccess) return hip_fail(e, "stream join");
    return ok();
}

static tc_dtw_status run_bwd(const tc_dtw_pairs_plan* p, const float* x, const float* y, const void* saved,
                             const float* grad_dist, float* grad_x, float* grad_y, hipStream_t s0) {
    char* base = static_cast<char*>(p->buf);
    int32_t* counters = reinterpret_cast<int32_t*>(base);
    hipError_t e = launch_zero_i32(counters, TC_DTW_PLAN_MAX_CLASSES, s0);
    if (e != hipSuccess) return hip_fail(e, "counter reset");
    const size_t lim = lds_limit();
    RunStreams* rs = run_streams(e);
    if (!rs) return hip_fail(e, "run streams");
    std::lock_guard<std::mutex> lk(rs->mu);
    if ((e = fork_from(rs, s0)) != hipSuccess) return hip_fail(e, "stream fork");
    for (int k = 0; k < p->nclasses; ++k) {
        hipStream_t s = rs->s[p->cls[k].stream % TC_DTW_RUN_STREAMS];
        const tc_dtw_plan_class& c = p->cls[k];
        DtwBwdArgs a;
        std::memset(&a, 0, sizeof a);
        a.x = x;
        a.y = y;
        a.desc = reinterpret_cast<const PairDesc*>(base + c.desc_off);
        a.uniform = 0;
        a.npairs = p->npairs;
        a.codes = static_cast<const uint32_t*>(saved);
        a.grad_dist = grad_dist;
        a.grad_x = grad_x;
        a.grad_y = grad_y;
        a.counter = counters + k;
        const size_t lds = bwd_lds_bytes(c.maxm, c.maxn, c.max_words, c.dim);
        if (lds > lim) { (void)join_into(rs, s0); return fail(TC_DTW_ERR_UNSUPPORTED, "series too long for the backward's LDS"); }
        e = launch_dtw_bwd(a, c.maxm, c.maxn, c.max_words, c.dim, c.nitems,
                           persistent_grid(lds, p->waves_per_cu, c.nitems), s);
        if (e != hipSuccess) { (void)join_into(rs, s0); return hip_fail(e, "dtw backward launch"); }
    }
    if ((e = join_into(rs, s0)) != hipSuccess) return hip_fail(e, "stream join");
    return ok();
}

// Pairs per wave for the uniform diagonal mapping, limited by LDS.
static int pairs_per_wave(const PairsPlan& P) {
    if (P.urows) return 1;
    int np = kWave / (P.W + 1);
    const size_t lim = lds_limit();
    while (np > 1 && diag_lds_bytes(P.m, P.n, P.W, P.D, np) > lim) --np;
    return np;
}

// The direct calls plan into their workspace on every call.
static tc_dtw_status plan_in_workspace(const PairsPlan& P, void* ws, size_t ws_bytes, hipStream_t s,
                                       tc_dtw_pairs_plan& out) {
    std::vector<size_t> off;
    const size_t need = plan_layout(P, &off);
    if (!ws || ws_bytes < need)
        return fail(TC_DTW_ERR_WORKSPACE, "workspace smaller than its *_workspace_bytes() query");
    to_public(P, off, ws, ws_bytes, &out);
    return upload(P, off, ws, s);
}

// The direct call (declared in api_common.h).  `buffer` runs after the
// host-side checks and before any HIP call of this function.
tc_dtw_status banded_direct(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win, uint32_t flags,
                            float* dist, void* saved, void* ws, size_t ws_bytes, bool fork,
                            tc_dtw_status (*buffer)(size_t need, void* ctx, void** buf, size_t* bytes),
                            void* ctx, hipStream_t s) {
    PairsPlan P;
    HostSet X, Y;
    tc_dtw_status st = make_plan(x, y, win, nullptr, false, P, X, Y);
    if (st != TC_DTW_OK) return st;
    if (!dist) return fail(TC_DTW_ERR_INVALID, "null dist pointer");
    if (flags & ~TC_DTW_F64) return fail(TC_DTW_ERR_INVALID, "unknown flag bits");
    const size_t need = plan_layout(P, nullptr);
    if (buffer && (st = buffer(need, ctx, &ws, &ws_bytes)) != TC_DTW_OK) return st;
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(TC_DTW_ERR_WORKSPACE, "workspace smaller than tc_dtw_banded_workspace_bytes()");
    if ((st = check_device()) != TC_DTW_OK) return st;
    const bool f64 = (flags & TC_DTW_F64) != 0;
    if (!P.uniform) {
        tc_dtw_pairs_plan pl;
        if ((st = plan_in_workspace(P, ws, ws_bytes, s, pl)) != TC_DTW_OK) return st;
        return run_fwd(&pl, X.data, Y.data, flags, dist, saved, s, fork);
    }
    DtwFwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.x = X.data;
    a.y = Y.data;
    a.D = P.D;
    a.npairs = P.npairs;
    a.dist = dist;
    a.codes = static_cast<uint32_t*>(saved);
    a.uniform = 1;
    a.m = P.m; a.n = P.n; a.W = P.W;
    a.P = pairs_per_wave(P);
    a.wodd = P.W & 1;
    a.codes_stride = P.codes_stride;
    if (fwd_lds_bytes(a, P.urows, f64) > lds_limit())
        return fail(TC_DTW_ERR_UNSUPPORTED, "series too long for the LDS staging of one pair");
    const int items = P.urows ? P.npairs : (P.npairs + a.P - 1) / a.P;
    if (!f64 && !P.urows && items <= kCoopMaxItems) {
        // too few items to fill the chip with one wave each: the serial chain of the recurrence
        // sets the time, so three more waves per item form the point costs ahead of it
        DtwFwdArgs c = a;
        while (c.P > 1 && diag_coop_lds_bytes(P.m, P.n, P.W, P.D, c.P) > lds_limit()) --c.P;
        if (diag_coop_lds_bytes(P.m, P.n, P.W, P.D, c.P) <= lds_limit()) {
            const hipError_t e = launch_dtw_diag_coop(c, saved != nullptr, (P.npairs + c.P - 1) / c.P, s);
            if (e != hipSuccess) return hip_fail(e, "dtw forward launch");
            return ok();
        }
    }
    const hipError_t e = launch_dtw_fwd(a, f64, saved != nullptr, P.urows, items, 0, s);
    if (e != hipSuccess) return hip_fail(e, "dtw forward launch");
    return ok();
}


}  // namespace tcdtw

using namespace tcdtw;

extern "C" {

size_t tc_dtw_banded_workspace_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y,
                                     tc_dtw_window win, uint32_t flags) {
    (void)flags;
    PairsPlan P;
    HostSet X, Y;
    if (make_plan(x, y, win, nullptr, false, P, X, Y) != TC_DTW_OK) return 0;
    return plan_layout(P, nullptr);
}

size_t tc_dtw_saved_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win) {
    PairsPlan P;
    HostSet X, Y;
    if (make_plan(x, y, win, nullptr, false, P, X, Y) != TC_DTW_OK) return 0;
    return (size_t)P.saved_words * 4;
}

tc_dtw_status tc_dtw_banded(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                            uint32_t flags, float* dist, void* saved,
                            void* ws, size_t ws_bytes, tc_dtw_stream stream) {
    return banded_direct(x, y, win, flags, dist, saved, ws, ws_bytes, true, nullptr, nullptr,
                         reinterpret_cast<hipStream_t>(stream));
}

size_t tc_dtw_backward_workspace_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y,
                                       tc_dtw_window win) {
    return tc_dtw_banded_workspace_bytes(x, y, win, 0);
}

tc_dtw_status tc_dtw_backward(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                              const void* saved, const float* grad_dist,
                              float* grad_x, float* grad_y,
                              void* ws, size_t ws_bytes, tc_dtw_stream stream) {
    PairsPlan P;
    HostSet X, Y;
    tc_dtw_status st = make_plan(x, y, win, nullptr, false, P, X, Y);
    if (st != TC_DTW_OK) return st;
    if (!saved) return fail(TC_DTW_ERR_INVALID, "null saved pointer");
    if (!grad_dist || !grad_x || !grad_y) return fail(TC_DTW_ERR_INVALID, "null gradient pointer");
    const size_t need = plan_layout(P, nullptr);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(TC_DTW_ERR_WORKSPACE, "workspace smaller than tc_dtw_backward_workspace_bytes()");
    if ((st = check_device()) != TC_DTW_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!P.uniform) {
        tc_dtw_pairs_plan pl;
        if ((st = plan_in_workspace(P, ws, ws_bytes, s, pl)) != TC_DTW_OK) return st;
        return run_bwd(&pl, X.data, Y.data, saved, grad_dist, grad_x, grad_y, s);
    }
    DtwBwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.x = X.data;
    a.y = Y.data;
    a.D = P.D;
    a.npairs = P.npairs;
    a.codes = static_cast<const uint32_t*>(saved);
    a.grad_dist = grad_dist;
    a.grad_x = grad_x;
    a.grad_y = grad_y;
    a.uniform = 1;
    a.urows = P.urows ? 1 : 0;
    a.m = P.m; a.n = P.n; a.W = P.W;
    a.codes_stride = P.codes_stride;
    if (bwd_lds_bytes(P.m, P.n, P.codes_stride, P.D) > lds_limit())
        return fail(TC_DTW_ERR_UNSUPPORTED, "series too long for the backward's LDS");
    const hipError_t e = launch_dtw_bwd(a, P.m, P.n, P.codes_stride, P.D, P.npairs, 0, s);
    if (e != hipSuccess) return hip_fail(e, "dtw backward launch");
    return ok();
}

size_t tc_dtw_pairs_plan_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                               const tc_dtw_tuning* tune) {
    PairsPlan P;
    HostSet X, Y;
    if (make_plan(x, y, win, tune, true, P, X, Y) != TC_DTW_OK) return 0;
    return plan_layout(P, nullptr);
}

tc_dtw_status tc_dtw_pairs_plan_build(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                                      const tc_dtw_tuning* tune, void* buf, size_t bytes,
                                      tc_dtw_pairs_plan* plan, tc_dtw_stream stream) {
    PairsPlan P;
    HostSet X, Y;
    tc_dtw_status st = make_plan(x, y, win, tune, true, P, X, Y);
    if (st != TC_DTW_OK) return st;
    if (!plan) return fail(TC_DTW_ERR_INVALID, "null plan");
    if ((st = check_device()) != TC_DTW_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((st = plan_in_workspace(P, buf, bytes, s, *plan)) != TC_DTW_OK) return st;
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    return ok();
}

tc_dtw_status tc_dtw_banded_run(const tc_dtw_pairs_plan* plan, const float* x, const float* y,
                                uint32_t flags, float* dist, void* saved, tc_dtw_stream stream) {
    tc_dtw_status st = check_plan(plan);
    if (st != TC_DTW_OK) return st;
    if (!x || !y || !dist) return fail(TC_DTW_ERR_INVALID, "null x, y or dist pointer");
    if (flags & ~TC_DTW_F64) return fail(TC_DTW_ERR_INVALID, "unknown flag bits");
    if ((st = check_device()) != TC_DTW_OK) return st;
    return run_fwd(plan, x, y, flags, dist, saved, reinterpret_cast<hipStream_t>(stream));
}

tc_dtw_status tc_dtw_backward_run(const tc_dtw_pairs_plan* plan, const float* x, const float* y,
                                  const void* saved, const float* grad_dist, float* grad_x,
                                  float* grad_y, tc_dtw_stream stream) {
    tc_dtw_status st = check_plan(plan);
    if (st != TC_DTW_OK) return st;
    if (!x || !y || !saved || !grad_dist || !grad_x || !grad_y)
        return fail(TC_DTW_ERR_INVALID, "null pointer argument");
    if ((st = check_device()) != TC_DTW_OK) return st;
    return run_bwd(plan, x, y, saved, grad_dist, grad_x, grad_y, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
