// C ABI: banded DTW of pairs and its backward.
#include <algorithm>
#include <cstring>

#include "api_common.h"

namespace tcdtw {

// Launch plan for a batch of pairs.
struct PairsPlan {
    bool uniform = false;
    int m = 0, n = 0, W = 0, D = 0, npairs = 0;
    // ragged: work lists by kernel (diagonal, even / odd W) and row-systolic
    std::vector<PairDesc> lists[3];
    int maxm[3] = {0, 0, 0}, maxn[3] = {0, 0, 0}, maxW[3] = {0, 0, 0};
    int64_t saved_words = 0;
    int64_t codes_stride = 0;   // uniform
};

static size_t lds_limit() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 65536;
    return p.sharedMemPerBlock;
}

static tc_dtw_status make_plan(const tc_dtw_batch* xb, const tc_dtw_batch* yb, tc_dtw_window w,
                               PairsPlan& P, HostSet& X, HostSet& Y) {
    tc_dtw_status st;
    if ((st = read_set(xb, "x", X)) != TC_DTW_OK) return st;
    if ((st = read_set(yb, "y", Y)) != TC_DTW_OK) return st;
    if ((st = check_window(w)) != TC_DTW_OK) return st;
    if (X.count != Y.count) return fail(TC_DTW_ERR_INVALID, "x and y must hold the same number of series");
    if (X.dim != Y.dim) return fail(TC_DTW_ERR_INVALID, "x and y must have the same dim");
    P = PairsPlan();
    P.D = X.dim;
    P.npairs = X.count;
    if (X.uniform && Y.uniform) {
        P.uniform = true;
        P.m = X.ulen;
        P.n = Y.ulen;
        P.W = window_eff(P.m, P.n, w);
        P.codes_stride = codes_words(P.m, P.n, P.W);
        P.saved_words = P.codes_stride * P.npairs;
        return TC_DTW_OK;
    }
    int64_t soff = 0;
    for (int b = 0; b < P.npairs; ++b) {
        PairDesc d;
        d.m = X.length(b);
        d.n = Y.length(b);
        d.W = window_eff(d.m, d.n, w);
        d.xoff = X.offset(b);
        d.yoff = Y.offset(b);
        d.out = b;
        d.saved_off = soff;
        soff += codes_words(d.m, d.n, d.W);
        const int k = d.W <= kDiagMaxW ? (d.W & 1) : 2;
        P.lists[k].push_back(d);
        P.maxm[k] = std::max(P.maxm[k], d.m);
        P.maxn[k] = std::max(P.maxn[k], d.n);
        P.maxW[k] = std::max(P.maxW[k], d.W);
    }
    P.saved_words = soff;
    // longest items first: the hardware scheduler then fills the tail with short ones
    for (auto& L : P.lists)
        std::sort(L.begin(), L.end(), [](const PairDesc& a, const PairDesc& b) {
            return (int64_t)a.m * a.W > (int64_t)b.m * b.W;
        });
    return TC_DTW_OK;
}

static size_t plan_ws_bytes(const PairsPlan& P) {
    if (P.uniform) return 0;
    Carve c(nullptr, 0);
    for (auto& L : P.lists) c.take<PairDesc>(L.size());
    return c.need();
}

static tc_dtw_status check_lds(const PairsPlan& P, bool f64) {
    const size_t lim = lds_limit();
    auto fwd_lds = [&](int m, int n, int W, int np) {
        return W <= kDiagMaxW ? diag_lds_bytes(m, n, W, P.D, np) : rows_lds_bytes(n, W, P.D, f64);
    };
    if (P.uniform) {
        const int np = P.W <= kDiagMaxW ? kWave / (P.W + 1) : 1;
        if (fwd_lds(P.m, P.n, P.W, 1) > lim)
            return fail(TC_DTW_ERR_UNSUPPORTED, "series too long for the LDS staging of one pair");
        (void)np;
        return TC_DTW_OK;
    }
    for (int k = 0; k < 3; ++k)
        if (!P.lists[k].empty() && fwd_lds(P.maxm[k], P.maxn[k], P.maxW[k], 1) > lim)
            return fail(TC_DTW_ERR_UNSUPPORTED, "series too long for the LDS staging of one pair");
    return TC_DTW_OK;
}

// Pairs per wave for the uniform diagonal mapping, limited by LDS.
static int pairs_per_wave(const PairsPlan& P) {
    if (P.W > kDiagMaxW) return 1;
    int np = kWave / (P.W + 1);
    const size_t lim = lds_limit();
    while (np > 1 && diag_lds_bytes(P.m, P.n, P.W, P.D, np) > lim) --np;
    return np;
}

}  // namespace tcdtw

using namespace tcdtw;

extern "C" {

size_t tc_dtw_banded_workspace_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y,
                                     tc_dtw_window win, uint32_t flags) {
    (void)flags;
    PairsPlan P;
    HostSet X, Y;
    if (make_plan(x, y, win, P, X, Y) != TC_DTW_OK) return 0;
    return plan_ws_bytes(P);
}

size_t tc_dtw_saved_bytes(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win) {
    PairsPlan P;
    HostSet X, Y;
    if (make_plan(x, y, win, P, X, Y) != TC_DTW_OK) return 0;
    return (size_t)P.saved_words * 4;
}

tc_dtw_status tc_dtw_banded(const tc_dtw_batch* x, const tc_dtw_batch* y, tc_dtw_window win,
                            uint32_t flags, float* dist, void* saved,
                            void* ws, size_t ws_bytes, tc_dtw_stream stream) {
    PairsPlan P;
    HostSet X, Y;
    tc_dtw_status st = make_plan(x, y, win, P, X, Y);
    if (st != TC_DTW_OK) return st;
    if (!dist) return fail(TC_DTW_ERR_INVALID, "null dist pointer");
    if (flags & ~TC_DTW_F64) return fail(TC_DTW_ERR_INVALID, "unknown flag bits");
    const size_t need = plan_ws_bytes(P);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(TC_DTW_ERR_WORKSPACE, "workspace smaller than tc_dtw_banded_workspace_bytes()");
    if ((st = check_device()) != TC_DTW_OK) return st;
    const bool f64 = (flags & TC_DTW_F64) != 0;
    if ((st = check_lds(P, f64)) != TC_DTW_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool save = saved != nullptr;

    DtwFwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.x = X.data;
    a.y = Y.data;
    a.D = P.D;
    a.npairs = P.npairs;
    a.dist = dist;
    a.codes = static_cast<uint32_t*>(saved);
    hipError_t e;
    if (P.uniform) {
        a.uniform = 1;
        a.m = P.m; a.n = P.n; a.W = P.W;
        a.P = pairs_per_wave(P);
        a.wodd = P.W & 1;
        a.codes_stride = P.codes_stride;
        const int items = P.W <= kDiagMaxW ? (P.npairs + a.P - 1) / a.P : P.npairs;
        e = launch_dtw_fwd(a, f64, save, P.W, items, s);
        if (e != hipSuccess) return hip_fail(e, "dtw forward launch");
        return ok();
    }
    Carve c(ws, ws_bytes);
    for (int k = 0; k < 3; ++k) {
        auto& L = P.lists[k];
        if (L.empty()) continue;
        PairDesc* d = c.take<PairDesc>(L.size());
        e = hipMemcpyAsync(d, L.data(), L.size() * sizeof(PairDesc), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
        a.uniform = 0;
        a.desc = d;
        a.m = P.maxm[k]; a.n = P.maxn[k]; a.W = P.maxW[k];
        a.P = 1;
        a.wodd = (k == 1);
        e = launch_dtw_fwd(a, f64, save, P.maxW[k], (int)L.size(), s);
        if (e != hipSuccess) return hip_fail(e, "dtw forward launch");
    }
    return ok();
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
    tc_dtw_status st = make_plan(x, y, win, P, X, Y);
    if (st != TC_DTW_OK) return st;
    if (!saved) return fail(TC_DTW_ERR_INVALID, "null saved pointer");
    if (!grad_dist || !grad_x || !grad_y) return fail(TC_DTW_ERR_INVALID, "null gradient pointer");
    const size_t need = plan_ws_bytes(P);
    if (need > 0 && (!ws || ws_bytes < need))
        return fail(TC_DTW_ERR_WORKSPACE, "workspace smaller than tc_dtw_backward_workspace_bytes()");
    if ((st = check_device()) != TC_DTW_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
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
    hipError_t e;
    if (P.uniform) {
        a.uniform = 1;
        a.m = P.m; a.n = P.n; a.W = P.W;
        a.codes_stride = P.codes_stride;
        e = launch_dtw_bwd(a, P.m, P.n, P.W, P.npairs, s);
        if (e != hipSuccess) return hip_fail(e, "dtw backward launch");
        return ok();
    }
    Carve c(ws, ws_bytes);
    for (int k = 0; k < 3; ++k) {
        auto& L = P.lists[k];
        if (L.empty()) continue;
        PairDesc* d = c.take<PairDesc>(L.size());
        e = hipMemcpyAsync(d, L.data(), L.size() * sizeof(PairDesc), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "descriptor upload");
        a.uniform = 0;
        a.desc = d;
        e = launch_dtw_bwd(a, P.maxm[k], P.maxn[k], P.maxW[k], (int)L.size(), s);
        if (e != hipSuccess) return hip_fail(e, "dtw backward launch");
    }
    return ok();
}

}  // extern "C"
