// C ABI: candidate index, dense lower bounds and the 1-NN search.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "api_common.h"

namespace tcdtw {

static const double kUnit = 1.0 / 16777216.0;   // float32 unit roundoff 2^-24

// Section layout of an index buffer.
struct IndexLayout {
    bool uniform;
    int count, dim, ulen, maxlen, ntiles;
    int64_t total_len;
    size_t off_series, off_tiles, off_gamma, off_meta, off_range, off_dims, bytes;
};

static IndexLayout index_layout(const HostSet& R) {
    IndexLayout L;
    L.uniform = R.uniform;
    L.count = R.count;
    L.dim = R.dim;
    L.ulen = R.uniform ? R.ulen : 0;
    L.maxlen = R.maxlen;
    L.total_len = 0;
    int64_t elems = 0;
    for (int s = 0; s < R.count; ++s) {
        L.total_len += R.length(s);
        elems += (int64_t)R.length(s) * R.dimension(s);
    }
    L.ntiles = R.uniform ? (R.count + 63) / 64 : 0;
    Carve c(nullptr, 0);
    auto at = [&](size_t bytes) { c.used = (c.used + 255) & ~(size_t)255; size_t o = c.used; c.used += bytes; return o; };
    L.off_series = at((size_t)elems * 4);
    L.off_tiles = at(R.uniform ? (size_t)L.ntiles * (((size_t)R.ulen * R.dim + 3) / 4 * 4) * 64 * 4 : 0);
    L.off_gamma = at((size_t)L.total_len * 4);
    L.off_meta = at((size_t)R.count * (8 + 8 + 4 + 8) + 8);
    L.off_range = at(8);
    L.off_dims = at(R.mixed ? (size_t)R.count * 4 : 0);
    L.bytes = c.need();
    return L;
}

// Banks of an index with per-series dims: maximal runs of equal D, each D in one run.
static tc_dtw_status index_banks(const HostSet& R, tc_dtw_index& out) {
    out.nbanks = 0;
    if (!R.mixed) return TC_DTW_OK;
    int s = 0;
    while (s < R.count) {
        const int D = R.dimension(s);
        int e = s;
        while (e < R.count && R.dimension(e) == D) ++e;
        for (int b = 0; b < out.nbanks; ++b)
            if (out.bank_dim[b] == D)
                return fail(TC_DTW_ERR_UNSUPPORTED, "references of one dimension must form one contiguous run");
        if (out.nbanks == TC_DTW_MAX_BANKS)
            return fail(TC_DTW_ERR_UNSUPPORTED, "an index holds at most TC_DTW_MAX_BANKS banks");
        out.bank_dim[out.nbanks] = D;
        out.bank_first[out.nbanks] = s;
        out.bank_count[out.nbanks] = e - s;
        ++out.nbanks;
        s = e;
    }
    return TC_DTW_OK;
}

static tc_dtw_status check_index(const tc_dtw_index* ix) {
    if (!ix || !ix->buf) return fail(TC_DTW_ERR_INVALID, "null index");
    if (ix->count < 1 || ix->dim < 1 || ix->dim > 64) return fail(TC_DTW_ERR_INVALID, "index not built");
    return TC_DTW_OK;
}

static tc_dtw_status check_params(const tc_dtw_knn_params* p) {
    if (!p) return fail(TC_DTW_ERR_INVALID, "null params");
    tc_dtw_status st = check_window(p->window);
    if (st != TC_DTW_OK) return st;
    if (p->k < 1) return fail(TC_DTW_ERR_INVALID, "k must be >= 1");
    if (p->k > kMaxK) return fail(TC_DTW_ERR_UNSUPPORTED, "k is limited to 32");
    if (p->independent != 0 && p->independent != 1) return fail(TC_DTW_ERR_INVALID, "independent must be 0 or 1");
    if (p->reuse_query_meta != 0 && p->reuse_query_meta != 1)
        return fail(TC_DTW_ERR_INVALID, "reuse_query_meta must be 0 or 1");
    if (p->independent && (p->bounds & (TC_DTW_LB_PC | TC_DTW_LB_TI)))
        return fail(TC_DTW_ERR_UNSUPPORTED, "LB_PC and LB_TI bound the dependent DTW only (independent DTW: LB_MV)");
    if (p->bounds & ~(TC_DTW_LB_MV | TC_DTW_LB_PC | TC_DTW_LB_TI))
        return fail(TC_DTW_ERR_INVALID, "unknown bound bits");
    if ((p->bounds & (TC_DTW_LB_PC | TC_DTW_LB_TI)) && !(p->bounds & TC_DTW_LB_MV))
        return fail(TC_DTW_ERR_INVALID, "LB_PC and LB_TI are deployed behind LB_MV (set TC_DTW_LB_MV)");
    if (p->pc_levels < 2 || p->pc_clusters < 1 || p->pc_group < 1)
        return fail(TC_DTW_ERR_INVALID, "LB_PC needs levels >= 2, clusters >= 1, group >= 1");
    if (!(p->prune_margin >= 0.0f) || !(p->trigger_ti >= 0.0f) || !(p->trigger_pc >= 0.0f))
        return fail(TC_DTW_ERR_INVALID, "margins and triggers must be >= 0");
    if (p->seed_r < 0) return fail(TC_DTW_ERR_INVALID, "seed_r must be >= 0");
    return TC_DTW_OK;
}

// Everything a uniform search needs, with workspace offsets.
struct KnnPlan {
    int nq, nc, m, n, D, W, R, P, cap, ntiles, k;
    bool indep;
    bool plain, abandon, gate, pc, ti;
    bool cand;              // LB_PC against candidate-side boxes (params.pc_cand)
    int ngroups, max_pts;
    size_t o_env, o_lb, o_seeds, o_seed_dist, o_list, o_list_dist, o_cnt, o_glist, o_gcnt, o_prefix,
        o_items, o_counters, o_key, o_stats, o_boxes, o_nbox, o_qstep, o_glb, o_tlist, o_tlb, o_tout,
        o_tcnt, o_ppc, o_pti, o_cntmv, o_part, o_topk, bytes;
    int nseg = 1;
};



static tc_dtw_status make_knn_plan(const tc_dtw_index* ix, const tc_dtw_batch* qb, const tc_dtw_knn_params* p,
                                   KnnPlan& K, HostSet& Qs) {
    tc_dtw_status st;
    if ((st = check_index(ix)) != TC_DTW_OK) return st;
    if ((st = read_set(qb, "queries", Qs)) != TC_DTW_OK) return st;
    if (Qs.mixed) return fail(TC_DTW_ERR_UNSUPPORTED, "a search needs one dim for all queries (dims must be NULL)");
    if ((st = check_params(p)) != TC_DTW_OK) return st;
    if (Qs.dim != ix->dim) return fail(TC_DTW_ERR_INVALID, "queries and index have different dims");
    if (!Qs.uniform || ix->uniform_len <= 0)
        return fail(TC_DTW_ERR_UNSUPPORTED, "this search needs uniform query and candidate lengths");
    K.nq = Qs.count;
    K.nc = ix->count;
    K.m = Qs.ulen;
    K.n = ix->uniform_len;
    K.D = ix->dim;
    K.W = window_eff(K.m, K.n, p->window);
    K.plain = (p->bounds == 0);
    K.abandon = !K.plain && p->early_abandon != 0;
    K.gate = (p->bounds & (TC_DTW_LB_PC | TC_DTW_LB_TI)) != 0;
    K.pc = (p->bounds & TC_DTW_LB_PC) != 0;
    K.ti = (p->bounds & TC_DTW_LB_TI) != 0;
    K.ngroups = (K.n + p->pc_group - 1) / p->pc_group;
    K.max_pts = std::min(K.m, p->pc_group + 2 * K.W);
    K.cand = p->pc_cand != nullptr;
    if (K.cand) {
        const tc_dtw_cand_boxes* cb = p->pc_cand;
        if (!cb->buf || cb->count != K.nc || cb->dim != K.D || cb->query_len != K.m || cb->cand_len != K.n ||
            cb->weff != K.W || cb->levels != p->pc_levels || cb->clusters != p->pc_clusters ||
            cb->group != p->pc_group || !(cb->min_cell == p->pc_min_cell) ||
            cb->groups != (K.m + p->pc_group - 1) / p->pc_group)
            return fail(TC_DTW_ERR_INVALID,
                        "params.pc_cand was built for another index, query length, window or LB_PC parameters");
    }
    K.k = p->k;
    if (K.k > K.nc) return fail(TC_DTW_ERR_INVALID, "k exceeds the number of candidates");
    // at least k seeds, so that the k-th best is finite before the compaction
    K.R = K.plain ? 0 : std::min(std::min(std::max(p->seed_r > 0 ? p->seed_r : 4, K.k), kMaxSeeds), K.nc);
    K.indep = p->independent != 0;
    if (K.indep && (K.W > kDiagMaxW || nch_pad(K.D) > 4))
        return fail(TC_DTW_ERR_UNSUPPORTED, "independent DTW: band half-width up to 63 and up to 16 dimensions");
    K.P = knn_dtw_max_pairs(K.W, K.D, K.indep);
    K.cap = K.nc;
    K.ntiles = ix->ntiles;
    Carve c(nullptr, 0);
    auto at = [&](size_t bytes) { c.used = (c.used + 255) & ~(size_t)255; size_t o = c.used; c.used += bytes; return o; };
    const size_t nqt = (size_t)(K.nq + kQT - 1) / kQT;
    K.o_env = at(K.plain ? 0 : nqt * kQT * (((size_t)K.n * K.D + 3) / 4 * 4) * 2 * 4);
    K.o_lb = at(K.plain ? 0 : (size_t)K.nq * K.nc * 4);
    K.o_seeds = at((size_t)K.nq * std::max(K.R, 1) * 4);
    K.o_seed_dist = at((size_t)K.nq * std::max(K.R, 1) * 4);
    K.o_list = at((size_t)K.nq * K.cap * 4);
    K.o_list_dist = at((size_t)K.nq * K.cap * 4);
    K.o_cnt = at((size_t)K.nq * 4);
    K.o_glist = at(K.gate ? (size_t)K.nq * K.cap * 4 : 0);
    K.o_gcnt = at((size_t)K.nq * 4);
    K.o_prefix = at((size_t)(K.nq + 1) * 4);
    K.o_items = 0;   // placed after P is final (below)
    K.o_counters = at(kNumCounters * 4);
    K.o_key = at((size_t)K.nq * 8 * kKeyStride);
    K.o_stats = at(kNumStats * 8);
    const bool any_pc = K.pc || true;   // the dense bound matrix may ask for LB_PC / LB_TI too
    (void)any_pc;
    K.o_boxes = at(K.cand ? 0 : (size_t)K.nq * K.ngroups * p->pc_clusters * K.D * 2 * 4);
    K.o_nbox = at(K.cand ? 0 : (size_t)K.nq * K.ngroups * 4);
    K.o_qstep = at((size_t)K.nq * K.m * 4);
    K.o_glb = at(K.gate ? (size_t)K.nq * K.cap * 4 : 0);
    K.o_tlist = at(K.ti ? (size_t)K.nq * K.cap * 4 : 0);
    K.o_tlb = at(K.ti ? (size_t)K.nq * K.cap * 4 : 0);
    K.o_tout = at(K.ti ? (size_t)K.nq * K.cap * 4 : 0);
    K.o_tcnt = at((size_t)K.nq * 4);
    K.o_ppc = at((size_t)K.nq * 4);
    K.o_pti = at((size_t)K.nq * 4);
    K.o_cntmv = at((size_t)K.nq * 4);
    K.nseg = K.plain ? 1 : lb_mv_segments(K.ntiles, K.nq, K.n * K.D);
    K.o_part = at(K.nseg > 1 ? (size_t)K.nseg * K.nq * K.nc * 4 : 0);
    K.o_topk = at(K.k > 1 ? (size_t)K.nq * K.k * 8 : 0);
    K.bytes = c.need();
    {
        // the boxes of one expanded window are built in LDS; its cell keys need Lv^D < 2^63
        unsigned long long pw = 1;
        for (int t = 0; t < K.D; ++t) {
            if (pw > (1ull << 62) / (unsigned long long)p->pc_levels) {
                if (K.pc) return fail(TC_DTW_ERR_UNSUPPORTED, "pc_levels^dim does not fit 63 bits");
                break;
            }
            pw *= (unsigned long long)p->pc_levels;
        }
    }
    const size_t lim = 163840;
    if (knn_dtw_lds_bytes(K.m, K.n, K.W, K.D, 1) > lim || knn_final_lds_bytes(K.m, K.n, K.W, K.D) > lim)
        return fail(TC_DTW_ERR_UNSUPPORTED, "series too long for the LDS staging of one pair");
    while (K.P > 1 && knn_dtw_lds_bytes(K.m, K.n, K.W, K.D, K.P) > lim) --K.P;
    // work items: chunks of P list entries per query (seeds need fewer); LB_TI takes one pair per item
    K.o_items = at((size_t)K.nq * K.cap * 4);
    K.bytes = c.need();
    return TC_DTW_OK;
}

static KnnPlanDev dev_plan(const KnnPlan& K, const tc_dtw_index* ix, const HostSet& Qs, char* ws) {
    KnnPlanDev d;
    std::memset(&d, 0, sizeof d);
    char* base = static_cast<char*>(ix->buf);
    d.Q = Qs.data;
    d.C = reinterpret_cast<const float*>(base + ix->off_series);
    d.tiles = reinterpret_cast<const float*>(base + ix->off_tiles);
    d.nq = K.nq; d.nc = K.nc; d.m = K.m; d.n = K.n; d.D = K.D; d.W = K.W;
    d.ntiles = K.ntiles; d.R = K.R; d.cap = K.cap;
    d.env = K.plain ? nullptr : reinterpret_cast<float*>(ws + K.o_env);
    d.lb = K.plain ? nullptr : reinterpret_cast<float*>(ws + K.o_lb);
    d.seeds = reinterpret_cast<int32_t*>(ws + K.o_seeds);
    d.seed_dist = reinterpret_cast<float*>(ws + K.o_seed_dist);
    d.list = reinterpret_cast<uint32_t*>(ws + K.o_list);
    d.list_dist = reinterpret_cast<float*>(ws + K.o_list_dist);
    d.cnt = reinterpret_cast<int32_t*>(ws + K.o_cnt);
    d.glist = K.gate ? reinterpret_cast<uint32_t*>(ws + K.o_glist) : nullptr;
    d.gcnt = reinterpret_cast<int32_t*>(ws + K.o_gcnt);
    d.prefix = reinterpret_cast<int32_t*>(ws + K.o_prefix);
    d.item_query = reinterpret_cast<int32_t*>(ws + K.o_items);
    d.counters = reinterpret_cast<int32_t*>(ws + K.o_counters);
    d.key = reinterpret_cast<unsigned long long*>(ws + K.o_key);
    d.stats = reinterpret_cast<unsigned long long*>(ws + K.o_stats);
    d.nseg = K.nseg;
    d.part = K.nseg > 1 ? reinterpret_cast<float*>(ws + K.o_part) : nullptr;
    d.k = K.k;
    d.topk = K.k > 1 ? reinterpret_cast<unsigned long long*>(ws + K.o_topk) : nullptr;
    d.status = status_word();
    return d;
}

struct KnnExtra {
    float* boxes;
    int32_t* nbox;
    float* qstep;
    float* glb;
    uint32_t* tlist;
    float* tlb;
    float* tout;
    int32_t* tcnt;
    int32_t* ppc;
    int32_t* pti;
    int32_t* cntmv;
};

static KnnExtra extra_plan(const KnnPlan& K, char* ws) {
    KnnExtra x;
    x.boxes = reinterpret_cast<float*>(ws + K.o_boxes);
    x.nbox = reinterpret_cast<int32_t*>(ws + K.o_nbox);
    x.qstep = reinterpret_cast<float*>(ws + K.o_qstep);
    x.glb = K.gate ? reinterpret_cast<float*>(ws + K.o_glb) : nullptr;
    x.tlist = K.ti ? reinterpret_cast<uint32_t*>(ws + K.o_tlist) : nullptr;
    x.tlb = K.ti ? reinterpret_cast<float*>(ws + K.o_tlb) : nullptr;
    x.tout = K.ti ? reinterpret_cast<float*>(ws + K.o_tout) : nullptr;
    x.tcnt = reinterpret_cast<int32_t*>(ws + K.o_tcnt);
    x.ppc = reinterpret_cast<int32_t*>(ws + K.o_ppc);
    x.pti = reinterpret_cast<int32_t*>(ws + K.o_pti);
    x.cntmv = reinterpret_cast<int32_t*>(ws + K.o_cntmv);
    return x;
}

static PcArgs pc_args(const KnnPlan& K, const KnnPlanDev& d, const KnnExtra& x, const tc_dtw_index* ix,
                      const tc_dtw_knn_params* p) {
    PcArgs a;
    std::memset(&a, 0, sizeof a);
    a.Q = d.Q; a.C = d.C;
    a.nq = K.nq; a.nc = K.nc; a.m = K.m; a.n = K.n; a.D = K.D; a.W = K.W;
    a.Lv = p->pc_levels; a.K = p->pc_clusters; a.w = p->pc_group;
    a.ngroups = K.ngroups; a.max_pts = K.max_pts;
    a.floor_len = p->pc_min_cell;
    a.range = reinterpret_cast<const float*>(static_cast<const char*>(ix->buf) + ix->off_range);
    a.boxes = x.boxes; a.nbox = x.nbox;
    if (K.cand) {
        const tc_dtw_cand_boxes* cb = p->pc_cand;
        a.cand = 1;
        a.boxes = static_cast<float*>(cb->buf);
        a.nbox = reinterpret_cast<int32_t*>(static_cast<char*>(cb->buf) + cb->off_nbox);
        a.ngroups = cb->groups;
    }
    a.cap = K.cap;
    a.prefix = d.prefix; a.item_query = d.item_query; a.counter = d.counters + 2;
    a.lb_mv = d.lb;
    a.keep = 1.0 - (double)p->prune_margin;
    a.e2 = (double)p->trigger_pc * (double)p->trigger_pc;
    return a;
}

static TiArgs ti_args(const KnnPlan& K, const KnnPlanDev& d, const KnnExtra& x, const tc_dtw_index* ix,
                      const tc_dtw_knn_params* p) {
    TiArgs a;
    std::memset(&a, 0, sizeof a);
    a.Q = d.Q; a.C = d.C;
    a.qstep = x.qstep;
    a.gamma = reinterpret_cast<const float*>(static_cast<const char*>(ix->buf) + ix->off_gamma);
    a.nq = K.nq; a.nc = K.nc; a.m = K.m; a.n = K.n; a.D = K.D; a.W = K.W;
    a.P = p->ti_period; a.top = p->ti_top ? 1 : 0;
    a.cap = K.cap;
    a.prefix = d.prefix; a.item_query = d.item_query; a.counter = d.counters + 3;
    a.e2 = (double)p->trigger_ti * (double)p->trigger_ti;
    return a;
}

static float dp_gamma(int m, int n, int D) {
    return (float)(1.01 * (double)(m + n + 4 * nch_pad(D) + 2) * kUnit);
}

static int persistent_blocks(size_t lds, int64_t max_items, int max_per_cu = 24) {
    // one-wave blocks: up to 6 per SIMD (register file; max_per_cu for lighter kernels), fewer
    // when LDS runs out
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(max_per_cu, 163840 / std::max<size_t>(lds, 1)));
    int64_t nb = (int64_t)256 * per_cu;
    if (max_items < nb) nb = std::max<int64_t>(max_items, 1);
    return (int)nb;
}

static KnnDtwArgs list_args(const KnnPlan& K, const KnnPlanDev& d, bool seeds, bool abandon) {
    KnnDtwArgs a;
    std::memset(&a, 0, sizeof a);
    a.Q = d.Q; a.C = d.C;
    a.nq = K.nq; a.m = K.m; a.n = K.n; a.D = K.D; a.W = K.W; a.P = K.P; a.gs = knn_lane_stride(K.W, K.indep);
    a.k = K.k; a.topk = d.topk; a.indep = K.indep ? 1 : 0;
    if (seeds) {
        a.list = reinterpret_cast<const uint32_t*>(d.seeds);
        a.list_dist = d.seed_dist;
        a.cnt = d.cnt;      // unused with cnt_uniform
        a.cnt_uniform = K.R;
        a.cap = K.R;
    } else {
        a.list = d.list;
        a.list_dist = d.list_dist;
        a.cnt = d.cnt;
        a.cnt_uniform = 0;
        a.cap = K.cap;
    }
    a.prefix = d.prefix;
    a.item_query = d.item_query;
    a.counter = d.counters + (seeds ? 0 : 1);
    a.key = d.key;
    a.stats = d.stats;
    a.gamma = dp_gamma(K.m, K.n, K.D);
    a.abandon = abandon ? 1 : 0;
    a.band_cells = band_cells(K.m, K.n, K.W);
    return a;
}

// ------------------------------------------------------------ ragged banks
// Queries or candidates of uneven lengths (one D): LB_MV with per-pair
// windows (query sparse tables), DTW on the row mapping, float64 finalize.
struct RaggedPlan {
    int nq = 0, nc = 0, D = 0, R = 0, maxm = 0, maxn = 0;
    bool plain = false, abandon = true;
    bool banks = false;         // the index holds banks of several D
    uint64_t pairs = 0;         // query-candidate pairs (query-bank pairs with banks)
    tc_dtw_window win{};
    std::vector<int64_t> q_off, t_off;
    std::vector<int32_t> q_len, q_dim, q_cb, q_ce;   // with banks: D and candidate range of each query
    // grouped searches (banks): queries in bank order, q_out[k] the caller's index of query k, and
    // each bank's query range, D and size
    bool grouped = false;
    std::vector<int32_t> q_out;
    std::vector<int> g_q0, g_q1, g_D, g_size;
    int64_t tab_floats = 0;
    size_t o_lb, o_seeds, o_seed_dist, o_list, o_list_dist, o_cnt, o_gcnt, o_prefix, o_items, o_counters,
        o_key, o_stats, o_qoff, o_qlen, o_toff, o_tab, o_qdim, o_qcb, o_qce, o_qout, bytes;
};

static bool is_ragged_search(const tc_dtw_index* ix, const tc_dtw_batch* qb) {
    if (!ix || !qb) return false;
    return ix->uniform_len <= 0 || ix->nbanks > 0 || qb->len != nullptr || qb->offset != nullptr ||
           qb->dims != nullptr;
}

// group: with banks, order the queries by bank (searches: each bank's DTWs then run as one launch
// sized for that bank); the bound matrix keeps the caller's order.
static tc_dtw_status make_ragged_plan(const tc_dtw_index* ix, const tc_dtw_batch* qb, const tc_dtw_knn_params* p,
                                      RaggedPlan& K, HostSet& Qs, bool group = false) {
    tc_dtw_status st;
    if ((st = check_index(ix)) != TC_DTW_OK) return st;
    if ((st = read_set(qb, "queries", Qs)) != TC_DTW_OK) return st;
    if (Qs.mixed && ix->nbanks == 0)
        return fail(TC_DTW_ERR_UNSUPPORTED, "queries of several dims need an index of several banks");
    if ((st = check_params(p)) != TC_DTW_OK) return st;
    if (ix->nbanks == 0 && Qs.dim != ix->dim) return fail(TC_DTW_ERR_INVALID, "queries and index have different dims");
    if (p->bounds & (TC_DTW_LB_PC | TC_DTW_LB_TI))
        return fail(TC_DTW_ERR_UNSUPPORTED, "LB_PC and LB_TI need uniform query and candidate lengths");
    if (p->k > 1) return fail(TC_DTW_ERR_UNSUPPORTED, "k > 1 needs uniform query and candidate lengths");
    if (p->independent) return fail(TC_DTW_ERR_UNSUPPORTED, "independent DTW needs uniform query and candidate lengths");
    K = RaggedPlan();
    K.nq = Qs.count;
    K.nc = ix->count;
    K.D = std::max(Qs.dim, ix->dim);   // the largest D sizes the LDS and the kernels' chunk count
    K.banks = ix->nbanks > 0;
    // order[k]: the caller's index of internal query k
    std::vector<int32_t> order(K.nq);
    for (int q = 0; q < K.nq; ++q) order[q] = q;
    if (K.banks) {
        std::vector<int> bank_of(K.nq);
        for (int q = 0; q < K.nq; ++q) {
            const int D = Qs.dimension(q);
            int b = 0;
            while (b < ix->nbanks && ix->bank_dim[b] != D) ++b;
            if (b == ix->nbanks) return fail(TC_DTW_ERR_INVALID, "a query's dim has no bank in the index");
            bank_of[q] = b;
        }
        if (group) {
            K.grouped = true;
            std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return bank_of[x] < bank_of[y]; });
            K.q_out = order;
            for (int k = 0; k < K.nq;) {
                const int b = bank_of[order[k]];
                int e = k;
                while (e < K.nq && bank_of[order[e]] == b) ++e;
                K.g_q0.push_back(k);
                K.g_q1.push_back(e);
                K.g_D.push_back(ix->bank_dim[b]);
                K.g_size.push_back(ix->bank_count[b]);
                k = e;
            }
        }
        K.q_dim.resize(K.nq);
        K.q_cb.resize(K.nq);
        K.q_ce.resize(K.nq);
        for (int k = 0; k < K.nq; ++k) {
            const int b = bank_of[order[k]];
            K.q_dim[k] = ix->bank_dim[b];
            K.q_cb[k] = ix->bank_first[b];
            K.q_ce[k] = ix->bank_first[b] + ix->bank_count[b];
            K.pairs += (uint64_t)ix->bank_count[b];
        }
    } else {
        K.pairs = (uint64_t)K.nq * K.nc;
    }
    K.win = p->window;
    K.plain = (p->bounds & TC_DTW_LB_MV) == 0;
    K.abandon = p->early_abandon != 0;
    K.R = K.plain ? 0 : std::min(std::min(p->seed_r > 0 ? p->seed_r : 4, kMaxSeeds), K.nc);
    K.maxn = ix->max_len;
    K.q_off.resize(K.nq);
    K.q_len.resize(K.nq);
    K.t_off.resize(K.nq);
    for (int k = 0; k < K.nq; ++k) {
        const int q = order[k];
        const int m = Qs.length(q);
        K.q_off[k] = Qs.offset(q);
        K.q_len[k] = m;
        K.maxm = std::max(K.maxm, m);
        K.t_off[k] = K.tab_floats;
        int L = 0;
        while ((1 << L) <= m) ++L;   // floor(log2 m) + 1
        K.tab_floats += 2LL * L * m * Qs.dimension(q);
    }
    const size_t lim = 163840;
    if (rknn_final_lds_bytes(K.maxn, K.D) > lim)
        return fail(TC_DTW_ERR_UNSUPPORTED, "candidates too long for the row buffer of one pair");
    Carve c(nullptr, 0);
    auto at = [&](size_t bytes) { c.used = (c.used + 255) & ~(size_t)255; size_t o = c.used; c.used += bytes; return o; };
    const size_t pairs = (size_t)K.nq * K.nc;
    K.o_lb = at(K.plain ? 0 : pairs * 4);
    K.o_seeds = at((size_t)K.nq * std::max(K.R, 1) * 4);
    K.o_seed_dist = at((size_t)K.nq * std::max(K.R, 1) * 4);
    K.o_list = at(pairs * 4);
    K.o_list_dist = at(pairs * 4);
    K.o_cnt = at((size_t)K.nq * 4);
    K.o_gcnt = at((size_t)K.nq * 4);
    K.o_prefix = at((size_t)(K.nq + 1) * 4);
    K.o_items = at(pairs * 4);
    K.o_counters = at(kNumCounters * 4);
    K.o_key = at((size_t)K.nq * 8 * kKeyStride);
    K.o_stats = at(kNumStats * 8);
    K.o_qoff = at((size_t)K.nq * 8);
    K.o_qlen = at((size_t)K.nq * 4);
    K.o_toff = at((size_t)K.nq * 8);
    K.o_tab = at(K.plain ? 0 : (size_t)K.tab_floats * 4);
    K.o_qdim = at(K.banks ? (size_t)K.nq * 4 : 0);
    K.o_qcb = at(K.banks ? (size_t)K.nq * 4 : 0);
    K.o_qce = at(K.banks ? (size_t)K.nq * 4 : 0);
    K.o_qout = at(K.grouped ? (size_t)K.nq * 4 : 0);
    K.bytes = c.need();
    return TC_DTW_OK;
}

// Uploads the per-query metadata of a ragged search and points `r` at it.
// With `copy` false the workspace already holds the metadata (params.reuse_query_meta).
static hipError_t ragged_upload(const RaggedPlan& K, char* w, RaggedKnnArgs& r, hipStream_t s, bool copy = true) {
    hipError_t e;
    // pageable host memory: the copies are staged before the calls return
    if (copy &&
        ((e = hipMemcpyAsync(w + K.o_qoff, K.q_off.data(), K.nq * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
         (e = hipMemcpyAsync(w + K.o_qlen, K.q_len.data(), K.nq * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
         (e = hipMemcpyAsync(w + K.o_toff, K.t_off.data(), K.nq * 8, hipMemcpyHostToDevice, s)) != hipSuccess))
        return e;
    r.q_off = reinterpret_cast<const int64_t*>(w + K.o_qoff);
    r.q_len = reinterpret_cast<const int32_t*>(w + K.o_qlen);
    r.t_off = reinterpret_cast<const int64_t*>(w + K.o_toff);
    r.q_dim = r.q_cb = r.q_ce = nullptr;
    if (K.banks) {
        if (copy &&
            ((e = hipMemcpyAsync(w + K.o_qdim, K.q_dim.data(), K.nq * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
             (e = hipMemcpyAsync(w + K.o_qcb, K.q_cb.data(), K.nq * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
             (e = hipMemcpyAsync(w + K.o_qce, K.q_ce.data(), K.nq * 4, hipMemcpyHostToDevice, s)) != hipSuccess))
            return e;
        r.q_dim = reinterpret_cast<const int32_t*>(w + K.o_qdim);
        r.q_cb = reinterpret_cast<const int32_t*>(w + K.o_qcb);
        r.q_ce = reinterpret_cast<const int32_t*>(w + K.o_qce);
        r.bank_max = 0;
        for (int q = 0; q < K.nq; ++q) r.bank_max = std::max(r.bank_max, K.q_ce[q] - K.q_cb[q]);
    }
    r.q_out = nullptr;
    if (K.grouped) {
        if (copy && (e = hipMemcpyAsync(w + K.o_qout, K.q_out.data(), K.nq * 4, hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        r.q_out = reinterpret_cast<const int32_t*>(w + K.o_qout);
    }
    return hipSuccess;
}

static tc_dtw_status knn_ragged(const tc_dtw_index* ix, const tc_dtw_batch* queries, const tc_dtw_knn_params* p,
                                int32_t* nn_idx, float* nn_dist, tc_dtw_knn_stats* stats, void* ws, size_t ws_bytes,
                                hipStream_t s) {
    RaggedPlan K;
    HostSet Qs;
    tc_dtw_status st = make_ragged_plan(ix, queries, p, K, Qs, true);
    if (st != TC_DTW_OK) return st;
    if (!nn_idx || !nn_dist) return fail(TC_DTW_ERR_INVALID, "null output pointer");
    if (!ws || ws_bytes < K.bytes) return fail(TC_DTW_ERR_WORKSPACE, "workspace smaller than tc_dtw_knn_workspace_bytes()");
    if ((st = check_device()) != TC_DTW_OK) return st;
    char* w = static_cast<char*>(ws);
    char* base = static_cast<char*>(ix->buf);
    const int64_t* c_off = reinterpret_cast<const int64_t*>(base + ix->off_meta);
    const int32_t* c_len = reinterpret_cast<const int32_t*>(c_off + 2 * (int64_t)ix->count);

    KnnPlanDev d;
    std::memset(&d, 0, sizeof d);
    d.Q = Qs.data;
    d.C = reinterpret_cast<const float*>(base + ix->off_series);
    d.nq = K.nq; d.nc = K.nc; d.D = K.D; d.R = K.R; d.cap = K.nc;
    d.lb = K.plain ? nullptr : reinterpret_cast<float*>(w + K.o_lb);
    d.seeds = reinterpret_cast<int32_t*>(w + K.o_seeds);
    d.seed_dist = reinterpret_cast<float*>(w + K.o_seed_dist);
    d.list = reinterpret_cast<uint32_t*>(w + K.o_list);
    d.list_dist = reinterpret_cast<float*>(w + K.o_list_dist);
    d.cnt = reinterpret_cast<int32_t*>(w + K.o_cnt);
    d.gcnt = reinterpret_cast<int32_t*>(w + K.o_gcnt);
    d.prefix = reinterpret_cast<int32_t*>(w + K.o_prefix);
    d.item_query = reinterpret_cast<int32_t*>(w + K.o_items);
    d.counters = reinterpret_cast<int32_t*>(w + K.o_counters);
    d.key = reinterpret_cast<unsigned long long*>(w + K.o_key);
    d.stats = reinterpret_cast<unsigned long long*>(w + K.o_stats);

    RaggedKnnArgs r;
    std::memset(&r, 0, sizeof r);
    r.Q = d.Q;
    r.C = d.C;
    r.c_off = c_off;
    r.c_len = c_len;
    r.nq = K.nq; r.nc = K.nc; r.D = K.D; r.maxm = K.maxm; r.maxn = K.maxn;
    r.window = K.win.window; r.num = K.win.frac_num; r.den = K.win.frac_den;
    r.tab = K.plain ? nullptr : reinterpret_cast<float*>(w + K.o_tab);
    r.lb = d.lb;
    r.prefix = d.prefix; r.item_query = d.item_query; r.counter = d.counters + 1;
    r.key = d.key; r.stats = d.stats;
    r.seeds = d.seeds; r.seed_dist = d.seed_dist; r.R = K.R; r.list_cnt = d.cnt;
    r.nn_idx = nn_idx; r.nn_dist = nn_dist;
    r.status = status_word();

    hipEvent_t ev[8];
    const bool timed = stats != nullptr;
    if (timed)
        for (auto& x : ev) (void)hipEventCreate(&x);
    auto mark = [&](int i) { if (timed) (void)hipEventRecord(ev[i], s); };
    hipError_t e;
    if ((e = ragged_upload(K, w, r, s, p->reuse_query_meta == 0)) != hipSuccess)
        return hip_fail(e, "query metadata upload");
    d.q_cb = r.q_cb;
    d.q_ce = r.q_ce;
    mark(0);
    if ((e = launch_knn_prep(d, s)) != hipSuccess) return hip_fail(e, "prep");
    if (!K.plain && (e = launch_rq_tables(r, s)) != hipSuccess) return hip_fail(e, "query tables");
    mark(1);
    // grouped queries: one launch per bank, with that bank's D, size and query range
    auto group_args = [&](const RaggedKnnArgs& base, size_t g) {
        RaggedKnnArgs a = base;
        a.q0 = K.g_q0[g];
        a.q1 = K.g_q1[g];
        a.D = K.g_D[g];
        a.bank_max = K.g_size[g];
        return a;
    };
    if (!K.plain) {
        if (K.grouped) {
            for (size_t g = 0; g < K.g_q0.size(); ++g)
                if ((e = launch_rlb_mv(group_args(r, g), s)) != hipSuccess) return hip_fail(e, "lb_mv");
        } else if ((e = launch_rlb_mv(r, s)) != hipSuccess) {
            return hip_fail(e, "lb_mv");
        }
    }
    mark(2);
    const size_t lds = rknn_dtw_lds_bytes(K.maxn, K.D);
    // the DTW list launches of one stage: one per bank (its own work counter, cleared with the
    // others when the call starts) or one over every query
    auto dtw_launches = [&](const RaggedKnnArgs& a, int64_t per_query, int stage) -> hipError_t {
        if (!K.grouped)
            return launch_rknn_dtw(a, persistent_blocks(lds, (int64_t)K.nq * per_query), s);
        for (size_t g = 0; g < K.g_q0.size(); ++g) {
            RaggedKnnArgs b = group_args(a, g);
            b.counter = d.counters + 1 + 8 * stage + (int)g;
            const int64_t items = (int64_t)(b.q1 - b.q0) * std::min<int64_t>(per_query, b.bank_max);
            hipError_t e2 = launch_rknn_dtw(b, persistent_blocks(rknn_dtw_lds_bytes(K.maxn, b.D), items), s);
            if (e2 != hipSuccess) return e2;
        }
        return hipSuccess;
    };
    KnnDtwArgs scan;
    std::memset(&scan, 0, sizeof scan);
    scan.nq = K.nq; scan.P = 1; scan.prefix = d.prefix; scan.item_query = d.item_query; scan.counter = r.counter;
    if (!K.plain && K.R > 0) {
        if ((e = launch_topr(d, s)) != hipSuccess) return hip_fail(e, "seed selection");
        scan.cnt = d.cnt; scan.cnt_uniform = K.R;
        if ((e = launch_chunk_scan(scan, s)) != hipSuccess) return hip_fail(e, "seed scan");
        RaggedKnnArgs a = r;
        a.list = reinterpret_cast<const uint32_t*>(d.seeds);
        a.list_dist = d.seed_dist;
        a.cap = K.R;
        a.abandon = 0;
        if ((e = dtw_launches(a, K.R, 1)) != hipSuccess) return hip_fail(e, "seed dtw");
    }
    mark(3);
    const double keep = 1.0 - (double)p->prune_margin;
    if ((e = launch_compact(d, K.plain ? 0.0 : keep, 1e300, 0, s)) != hipSuccess) return hip_fail(e, "compaction");
    mark(4);
    {
        scan.cnt = d.cnt; scan.cnt_uniform = 0;
        if ((e = launch_chunk_scan(scan, s)) != hipSuccess) return hip_fail(e, "dtw scan");
        mark(5);
        RaggedKnnArgs a = r;
        a.list = d.list;
        a.list_dist = d.list_dist;
        a.cap = K.nc;
        a.abandon = K.abandon ? 1 : 0;
        if ((e = dtw_launches(a, K.nc, 2)) != hipSuccess) return hip_fail(e, "dtw");
    }
    mark(6);
    {
        RaggedKnnArgs a = r;
        a.list = d.list;
        a.list_dist = d.list_dist;
        a.cap = K.nc;
        if ((e = launch_rknn_finalize(a, s)) != hipSuccess) return hip_fail(e, "finalize");
    }
    mark(7);
    if (timed) {
        unsigned long long h[kNumStats];
        e = hipMemcpyAsync(h, d.stats, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "stats readback");
        std::memset(stats, 0, sizeof *stats);
        stats->pairs = K.pairs;
        stats->pruned_mv = h[kStPrunedMv];
        stats->dtw_started = h[kStDtwStarted];
        stats->dtw_abandoned = h[kStDtwAbandoned];
        stats->dtw_completed = h[kStDtwStarted] - h[kStDtwAbandoned];
        stats->cells = h[kStCells];
        stats->rescored = h[kStRescored];
        for (int i = 0; i < 7; ++i) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            stats->stage_ms[i] = ms;
        }
        float tot = 0.0f;
        (void)hipEventElapsedTime(&tot, ev[0], ev[7]);
        stats->stage_ms[7] = tot;
        for (auto& x : ev) (void)hipEventDestroy(x);
    }
    return ok();
}

}  // namespace tcdtw

using namespace tcdtw;

extern "C" {

void tc_dtw_knn_params_default(tc_dtw_knn_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->window.frac_num = 1;
    p->window.frac_den = 10;
    p->bounds = TC_DTW_LB_MV;
    p->early_abandon = 1;
    p->ti_period = 5;
    p->ti_top = 1;
    p->pc_levels = 2;
    p->pc_clusters = 6;
    p->pc_group = 6;
    p->pc_min_cell = 0.0f;
    p->trigger_ti = 0.1f;
    p->trigger_pc = 0.1f;
    p->prune_margin = 1e-6f;
    p->seed_r = 4;
    p->k = 1;
    p->independent = 0;
}

size_t tc_dtw_index_bytes(const tc_dtw_batch* refs) {
    HostSet R;
    if (read_set(refs, "refs", R) != TC_DTW_OK) return 0;
    tc_dtw_index tmp;
    if (index_banks(R, tmp) != TC_DTW_OK) return 0;
    return index_layout(R).bytes;
}

tc_dtw_status tc_dtw_build_index(const tc_dtw_batch* refs, void* buf, size_t bytes, tc_dtw_index* out,
                                 tc_dtw_stream stream) {
    HostSet R;
    tc_dtw_status st = read_set(refs, "refs", R);
    if (st != TC_DTW_OK) return st;
    if (!buf || !out) return fail(TC_DTW_ERR_INVALID, "null index buffer or output");
    tc_dtw_index banks;
    std::memset(&banks, 0, sizeof banks);
    if ((st = index_banks(R, banks)) != TC_DTW_OK) return st;
    const IndexLayout L = index_layout(R);
    if (bytes < L.bytes) return fail(TC_DTW_ERR_WORKSPACE, "index buffer smaller than tc_dtw_index_bytes()");
    if ((st = check_device()) != TC_DTW_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(buf);
    IndexBuildArgs a;
    std::memset(&a, 0, sizeof a);
    a.src = R.data;
    a.count = R.count;
    a.ulen = L.ulen;
    a.D = R.dim;
    a.maxlen = R.maxlen;
    a.ntiles = L.ntiles;
    a.total_len = L.total_len;
    a.series = reinterpret_cast<float*>(base + L.off_series);
    a.tiles = L.uniform ? reinterpret_cast<float*>(base + L.off_tiles) : nullptr;
    a.gamma = reinterpret_cast<float*>(base + L.off_gamma);
    a.range_keys = reinterpret_cast<uint32_t*>(base + L.off_range);
    a.status = status_word();
    // meta: dst offsets, gamma offsets, lengths, source offsets
    int64_t* dst_off = reinterpret_cast<int64_t*>(base + L.off_meta);
    int64_t* gam_off = dst_off + R.count;
    int32_t* lens = reinterpret_cast<int32_t*>(gam_off + R.count);
    int64_t* src_off = reinterpret_cast<int64_t*>(lens + R.count + (R.count & 1));
    std::vector<int64_t> h_dst(R.count), h_gam(R.count), h_src(R.count);
    std::vector<int32_t> h_len(R.count);
    int64_t next = 0, gnext = 0;
    for (int k = 0; k < R.count; ++k) {
        h_len[k] = R.length(k);
        h_src[k] = R.offset(k);
        h_dst[k] = next;
        h_gam[k] = gnext;
        next += (int64_t)h_len[k] * R.dimension(k);
        gnext += h_len[k];
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(dst_off, h_dst.data(), R.count * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(gam_off, h_gam.data(), R.count * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(lens, h_len.data(), R.count * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(src_off, h_src.data(), R.count * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "index metadata upload");
    if (R.mixed) {
        int32_t* dims = reinterpret_cast<int32_t*>(base + L.off_dims);
        if ((e = hipMemcpyAsync(dims, R.dims.data(), R.count * 4, hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, "index metadata upload");
        a.dims = dims;
    }
    a.dst_off = dst_off;
    a.gamma_off = gam_off;
    a.lens = lens;
    a.src_off = src_off;
    if ((e = launch_index_build(a, s)) != hipSuccess) return hip_fail(e, "index build launch");
    std::memset(out, 0, sizeof *out);
    out->buf = buf;
    out->bytes = L.bytes;
    out->count = R.count;
    out->dim = R.dim;
    out->uniform_len = L.ulen;
    out->max_len = R.maxlen;
    out->ntiles = L.ntiles;
    out->off_series = (int64_t)L.off_series;
    out->off_tiles = (int64_t)L.off_tiles;
    out->off_gamma = (int64_t)L.off_gamma;
    out->off_meta = (int64_t)L.off_meta;
    out->off_range = (int64_t)L.off_range;
    out->total_len = L.total_len;
    out->off_dims = R.mixed ? (int64_t)L.off_dims : 0;
    out->nbanks = banks.nbanks;
    for (int b = 0; b < banks.nbanks; ++b) {
        out->bank_dim[b] = banks.bank_dim[b];
        out->bank_first[b] = banks.bank_first[b];
        out->bank_count[b] = banks.bank_count[b];
    }
    return ok();
}

size_t tc_dtw_knn_workspace_bytes(const tc_dtw_index* ix, const tc_dtw_batch* queries,
                                  const tc_dtw_knn_params* p) {
    if (is_ragged_search(ix, queries)) {
        RaggedPlan R;
        HostSet Qr;
        return make_ragged_plan(ix, queries, p, R, Qr, true) == TC_DTW_OK ? R.bytes : 0;
    }
    KnnPlan K;
    HostSet Q;
    if (make_knn_plan(ix, queries, p, K, Q) != TC_DTW_OK) return 0;
    return K.bytes;
}

tc_dtw_status tc_dtw_knn(const tc_dtw_index* ix, const tc_dtw_batch* queries, const tc_dtw_knn_params* p,
                         int32_t* nn_idx, float* nn_dist, tc_dtw_knn_stats* stats, void* ws,
                         size_t ws_bytes, tc_dtw_stream stream) {
    if (is_ragged_search(ix, queries))
        return knn_ragged(ix, queries, p, nn_idx, nn_dist, stats, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream));
    KnnPlan K;
    HostSet Qs;
    tc_dtw_status st = make_knn_plan(ix, queries, p, K, Qs);
    if (st != TC_DTW_OK) return st;
    if (!nn_idx || !nn_dist) return fail(TC_DTW_ERR_INVALID, "null output pointer");
    if (K.ti && ti_lds_bytes(K.m, K.n, K.D, p->ti_period, K.W) > 163840)
        return fail(TC_DTW_ERR_UNSUPPORTED, "LB_TI stages a pair in LDS: series too long");
    if (!ws || ws_bytes < K.bytes) return fail(TC_DTW_ERR_WORKSPACE, "workspace smaller than tc_dtw_knn_workspace_bytes()");
    if ((st = check_device()) != TC_DTW_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    const KnnExtra x = extra_plan(K, w);
    KnnPlanDev dd = dev_plan(K, ix, Qs, w);
    dd.clear[0] = x.tcnt;
    dd.clear[1] = x.ppc;
    dd.clear[2] = x.pti;
    const KnnPlanDev d = dd;

    hipEvent_t ev[10];   // stage marks 0-7; 8-9 around the LB_TI launch
    const bool timed = stats != nullptr;
    if (timed)
        for (auto& x : ev) (void)hipEventCreate(&x);
    auto mark = [&](int i) { if (timed) (void)hipEventRecord(ev[i], s); };

    hipError_t e;
    mark(0);
    if ((e = launch_knn_prep(d, s)) != hipSuccess) return hip_fail(e, "prep");
    if (K.ti && (e = launch_query_steps(d.Q, K.nq, K.m, K.D, x.qstep, s)) != hipSuccess) return hip_fail(e, "query steps");
    if (K.pc && !K.cand && (e = launch_pc_boxes(pc_args(K, d, x, ix, p), s)) != hipSuccess) return hip_fail(e, "boxes");
    mark(1);
    if (!K.plain) {
        if ((e = launch_lb_mv(d, d.lb, s)) != hipSuccess) return hip_fail(e, "lb_mv");
    }
    mark(2);
    const size_t lds = knn_dtw_lds_bytes(K.m, K.n, K.W, K.D, K.P);
    if (!K.plain && K.R > 0) {
        if ((e = launch_topr(d, s)) != hipSuccess) return hip_fail(e, "seed selection");
        const KnnDtwArgs a = list_args(K, d, true, false);
        const int64_t items = (int64_t)K.nq * ((K.R + K.P - 1) / K.P);
        if ((e = launch_chunk_scan(a, s)) != hipSuccess) return hip_fail(e, "seed scan");
        if ((e = launch_dtw_lists(a, persistent_blocks(lds, items), s)) != hipSuccess) return hip_fail(e, "seed dtw");
    }
    mark(3);
    const double keep = 1.0 - (double)p->prune_margin;
    const double e_pc = p->trigger_pc, e_ti = p->trigger_ti;
    double gate_e2 = 1e300;
    if (K.pc) gate_e2 = std::min(gate_e2, e_pc * e_pc);
    if (K.ti) gate_e2 = std::min(gate_e2, e_ti * e_ti);
    if ((e = launch_compact(d, K.plain ? 0.0 : keep, gate_e2, K.gate ? 1 : 0, s)) != hipSuccess)
        return hip_fail(e, "compaction");
    mark(4);
    if (K.gate) {
        // Sec. 6: advanced bounds only for gated pairs; LB_PC first, then LB_TI
        if ((e = launch_copy_i32(d.cnt, x.cntmv, K.nq, s)) != hipSuccess) return hip_fail(e, "snapshot");
        const int pc_blocks = persistent_blocks(0, (int64_t)K.nq * K.cap, 32);   // up to 8 waves per SIMD (fewer where registers cap them)
        RouteArgs r;
        std::memset(&r, 0, sizeof r);
        r.nq = K.nq; r.nc = K.nc; r.cap = K.cap;
        r.lb_mv = d.lb; r.key = d.key; r.keep = keep;
        r.dtw_list = d.list; r.dtw_cnt = d.cnt;
        if (K.pc) {
            PcArgs a = pc_args(K, d, x, ix, p);
            a.in_list = d.glist; a.in_cnt = d.gcnt; a.in_uniform = 0;
            a.out_lb = x.glb; a.key = d.key;
            a.evaluated = d.stats + kStEvalPc;
            // query-side boxes: waves over 64 listed candidates of a query; candidate-side: one pair per wave
            const int per = K.cand ? 1 : kWave;
            if ((e = launch_list_items(d.gcnt, 0, K.nq, per, d.prefix, d.item_query, a.counter, s)) != hipSuccess)
                return hip_fail(e, "pc items");
            e = K.cand ? launch_lb_pc(a, pc_blocks, s) : launch_lb_pc_lanes(a, pc_blocks, s);
            if (e != hipSuccess) return hip_fail(e, "lb_pc");
            r.in_list = d.glist; r.in_cnt = d.gcnt; r.lb_prev = nullptr; r.lb_new = x.glb;
            r.next_list = K.ti ? x.tlist : nullptr; r.next_lb = x.tlb; r.next_cnt = x.tcnt;
            r.next_e2 = e_ti * e_ti;
            r.pruned = x.ppc;
            if ((e = launch_route(r, K.cap, s)) != hipSuccess) return hip_fail(e, "route pc");
        } else if (K.ti) {
            // no LB_PC: every gated pair goes to the LB_TI list with its LB_MV
            r.in_list = d.glist; r.in_cnt = d.gcnt; r.lb_prev = nullptr; r.lb_new = nullptr;
            r.next_list = x.tlist; r.next_lb = x.tlb; r.next_cnt = x.tcnt; r.next_e2 = -1.0;
            r.pruned = x.ppc;
            if ((e = launch_route(r, K.cap, s)) != hipSuccess) return hip_fail(e, "route mv");
        }
        if (K.ti) {
            TiArgs a = ti_args(K, d, x, ix, p);
            a.in_list = x.tlist; a.out_lb = x.tout; a.lb_in = x.tlb; a.key = d.key;
            a.evaluated = d.stats + kStEvalTi;
            if (timed) (void)hipEventRecord(ev[8], s);
            if ((e = launch_list_items(x.tcnt, 0, K.nq, 1, d.prefix, d.item_query, a.counter, s)) != hipSuccess)
                return hip_fail(e, "ti items");
            const int ti_blocks = persistent_blocks(ti_lds_bytes(K.m, K.n, K.D, p->ti_period, K.W), (int64_t)K.nq * K.cap);
            if ((e = launch_lb_ti(a, ti_blocks, s)) != hipSuccess) return hip_fail(e, "lb_ti");
            if (timed) (void)hipEventRecord(ev[9], s);
            RouteArgs r2 = r;
            r2.in_list = x.tlist; r2.in_cnt = x.tcnt; r2.lb_prev = x.tlb; r2.lb_new = x.tout;
            r2.next_list = nullptr; r2.pruned = x.pti;
            if ((e = launch_route(r2, K.cap, s)) != hipSuccess) return hip_fail(e, "route ti");
        }
    }
    {
        const KnnDtwArgs a = list_args(K, d, false, K.abandon);
        const int64_t items = (int64_t)K.nq * ((K.nc + K.P - 1) / K.P);
        if ((e = launch_chunk_scan(a, s)) != hipSuccess) return hip_fail(e, "dtw scan");
        mark(5);
        if ((e = launch_dtw_lists(a, persistent_blocks(lds, items), s)) != hipSuccess) return hip_fail(e, "dtw");
    }
    mark(6);
    {
        KnnFinalArgs f;
        std::memset(&f, 0, sizeof f);
        f.Q = d.Q; f.C = d.C;
        f.nq = K.nq; f.m = K.m; f.n = K.n; f.D = K.D; f.W = K.W; f.R = K.R; f.cap = K.cap;
        f.seeds = d.seeds; f.seed_dist = d.seed_dist;
        f.list = d.list; f.list_dist = d.list_dist; f.cnt = d.cnt;
        f.gcnt = K.gate ? d.gcnt : nullptr;
        f.cnt_mv = K.gate ? x.cntmv : nullptr;
        f.pruned_pc = K.gate ? x.ppc : nullptr;
        f.pruned_ti = K.gate ? x.pti : nullptr;
        f.nc = K.nc;
        const double g = dp_gamma(K.m, K.n, K.D);
        f.ratio = (1.0 + g) / (1.0 - g) * (1.0 + 1e-9);
        f.k = K.k;
        f.indep = K.indep ? 1 : 0;
        f.nn_idx = nn_idx; f.nn_dist = nn_dist;
        f.stats = d.stats;
        f.key = d.key;
        if ((e = launch_knn_finalize(f, s)) != hipSuccess) return hip_fail(e, "finalize");
    }
    mark(7);
    if (timed) {
        unsigned long long h[kNumStats];
        e = hipMemcpyAsync(h, d.stats, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "stats readback");
        std::memset(stats, 0, sizeof *stats);
        stats->pairs = (uint64_t)K.nq * K.nc;
        stats->pruned_mv = h[kStPrunedMv];
        stats->pruned_pc = h[kStPrunedPc];
        stats->pruned_ti = h[kStPrunedTi];
        stats->dtw_started = h[kStDtwStarted];
        stats->dtw_abandoned = h[kStDtwAbandoned];
        stats->dtw_completed = h[kStDtwStarted] - h[kStDtwAbandoned];
        stats->cells = h[kStCells];
        stats->rescored = h[kStRescored];
        stats->evaluated_pc = h[kStEvalPc];
        stats->evaluated_ti = h[kStEvalTi];
        for (int i = 0; i < 7; ++i) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            stats->stage_ms[i] = ms;
        }
        float tot = 0.0f;
        (void)hipEventElapsedTime(&tot, ev[0], ev[7]);
        stats->stage_ms[7] = tot;
        if (K.gate && K.ti) (void)hipEventElapsedTime(&stats->lb_ti_ms, ev[8], ev[9]);
        for (auto& x : ev) (void)hipEventDestroy(x);
    }
    return ok();
}

// ------------------------------------------------ candidate-side boxes
// LB_PC with the roles swapped (Sec. 8): k_pc_boxes run over the candidates
// as the boxed series, with groups over query positions.
struct CandBoxGeom {
    int count, n, m, D, W, groups, max_pts, K;
    size_t off_nbox, bytes;
};

static tc_dtw_status cand_box_geom(const tc_dtw_index* ix, int32_t query_len, const tc_dtw_knn_params* p,
                                   CandBoxGeom& g) {
    tc_dtw_status st;
    if ((st = check_index(ix)) != TC_DTW_OK) return st;
    if ((st = check_params(p)) != TC_DTW_OK) return st;
    if (ix->uniform_len <= 0) return fail(TC_DTW_ERR_UNSUPPORTED, "candidate-side boxes need uniform candidate lengths");
    if (query_len < 1) return fail(TC_DTW_ERR_INVALID, "query_len must be >= 1");
    g.count = ix->count;
    g.n = ix->uniform_len;
    g.m = query_len;
    g.D = ix->dim;
    g.W = window_eff(g.m, g.n, p->window);
    g.groups = (g.m + p->pc_group - 1) / p->pc_group;
    g.max_pts = std::min(g.n, p->pc_group + 2 * g.W);
    g.K = p->pc_clusters;
    unsigned long long pw = 1;   // cell keys in base Lv need Lv^D < 2^63
    for (int t = 0; t < g.D; ++t) {
        if (pw > (1ull << 62) / (unsigned long long)p->pc_levels)
            return fail(TC_DTW_ERR_UNSUPPORTED, "pc_levels^dim does not fit 63 bits");
        pw *= (unsigned long long)p->pc_levels;
    }
    if (pc_boxes_lds_bytes(g.max_pts, g.K, g.D) > 163840)
        return fail(TC_DTW_ERR_UNSUPPORTED, "expanded window too long for the LDS box construction");
    const size_t boxes = (size_t)g.count * g.groups * g.K * g.D * 2 * 4;
    g.off_nbox = (boxes + 255) & ~(size_t)255;
    g.bytes = g.off_nbox + (size_t)g.count * g.groups * 4;
    return TC_DTW_OK;
}

size_t tc_dtw_cand_boxes_bytes(const tc_dtw_index* ix, int32_t query_len, const tc_dtw_knn_params* p) {
    CandBoxGeom g;
    return cand_box_geom(ix, query_len, p, g) == TC_DTW_OK ? g.bytes : 0;
}

tc_dtw_status tc_dtw_build_cand_boxes(const tc_dtw_index* ix, int32_t query_len, const tc_dtw_knn_params* p,
                                      void* buf, size_t bytes, tc_dtw_cand_boxes* out, tc_dtw_stream stream) {
    CandBoxGeom g;
    tc_dtw_status st = cand_box_geom(ix, query_len, p, g);
    if (st != TC_DTW_OK) return st;
    if (!out) return fail(TC_DTW_ERR_INVALID, "null descriptor");
    if (!buf || bytes < g.bytes) return fail(TC_DTW_ERR_INVALID, "buffer smaller than tc_dtw_cand_boxes_bytes()");
    if ((st = check_device()) != TC_DTW_OK) return st;
    PcArgs a;
    std::memset(&a, 0, sizeof a);
    a.Q = reinterpret_cast<const float*>(static_cast<const char*>(ix->buf) + ix->off_series);
    a.nq = g.count; a.m = g.n; a.n = g.m; a.D = g.D; a.W = g.W;
    a.Lv = p->pc_levels; a.K = g.K; a.w = p->pc_group;
    a.ngroups = g.groups; a.max_pts = g.max_pts;
    a.floor_len = p->pc_min_cell;
    a.range = reinterpret_cast<const float*>(static_cast<const char*>(ix->buf) + ix->off_range);
    a.boxes = static_cast<float*>(buf);
    a.nbox = reinterpret_cast<int32_t*>(static_cast<char*>(buf) + g.off_nbox);
    hipError_t e = launch_pc_boxes(a, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "candidate boxes");
    std::memset(out, 0, sizeof *out);
    out->buf = buf;
    out->off_nbox = (int64_t)g.off_nbox;
    out->count = g.count; out->dim = g.D; out->query_len = g.m; out->cand_len = g.n;
    out->weff = g.W; out->groups = g.groups;
    out->levels = p->pc_levels; out->clusters = p->pc_clusters; out->group = p->pc_group;
    out->min_cell = p->pc_min_cell;
    return ok();
}

size_t tc_dtw_lower_bounds_workspace_bytes(const tc_dtw_index* ix, const tc_dtw_batch* queries,
                                           const tc_dtw_knn_params* p, uint32_t kind) {
    if (is_ragged_search(ix, queries)) {
        if (kind != TC_DTW_LB_MV) return 0;
        RaggedPlan R;
        HostSet Qr;
        tc_dtw_knn_params pm = p ? *p : tc_dtw_knn_params{};
        pm.bounds = TC_DTW_LB_MV;
        return p && make_ragged_plan(ix, queries, &pm, R, Qr) == TC_DTW_OK ? R.bytes : 0;
    }
    KnnPlan K;
    HostSet Q;
    if (make_knn_plan(ix, queries, p, K, Q) != TC_DTW_OK) return 0;
    (void)kind;
    return K.bytes;
}

tc_dtw_status tc_dtw_lower_bounds(const tc_dtw_index* ix, const tc_dtw_batch* queries,
                                  const tc_dtw_knn_params* p, uint32_t kind, float* lb, void* ws,
                                  size_t ws_bytes, tc_dtw_stream stream) {
    if (is_ragged_search(ix, queries)) {
        if (kind != TC_DTW_LB_MV)
            return fail(TC_DTW_ERR_UNSUPPORTED, "LB_PC and LB_TI need uniform query and candidate lengths");
        if (!p) return fail(TC_DTW_ERR_INVALID, "null params");
        tc_dtw_knn_params pm = *p;
        pm.bounds = TC_DTW_LB_MV;
        RaggedPlan R;
        HostSet Qr;
        tc_dtw_status st = make_ragged_plan(ix, queries, &pm, R, Qr);
        if (st != TC_DTW_OK) return st;
        if (!lb) return fail(TC_DTW_ERR_INVALID, "null lb pointer");
        if (!ws || ws_bytes < R.bytes) return fail(TC_DTW_ERR_WORKSPACE, "workspace smaller than tc_dtw_lower_bounds_workspace_bytes()");
        if ((st = check_device()) != TC_DTW_OK) return st;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        char* w = static_cast<char*>(ws);
        char* base = static_cast<char*>(ix->buf);
        RaggedKnnArgs a;
        std::memset(&a, 0, sizeof a);
        a.Q = Qr.data;
        a.C = reinterpret_cast<const float*>(base + ix->off_series);
        a.c_off = reinterpret_cast<const int64_t*>(base + ix->off_meta);
        a.c_len = reinterpret_cast<const int32_t*>(a.c_off + 2 * (int64_t)ix->count);
        a.nq = R.nq; a.nc = R.nc; a.D = R.D; a.maxm = R.maxm; a.maxn = R.maxn;
        a.window = R.win.window; a.num = R.win.frac_num; a.den = R.win.frac_den;
        a.tab = reinterpret_cast<float*>(w + R.o_tab);
        a.lb = lb;
        a.status = status_word();
        hipError_t e;
        if ((e = ragged_upload(R, w, a, s)) != hipSuccess) return hip_fail(e, "query metadata upload");
        // with banks, a query's bound is computed for its own bank only: +inf elsewhere
        if (R.banks && (e = launch_fill_f32(lb, (int64_t)R.nq * R.nc, __builtin_inff(), s)) != hipSuccess)
            return hip_fail(e, "bound fill");
        if ((e = launch_rq_tables(a, s)) != hipSuccess) return hip_fail(e, "query tables");
        if ((e = launch_rlb_mv(a, s)) != hipSuccess) return hip_fail(e, "lb_mv");
        return ok();
    }
    KnnPlan K;
    HostSet Qs;
    tc_dtw_status st = make_knn_plan(ix, queries, p, K, Qs);
    if (st != TC_DTW_OK) return st;
    if (!lb) return fail(TC_DTW_ERR_INVALID, "null lb pointer");
    if (kind != TC_DTW_LB_MV && kind != TC_DTW_LB_PC && kind != TC_DTW_LB_TI)
        return fail(TC_DTW_ERR_INVALID, "kind must be one of TC_DTW_LB_MV, TC_DTW_LB_PC, TC_DTW_LB_TI");
    if (kind == TC_DTW_LB_TI && ti_lds_bytes(K.m, K.n, K.D, p->ti_period, K.W) > 163840)
        return fail(TC_DTW_ERR_UNSUPPORTED, "LB_TI stages a pair in LDS: series too long");
    if (K.plain) return fail(TC_DTW_ERR_INVALID, "params.bounds must include TC_DTW_LB_MV");
    if (!ws || ws_bytes < K.bytes) return fail(TC_DTW_ERR_WORKSPACE, "workspace smaller than tc_dtw_lower_bounds_workspace_bytes()");
    if ((st = check_device()) != TC_DTW_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const KnnPlanDev d = dev_plan(K, ix, Qs, static_cast<char*>(ws));
    const KnnExtra x = extra_plan(K, static_cast<char*>(ws));
    hipError_t e;
    if ((e = launch_knn_prep(d, s, kind != TC_DTW_LB_MV)) != hipSuccess) return hip_fail(e, "prep");
    if (kind == TC_DTW_LB_MV) {
        if ((e = launch_lb_mv(d, lb, s)) != hipSuccess) return hip_fail(e, "lb_mv");
    } else if (kind == TC_DTW_LB_PC) {
        PcArgs a = pc_args(K, d, x, ix, p);
        if (!K.cand && (e = launch_pc_boxes(a, s)) != hipSuccess) return hip_fail(e, "boxes");
        a.in_list = nullptr; a.in_uniform = K.nc; a.cap = K.nc; a.out_lb = lb; a.key = nullptr;
        const int per = K.cand ? 1 : kWave;
        if ((e = launch_list_items(nullptr, K.nc, K.nq, per, d.prefix, d.item_query, a.counter, s)) != hipSuccess)
            return hip_fail(e, "pc items");
        const int blocks = persistent_blocks(0, (int64_t)K.nq * ((K.nc + per - 1) / per));
        e = K.cand ? launch_lb_pc(a, blocks, s) : launch_lb_pc_lanes(a, blocks, s);
        if (e != hipSuccess) return hip_fail(e, "lb_pc");
    } else {
        if ((e = launch_query_steps(d.Q, K.nq, K.m, K.D, x.qstep, s)) != hipSuccess) return hip_fail(e, "query steps");
        TiArgs a = ti_args(K, d, x, ix, p);
        a.in_list = nullptr; a.cap = K.nc; a.out_lb = lb; a.key = nullptr;
        if ((e = launch_list_items(nullptr, K.nc, K.nq, 1, d.prefix, d.item_query, a.counter, s)) != hipSuccess)
            return hip_fail(e, "ti items");
        if ((e = launch_lb_ti(a, persistent_blocks(ti_lds_bytes(K.m, K.n, K.D, p->ti_period, K.W), (int64_t)K.nq * K.nc), s)) != hipSuccess)
            return hip_fail(e, "lb_ti");
    }
    return ok();
}

}  // extern "C"
