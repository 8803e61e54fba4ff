"""Benchmark of the 1-NN DTW search with the lower-bound cascade on one MI355X.

One step = one tc_dtw_knn call over the whole query batch (query
envelopes, LB_MV, best-so-far seeding, compaction, advanced bounds when
enabled, DTW of the survivors with early abandoning, float64 re-scoring of
near-tie finalists).  Inputs and the candidate index are resident in HBM
before the timed region; the index build is timed separately.

Prints one JSON line with:
  value       queries/s of the whole batch,
  roofline    the DTW kernel (the step's dominant kernel) as useful band
              cells/s against the VALU bound of (2D + 2) lane-operations per
              cell, its duration taken from HIP events recorded by the
              library on the search stream around that kernel,
  cpu_baseline  the FP64 oracle (exhaustive search, the plain definition)
              timed on a bounded sample of the same queries.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
T_START = time.perf_counter()
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (generator kwargs, window fraction, description)
    "cascade": (dict(nq=1000, nc=10000, T=256, D=8), (1, 10),
                "pruned 1-NN: 1000 queries x 10000 references, length 256, d=8, "
                "correlated walks with 8 warped prototypes, window 10% (W=25)"),
    "plain": (dict(nq=64, nc=256, T=64, D=3), (1, 10),
              "plain 1-NN: 64 queries x 256 references, length 64, d=3, random walks, window 10% (W=6)"),
}

# MI355X fp32 vector peak: 256 CUs x 2.4 GHz x 256 flops per CU per clock (128 lanes of fused
# multiply-add per clock, counted as 2 flops each; the rate assumes packed fp32) = 157.3 TFLOP/s.
# The DTW kernels issue plain (non-packed) fp32 instructions, one wave64 instruction per SIMD
# every 4 cycles = 39.3e12 lane-operations/s, so a kernel that issues one instruction per
# slot reaches at most (3d + 3) / (2 (2d + 2)) of the published peak.
FP32_PEAK_FLOPS = 256 * 2.4e9 * 256
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9

# The counter figures of the DTW survivor launch, with the digest of the sources the kernel is
# built from when they were taken: the traffic is reported only while the sources are unchanged.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "knn_dtw_ring_traffic_1000x10000_d8.md")
DTW_KERNEL_SOURCES = ("knn.hip", "dtw_core.h", "device_common.h")


STAGES = ("prep", "lb_mv", "seed", "compact", "lb_pc_ti", "dtw", "finalize", "total")

EXTRAS = ("full_cascade", "cand_boxes", "cascade_setup", "knn_k10", "knn_independent", "single_query_latency",
          "batched_pairs", "dtw_loss", "long_knn", "ragged_banks", "lb_mv_streaming", "plain_gpu", "windows",
          "trajectories", "small_graph")
# measured on every run: the batched and forward+backward pair rates of the metric, the plain
# (no bounds) method on the same GPU, the other windows, and the trajectory workload on which the
# advanced bounds prune
DEFAULT_EXTRAS = ("plain_gpu", "windows", "batched_pairs", "dtw_loss", "trajectories")


def source_digest(names=DTW_KERNEL_SOURCES):
    """sha256 (16 hex digits) of the named kernel sources, in order."""
    import hashlib
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2101_07731_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """(bytes per DTW survivor launch, digest) from the committed counter summary, or (None, reason)."""
    import re
    try:
        txt = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None, "no counter summary"
    md = re.search(r"source digest: `([0-9a-f]{16})`", txt)
    mb = re.search(r"bytes per launch: `([0-9.eE+]+)`", txt)
    if not md or not mb:
        return None, "counter summary without digest"
    if md.group(1) != source_digest():
        return None, "kernel sources changed since the counters were taken"
    return float(mb.group(1)), md.group(1)


def note(what):
    """One progress line per bench stage on stderr (the JSON line stays alone on stdout)."""
    print("bench: %s (%.1f s)" % (what, time.perf_counter() - T_START), file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cascade", choices=sorted(WORKLOADS))
    ap.add_argument("--bounds", default="mv")
    ap.add_argument("--frac", default=None, help="window fraction num/den, e.g. 1/10")
    ap.add_argument("--cpu-queries", type=int, default=300, help="queries in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extras", nargs="*", default=None, choices=EXTRAS, metavar="NAME",
                    help="also time further workloads: all of them with no name, else the named ones "
                         "(%s); %s always run unless --no-extras" % (", ".join(EXTRAS), ", ".join(DEFAULT_EXTRAS)))
    ap.add_argument("--no-extras", action="store_true", help="time the search step only")
    return ap.parse_args()


def _events_ms(fn, reps):
    """Average ms of fn() over reps runs, timed with events on torch's current
    stream (the stream the library enqueues on)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def band_cells(m, n, W):
    return sum(max(0, min(n - 1, i + W) - max(0, i - W) + 1) for i in range(m))


def w_eff(m, n, num, den):
    W = max(m, n) * num // den
    return min(max(W, abs(m - n)), max(m, n) - 1)


def extra_batched_pairs(dev, reps=5):
    """4096 pairs, lengths uniform in [64, 2048] (independent), d in {2,4,8,16,32},
    window 10%: autotuned plan, replayed from a HIP graph."""
    import torch
    from paper_2101_07731_amd import pairs, synth
    xs, ys = synth.ragged_pairs()
    X = [torch.from_numpy(a).to(dev) for a in xs]
    Y = [torch.from_numpy(a).to(dev) for a in ys]
    cells = sum(band_cells(a.shape[0], b.shape[0], w_eff(a.shape[0], b.shape[0], 1, 10)) for a, b in zip(xs, ys))
    t0 = time.perf_counter()
    best, times = pairs.autotune(X, Y, frac=(1, 10), reps=2)
    tune_s = time.perf_counter() - t0
    plan = pairs.Plan(X, Y, frac=(1, 10), diag_max_w=best[0], waves_per_cu=best[1], waves_per_pair=best[2])
    gf = pairs.GraphedForward(plan)
    ms_graph = _events_ms(gf.replay, reps)
    default = pairs.Plan(X, Y, frac=(1, 10))
    dist = torch.empty(default.count, dtype=torch.float32, device=dev)
    ms_default = _events_ms(lambda: default.forward(dist=dist), reps)
    ms_direct = _events_ms(lambda: pairs.banded(X, Y, frac=(1, 10)), 2)
    return {"workload": "4096 pairs, lengths U[64,2048] independent, d in {2,4,8,16,32}, window 10%",
            "pairs_per_s": round(len(xs) / (ms_graph * 1e-3), 1),
            "gcups": round(cells / (ms_graph * 1e-3) / 1e9, 2),
            "ms_graph_replay": round(ms_graph, 3),
            "ms_default_plan": round(ms_default, 3),
            "ms_direct_call_incl_planning": round(ms_direct, 3),
            "autotuned": {"diag_max_w": best[0], "waves_per_cu": best[1], "waves_per_pair": best[2],
                          "tune_s": round(tune_s, 2),
                          "choices_ms": {"%d/%d/%d" % k: round(v, 3) for k, v in sorted(times.items())}},
            "classes": default.classes()}


def extra_fwd_bwd(dev, reps=5):
    """DTW as a loss: 256 pairs of length 512, d = 12, window 10%: forward
    recording the argmin codes, then the adjoint backward."""
    import torch
    from paper_2101_07731_amd import pairs, synth
    x, y = synth.loss_pairs()
    X, Y = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    B, T = x.shape[0], x.shape[1]
    g = torch.ones(B, device=dev)

    def step():
        _, saved = pairs.banded(X, Y, frac=(1, 10), save=True)
        pairs.backward(X, Y, saved, g, frac=(1, 10))

    ms_fb = _events_ms(step, reps)
    ms_f = _events_ms(lambda: pairs.banded(X, Y, frac=(1, 10)), reps)
    return {"workload": "256 pairs, length 512, d=12, window 10% (W=51)",
            "fwd_bwd_pairs_per_s": round(B / (ms_fb * 1e-3), 1),
            "fwd_pairs_per_s": round(B / (ms_f * 1e-3), 1),
            "ms_fwd_bwd": round(ms_fb, 3), "ms_fwd": round(ms_f, 3),
            "fwd_gcups": round(B * band_cells(T, T, T // 10) / (ms_f * 1e-3) / 1e9, 2)}


def extra_ragged_banks(dev, reps=2):
    """256 queries of uneven length and d searching one of five banks (d in
    {2,4,8,16,32}, 4096 references of lengths U[64, 2048] each), window 10%
    of the longer series: the five banks in one index and one search call
    (each stage one launch over every query), beside one call per bank."""
    import torch
    from paper_2101_07731_amd import search, synth
    banks, queries = synth.ragged_banks()
    work = []
    for D, refs in banks.items():
        Q = [torch.from_numpy(q).to(dev) for d, q in queries if d == D]
        if not Q:
            continue
        ix = search.Index([torch.from_numpy(c).to(dev) for c in refs])
        work.append((D, ix, Q))
    st_all = {}

    def run():
        for D, ix, Q in work:
            st_all[D] = search.knn(ix, Q, frac=(1, 10), bounds="mv", stats=True)[2]

    ms = _events_ms(run, reps)
    pairs = sum(s["pairs"] for s in st_all.values())
    started = sum(s["dtw_started"] for s in st_all.values())
    cells = sum(s["cells"] for s in st_all.values())
    # the five banks in one index and all queries (mixed d) in one call: every stage one launch
    refs_all = [torch.from_numpy(c).to(dev) for D in sorted(banks) for c in banks[D]]
    ix_all = search.Index(refs_all)
    del refs_all
    Qall = [torch.from_numpy(q).to(dev) for _, q in queries]
    st1 = {}

    def run_one():
        st1.update(search.knn(ix_all, Qall, frac=(1, 10), bounds="mv", stats=True)[2])

    ms1 = _events_ms(run_one, reps)
    return {"workload": "256 queries, 5 banks (d in {2,4,8,16,32}) of 4096 references, lengths U[64,2048], window 10%",
            "queries_per_s": round(len(queries) / (ms1 * 1e-3), 2), "ms": round(ms1, 3),
            "pct_dtw_pruned": round(100.0 * (1 - st1["dtw_started"] / st1["pairs"]), 3),
            "gcups_dtw": round(st1["cells"] / (ms1 * 1e-3) / 1e9, 2),
            "stage_ms": {n: round(v, 4) for n, v in zip(STAGES, st1["stage_ms"])},
            "one_call_per_bank": {"queries_per_s": round(len(queries) / (ms * 1e-3), 2), "ms": round(ms, 3),
                                  "pct_dtw_pruned": round(100.0 * (1 - started / pairs), 3),
                                  "gcups_dtw": round(cells / (ms * 1e-3) / 1e9, 2),
                                  "per_bank_ms": {str(D): round(st_all[D]["stage_ms"][7], 3) for D in st_all},
                                  "stage_ms_sum": {n: round(sum(st_all[D]["stage_ms"][i] for D in st_all), 4)
                                                   for i, n in enumerate(STAGES)}}}


def extra_lb_mv_streaming(dev, reps=5):
    """LB_MV in the streaming regime (queries arriving one at a time, Sec. 7.1):
    1 and 8 queries against 40000 references of length 256, d = 8 (328 MB of
    element-major candidate tiles, more than the 256 MB Infinity Cache), as
    HBM bytes of the candidate tiles per second."""
    import torch
    from paper_2101_07731_amd import search, synth
    Q, Cs = synth.cascade_knn(nq=8, nc=40000, T=256, D=8, seed=7)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    del Cs
    out = {"workload": "LB_MV, 40000 references x 256 x 8 float32 (328 MB tiles), window 10%"}
    tile_bytes = 40000 * 256 * 8 * 4
    for nq in (1, 8):
        Qd = torch.from_numpy(Q[:nq]).to(dev)
        ms = _events_ms(lambda: search.lower_bounds(ix, Qd, kind="mv", frac=(1, 10)), reps)
        out["queries_%d" % nq] = {"ms": round(ms, 4), "GB_per_s": round(tile_bytes / (ms * 1e-3) / 1e9, 1),
                                  "frac_of_8TB_s": round(tile_bytes / (ms * 1e-3) / 8e12, 3)}
    return out


def extra_long_knn(dev, reps=3):
    """200 queries x 2000 references, length 1024, d = 16, window 10% (row mapping)."""
    import torch
    from paper_2101_07731_amd import search, synth
    Q, Cs = synth.long_knn()
    Qd, Cd = torch.from_numpy(Q).to(dev), torch.from_numpy(Cs).to(dev)
    ix = search.Index(Cd)
    out = {"workload": "200 x 2000, length 1024, d=16, window 10% (W=102)"}
    runs = [("mv", "mv", {}), ("plain", "plain", {})]
    # the point-clustering bound (Sec. 5) at K = 4 and 16 boxes per expanded window, Lv = 2
    for K in (4, 16):
        for e in (0.1, 0.5):
            runs.append(("mv+pc K=%d e=%g" % (K, e), "mv+pc", dict(pc_clusters=K, trigger_pc=e)))
    # the triangle bound (Sec. 4, P = 5 with TOP; the column mapping of bands wider than 63)
    runs.append(("mv+ti e=0.1", "mv+ti", dict(trigger_ti=0.1)))
    runs.append(("mv+pc+ti K=16", "mv+pc+ti", dict(pc_clusters=16, trigger_pc=0.1, trigger_ti=0.1)))
    for name, bounds, kw in runs:
        st = {}

        def run(bounds=bounds, kw=kw, st=st):
            st.update(search.knn(ix, Qd, frac=(1, 10), bounds=bounds, stats=True, **kw)[2])

        ms = _events_ms(run, reps)
        out[name] = {"queries_per_s": round(Q.shape[0] / (ms * 1e-3), 1), "ms": round(ms, 3),
                     "pct_dtw_pruned": round(100 * (1 - st["dtw_started"] / st["pairs"]), 3),
                     "pruned_mv": st["pruned_mv"], "pruned_pc": st["pruned_pc"], "pruned_ti": st["pruned_ti"],
                     "dtw_gcups": round(st["cells"] / (st["stage_ms"][5] * 1e-3) / 1e9, 2),
                     "stage_ms": {n: round(v, 4) for n, v in zip(STAGES, st["stage_ms"])}}
        if "ti" in bounds:
            # per-pair cost of LB_TI against the survivors' DTW (seeds, 4 per query, run apart)
            us_ti = st["lb_ti_ms"] * 1e3 / max(1, st["evaluated_ti"])
            us_dtw = st["stage_ms"][5] * 1e3 / max(1, st["dtw_started"] - 4 * Q.shape[0])
            out[name].update({"evaluated_ti": st["evaluated_ti"], "stage_ms_lb_ti": round(st["lb_ti_ms"], 3),
                              "lb_ti_per_pair_vs_dtw": round(us_ti / us_dtw, 3)})
    return out


def extra_cascade_setup(dev, ix, Qd, T, reps=3):
    """TC-DTW as the paper runs it (Sec. 6, Sec. 7.1): the bounds and their
    parameters chosen at setup time on a sample of queries (search.tune_cascade
    over the paper's grids), then the whole workload searched with that
    choice, beside LB_MV alone and the plain method.  For the benchmark
    workload at windows 5, 10 and 20% and for the long workload (K = 4 and
    16 boxes).  The paper's Table 3 ratios (CPU, UEA data) are context only."""
    import torch
    from paper_2101_07731_amd import search, synth

    def run_one(index, Q, nsample, **kw):
        best, times = search.tune_cascade(index, Q[:nsample], **kw)
        res = {"setup_sample_queries": nsample, "best": search.choice_name(best),
               "setup_ms_per_choice": {k: round(v, 3) for k, v in times.items()}}
        for name, args in (("tc_dtw", dict(kw, **best)), ("lb_mv", dict(kw, bounds="mv")),
                           ("plain", dict(kw, bounds="plain"))):
            st = {}

            def run(args=args, st=st):
                st.update(search.knn(index, Q, stats=True, **args)[2])

            ms = _events_ms(run, reps if name != "plain" else 1)
            res[name] = {"queries_per_s": round(Q.shape[0] / (ms * 1e-3), 2), "ms": round(ms, 3),
                         "pct_dtw_pruned": round(100.0 * (1 - st["dtw_started"] / st["pairs"]), 3),
                         "pruned": {"mv": st["pruned_mv"], "pc": st["pruned_pc"], "ti": st["pruned_ti"]}}
        res["speedup_tc_dtw_vs_plain"] = round(res["plain"]["ms"] / res["tc_dtw"]["ms"], 3)
        res["speedup_lb_mv_vs_plain"] = round(res["plain"]["ms"] / res["lb_mv"]["ms"], 3)
        return res

    out = {"paper_table3_context": "CPU, UEA data, W = 20: LB_MV 5.88x, TC-DTW 8.06x over the plain "
                                   "method; 51% / 63% of DTWs skipped (AMD Opteron)"}
    for fw in ((1, 20), (1, 10), (1, 5)):
        out["benchmark_W%d" % min(T * fw[0] // fw[1], T - 1)] = run_one(ix, Qd, 100, frac=fw)
    Q, Cs = synth.long_knn()
    ixl = search.Index(torch.from_numpy(Cs).to(dev))
    Ql = torch.from_numpy(Q).to(dev)
    for K in (4, 16):
        out["long_K%d" % K] = run_one(ixl, Ql, 40, frac=(1, 10), pc_clusters=K)
    return out


def extra_small_graph(dev, reps=50):
    """The small workload (64 queries x 256 references, length 64, d = 3, W = 6), whose call is
    bound by launches and host work: whole searches replayed from a HIP graph
    (search.GraphedSearch) against eager calls, LB_MV and no bounds; the replays' neighbours must
    equal the eager ones."""
    import numpy as np
    import torch
    from paper_2101_07731_amd import search, synth
    gen_kw, frac, _ = WORKLOADS["plain"]
    Q, Cs = synth.plain_knn(**gen_kw)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    Qd = torch.from_numpy(Q).to(dev)
    out = {"workload": WORKLOADS["plain"][2]}
    for b in ("mv", "plain"):
        kw = dict(frac=frac, bounds=b)
        wsb = search.knn_workspace_bytes(ix, Qd, **kw)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        ei, ed = search.knn(ix, Qd, workspace=ws, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            search.knn(ix, Qd, workspace=ws, **kw)
        torch.cuda.synchronize()
        eager_ms = (time.perf_counter() - t0) * 1e3 / reps
        try:
            g = search.GraphedSearch(ix, Qd, **kw)
        except Exception as err:   # a search that cannot be captured is reported, not timed
            out[b] = {"eager_ms": round(eager_ms, 4), "graph_error": str(err)}
            continue
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / reps
        gi, gd = g.replay()
        torch.cuda.synchronize()
        same = bool(np.array_equal(gi.cpu().numpy(), ei.cpu().numpy()) and
                    np.array_equal(gd.cpu().numpy(), ed.cpu().numpy()))
        out[b] = {"eager_ms": round(eager_ms, 4), "graph_ms": round(graph_ms, 4),
                  "eager_queries_per_s": round(Qd.shape[0] / eager_ms * 1e3, 1),
                  "graph_queries_per_s": round(Qd.shape[0] / graph_ms * 1e3, 1), "same_result": same}
    return out


def extra_trajectories(dev, reps=3):
    """Trajectory 1-NN (synth.trajectory_knn: 1000 queries x 10000 references,
    length 182, d = 3, window 10%), data on which the point-clustering bound
    (Sec. 5) prunes pairs that LB_MV cannot: LB_MV alone, each advanced bound
    behind it at the default triggers, the setup-stage choice (Sec. 6) made on
    100 queries, and the plain method, with the pairs each bound pruned."""
    import torch
    from paper_2101_07731_amd import search, synth
    Q, Cs = synth.trajectory_knn()
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    Qd = torch.from_numpy(Q).to(dev)
    out = {"workload": "1000 x 10000, length 182, d=3, 20 classes of smooth curves, noise 0.5, window 10% (W=18)",
           "paper_table3_context": "CPU, UEA Charactertrajectories (d = 3, length 182), W = 20: LB_MV 16.98x / "
                                   "89% of DTWs skipped, TC-DTW 25.31x / 99% over the plain method"}
    best, _ = search.tune_cascade(ix, Qd[:100], frac=(1, 10))
    out["setup_choice"] = search.choice_name(best)
    runs = [("plain", dict(bounds="plain")), ("mv", dict(bounds="mv")), ("mv+pc", dict(bounds="mv+pc")),
            ("mv+ti", dict(bounds="mv+ti")), ("mv+pc+ti", dict(bounds="mv+pc+ti")), ("setup_choice", best)]
    for name, kw in runs:
        st = {}

        def run(kw=kw, st=st):
            st.update(search.knn(ix, Qd, frac=(1, 10), stats=True, **kw)[2])

        ms = _events_ms(run, reps if name != "plain" else 1)
        out[name] = {"queries_per_s": round(Q.shape[0] / (ms * 1e-3), 1), "ms": round(ms, 3),
                     "pct_dtw_pruned": round(100 * (1 - st["dtw_started"] / st["pairs"]), 3),
                     "pruned": {"mv": st["pruned_mv"], "pc": st["pruned_pc"], "ti": st["pruned_ti"]},
                     "evaluated": {"pc": st["evaluated_pc"], "ti": st["evaluated_ti"]},
                     "stage_ms": {n: round(v, 4) for n, v in zip(STAGES, st["stage_ms"])}}
    for name in ("mv+pc", "mv+pc+ti", "setup_choice"):
        out["speedup_%s_vs_mv" % name] = round(out["mv"]["ms"] / out[name]["ms"], 3)
    out["speedup_mv_vs_plain"] = round(out["plain"]["ms"] / out["mv"]["ms"], 3)
    out["speedup_setup_choice_vs_plain"] = round(out["plain"]["ms"] / out["setup_choice"]["ms"], 3)
    return out


def cpu_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the search has no multi-GPU path "
              "(a query batch would be split across GPUs, each holding a full index copy); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2101_07731_amd import search, synth

    gen_kw, frac, desc = WORKLOADS[args.workload]
    if args.frac:
        a, b = args.frac.split("/")
        frac = (int(a), int(b))
    gen = synth.cascade_knn if args.workload == "cascade" else synth.plain_knn
    Q, Cs = gen(**gen_kw)
    dev = torch.device("cuda:0")
    Qd = torch.from_numpy(Q).to(dev)
    Cd = torch.from_numpy(Cs).to(dev)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    ix = search.Index(Cd)
    torch.cuda.synchronize()
    index_ms = (time.perf_counter() - t0) * 1e3

    kw = dict(frac=frac, bounds=args.bounds)
    wsb = search.knn_workspace_bytes(ix, Qd, **kw)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        search.knn(ix, Qd, stats=True, workspace=ws, **kw)
    torch.cuda.synchronize()

    steps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        idx, dist, st = search.knn(ix, Qd, stats=True, workspace=ws, **kw)
        steps.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    note("%d timed steps" % args.steps)

    nq, nc, T, D = Q.shape[0], Cs.shape[0], Q.shape[1], Q.shape[2]
    W = min(max(T * frac[0] // frac[1], 0), T - 1)
    band = sum(min(T - 1, i + W) - max(0, i - W) + 1 for i in range(T))
    ms_step = wall * 1e3 / args.steps
    qps = nq / (wall / args.steps)
    st = steps[-1]
    dtw_ms = float(np.mean([s["stage_ms"][5] for s in steps]))
    cells = float(np.mean([s["cells"] for s in steps]))
    flops_per_cell = 3 * D + 3
    achieved_gcells = cells / (dtw_ms * 1e-3) / 1e9
    achieved_tflops = achieved_gcells * 1e9 * flops_per_cell / 1e12
    peak_tflops = FP32_PEAK_FLOPS / 1e12
    traffic, traffic_src = measured_traffic()
    if not (args.workload == "cascade" and W == 25 and args.bounds == "mv"):
        traffic, traffic_src = None, "counters taken on the 1000 x 10000, W = 25, LB_MV workload only"
    pruned = 1.0 - st["dtw_started"] / st["pairs"]

    out = {
        "metric": "1-NN queries/s + banded-DTW GCUPS, % DTW pruned; batched & fwd+bwd pairs/s",
        "value": round(qps, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "queries": nq, "references": nc, "length": T, "d": D,
                   "window": W, "bounds": args.bounds, "parallelism": "single GPU"},
        "gcups_effective": round(nq * nc * band / (wall / args.steps) / 1e9, 2),
        "gcups_dtw_kernel": round(achieved_gcells, 2),
        "pct_dtw_pruned": round(100.0 * pruned, 3),
        "pct_dtw_abandoned_of_started": round(100.0 * st["dtw_abandoned"] / max(1, st["dtw_started"]), 3),
        "rescored": st["rescored"],
        "stage_ms": {k: round(float(np.mean([s["stage_ms"][i] for s in steps])), 4)
                     for i, k in enumerate(["prep", "lb_mv", "seed", "compact", "lb_pc_ti", "dtw",
                                            "finalize", "total"])},
        "index_build_ms": round(index_ms, 3),
        "roofline": {
            "kernel": "k_knn_dtw_ring" if W <= 63 else "k_knn_dtw_rows",
            "bound": "alu",
            "achieved": round(achieved_tflops, 3),
            "peak": round(peak_tflops, 1),
            "unit": "TFLOP/s",
            "frac": round(achieved_tflops / peak_tflops, 4),
            # HBM-side bytes per survivor launch from the FETCH_SIZE / WRITE_SIZE passes, calibrated
            # on the index copy kernel; null once the kernel's sources differ from the profiled build
            "traffic": traffic,
            "traffic_source": traffic_src,
            "per_unit": "%d flops per band cell (d subtractions, d squares accumulated by fused "
                        "multiply-add, a 3-way min counted as 2, an add); %.1f G cells/s" %
                        (flops_per_cell, achieved_gcells),
            "single_issue_frac": round(achieved_gcells * (2 * D + 2) * 1e9 / VALU_LANE_OPS, 4),
        },
    }

    extras = set() if args.no_extras else set(DEFAULT_EXTRAS)
    if args.extras is not None:
        extras |= set(args.extras or EXTRAS)
    if "windows" in extras:
        note("windows")
        # the same workload at windows 5% and 20% (W = 12 and 51), LB_MV, one search call per step
        wres = {}
        for fw in ((1, 20), (1, 5)):
            kww = dict(frac=fw, bounds=args.bounds)
            wsw = torch.empty(search.knn_workspace_bytes(ix, Qd, **kww), dtype=torch.uint8, device=dev)
            stw = {}

            def runw(kww=kww, wsw=wsw, stw=stw):
                stw.update(search.knn(ix, Qd, stats=True, workspace=wsw, **kww)[2])

            msw = _events_ms(runw, 5)
            Ww = min(T * fw[0] // fw[1], T - 1)
            wres["W%d" % Ww] = {"queries_per_s": round(nq / (msw * 1e-3), 2), "ms": round(msw, 3),
                                "pct_dtw_pruned": round(100.0 * (1 - stw["dtw_started"] / stw["pairs"]), 3),
                                "dtw_gcups": round(stw["cells"] / (stw["stage_ms"][5] * 1e-3) / 1e9, 2),
                                "stage_ms": {n: round(v, 4) for n, v in zip(STAGES, stw["stage_ms"])}}
        out["windows"] = wres
    if "full_cascade" in extras:
        note("full_cascade")
        kwf = dict(frac=frac, bounds="mv+pc+ti")
        search.knn(ix, Qd, **kwf)
        stf = {}

        def full():
            stf.update(search.knn(ix, Qd, stats=True, **kwf)[2])

        msf = _events_ms(full, 3)
        # per-pair costs in this search: LB_PC (its stage less the LB_TI launch), LB_TI, and the
        # survivors' DTW (the seeds, seed_r = 4 per query, run in their own stage)
        dtw_pairs = max(1, stf["dtw_started"] - 4 * nq)
        us_pc = (stf["stage_ms"][4] - stf["lb_ti_ms"]) * 1e3 / max(1, stf["evaluated_pc"])
        us_ti = stf["lb_ti_ms"] * 1e3 / max(1, stf["evaluated_ti"])
        us_dtw = stf["stage_ms"][5] * 1e3 / dtw_pairs
        out["full_cascade"] = {"bounds": "mv+pc+ti", "queries_per_s": round(nq / (msf * 1e-3), 2),
                               "pruned_pc": stf["pruned_pc"], "pruned_ti": stf["pruned_ti"],
                               "pct_dtw_pruned": round(100.0 * (1 - stf["dtw_started"] / stf["pairs"]), 3),
                               "stage_ms_lb_pc_ti": round(stf["stage_ms"][4], 3),
                               "stage_ms_lb_ti": round(stf["lb_ti_ms"], 3),
                               "evaluated_pc": stf["evaluated_pc"], "evaluated_ti": stf["evaluated_ti"],
                               "dtw_pairs": dtw_pairs,
                               "ns_per_pair": {"lb_pc": round(us_pc * 1e3, 3), "lb_ti": round(us_ti * 1e3, 3),
                                               "dtw": round(us_dtw * 1e3, 3)},
                               "per_pair_vs_dtw": {"lb_pc": round(us_pc / us_dtw, 3),
                                                   "lb_ti": round(us_ti / us_dtw, 3)}}
    if "cand_boxes" in extras:
        note("cand_boxes")
        # LB_PC (e = 0.5, so that it runs on more pairs) with the query's boxes built per query
        # (Sec. 5) against the candidates' boxes built once per index (Sec. 8, roles swapped)
        kwp = dict(frac=frac, bounds="mv+pc", trigger_pc=0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cb = search.CandBoxes(ix, T, frac=frac)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        res = {}
        for name, extra in (("query_boxes", {}), ("candidate_boxes", {"pc_cand": cb})):
            search.knn(ix, Qd, **kwp, **extra)
            stc = {}

            def run_pc(extra=extra, stc=stc):
                stc.update(search.knn(ix, Qd, stats=True, **kwp, **extra)[2])

            msc = _events_ms(run_pc, 3)
            res[name] = {"queries_per_s": round(nq / (msc * 1e-3), 2), "pruned_pc": stc["pruned_pc"],
                         "stage_ms_prep": round(stc["stage_ms"][0], 3),
                         "stage_ms_lb_pc": round(stc["stage_ms"][4], 3)}
        out["cand_boxes"] = {"bounds": "mv+pc", "trigger_pc": 0.5, "build_ms": round(build_ms, 3),
                             "bytes": int(cb.buf.numel()), **res}
    if "knn_k10" in extras:
        note("knn_k10")
        # the 10 nearest neighbours of every query (same workload and bounds)
        st10 = {}

        def k10():
            st10.update(search.knn(ix, Qd, stats=True, k=10, **kw)[2])

        ms10 = _events_ms(k10, 3)
        out["knn_k10"] = {"queries_per_s": round(nq / (ms10 * 1e-3), 2), "ms": round(ms10, 3),
                          "pct_dtw_pruned": round(100.0 * (1 - st10["dtw_started"] / st10["pairs"]), 3),
                          "rescored": st10["rescored"],
                          "stage_ms": {n: round(v, 4) for n, v in zip(STAGES, st10["stage_ms"])}}
    if "knn_independent" in extras:
        note("knn_independent")
        # independent DTW (Sec. 2 DTW_I) on the same workload, LB_MV bounds
        sti = {}

        def indep():
            sti.update(search.knn(ix, Qd, stats=True, independent=1, **kw)[2])

        msi = _events_ms(indep, 3)
        out["knn_independent"] = {"queries_per_s": round(nq / (msi * 1e-3), 2), "ms": round(msi, 3),
                                  "pct_dtw_pruned": round(100.0 * (1 - sti["dtw_started"] / sti["pairs"]), 3),
                                  "dtw_gcups": round(sti["cells"] / (sti["stage_ms"][5] * 1e-3) / 1e9, 2),
                                  "stage_ms": {n: round(v, 4) for n, v in zip(STAGES, sti["stage_ms"])}}
    if "single_query_latency" in extras:
        note("single_query_latency")
        # queries arriving one at a time (Sec. 7.1): one tc_dtw_knn call per query against the
        # same index; GPU time from events around each call, wall time including the host side
        ws1 = torch.empty(search.knn_workspace_bytes(ix, Qd[:1], **kw), dtype=torch.uint8, device=dev)
        for i in range(5):
            search.knn(ix, Qd[i:i + 1], workspace=ws1, **kw)
        torch.cuda.synchronize()
        gpu_ms, wall_ms = [], []
        for i in range(100):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record()
            search.knn(ix, Qd[i:i + 1], workspace=ws1, **kw)
            e1.record()
            e1.synchronize()
            wall_ms.append((time.perf_counter() - t0) * 1e3)
            gpu_ms.append(e0.elapsed_time(e1))
        stg = []
        for i in range(20):
            stg.append(search.knn(ix, Qd[i:i + 1], workspace=ws1, stats=True, **kw)[2]["stage_ms"])
        out["single_query_latency"] = {
            "queries": 100, "references": int(ix.count),
            "stage_ms_mean": {n: round(float(np.mean([x[j] for x in stg])), 4) for j, n in enumerate(STAGES)},
            "gpu_ms_p50": round(float(np.percentile(gpu_ms, 50)), 4),
            "gpu_ms_p99": round(float(np.percentile(gpu_ms, 99)), 4),
            "wall_ms_p50": round(float(np.percentile(wall_ms, 50)), 4),
            "wall_ms_p99": round(float(np.percentile(wall_ms, 99)), 4)}
    if "cascade_setup" in extras:
        note("cascade_setup")
        out["cascade_setup"] = extra_cascade_setup(dev, ix, Qd, T)
    for name, fn in (("batched_pairs", extra_batched_pairs), ("dtw_loss", extra_fwd_bwd),
                     ("long_knn", extra_long_knn), ("ragged_banks", extra_ragged_banks),
                     ("lb_mv_streaming", extra_lb_mv_streaming), ("trajectories", extra_trajectories),
                     ("small_graph", extra_small_graph)):
        if name in extras:
            note(name)
            out[name] = fn(dev)
    if "plain_gpu" in extras:
        note("plain_gpu")
        # the plain method (Sec. 7.2's "default windowed DTW": every DTW computed, no bounds, no
        # abandoning) on the same GPU: the whole batch in one call, and one call per query
        kwp = dict(frac=frac, bounds="plain")
        search.knn(ix, Qd, **kwp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, sp = search.knn(ix, Qd, stats=True, **kwp)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        nper = min(50, nq)
        wsp = torch.empty(search.knn_workspace_bytes(ix, Qd[:1], **kwp), dtype=torch.uint8, device=dev)
        search.knn(ix, Qd[:1], workspace=wsp, **kwp)
        ms_per_query = _events_ms(lambda: [search.knn(ix, Qd[i:i + 1], workspace=wsp, **kwp)
                                           for i in range(nper)], 1) / nper
        out["plain_gpu"] = {"queries_per_s": round(nq / tp, 2),
                            "dtw_kernel_gcups": round(sp["cells"] / (sp["stage_ms"][5] * 1e-3) / 1e9, 2),
                            "cascade_speedup": round(tp / (wall / args.steps), 3),
                            "one_query_per_call_queries_per_s": round(1e3 / ms_per_query, 2),
                            "cascade_speedup_vs_one_query_per_call": round(ms_per_query * nq / ms_step, 3)}

    if not args.no_cpu:
        note("cpu_baseline")
        import oracle as O
        nsamp = min(args.cpu_queries, nq)
        th = cpu_threads()
        gi, gd = idx.cpu().numpy(), dist.cpu().numpy()
        t0 = time.perf_counter()
        ri, rd = O.knn_exhaustive(Q[:nsamp], Cs, num=frac[0], den=frac[1], threads=th)
        tc = time.perf_counter() - t0
        ok = bool(np.array_equal(ri, gi[:nsamp]) and np.array_equal(rd.astype(np.float32), gd[:nsamp]))
        out["cpu_baseline"] = {"value": round(nsamp / tc, 3), "unit": "queries/s", "cores": th,
                               "kind": "oracle",
                               "sample": "first %d of %d queries against all %d references, exhaustive "
                                         "FP64 banded DTW (%.1f s)" % (nsamp, nq, nc, tc),
                               "matches_gpu": ok}
        # the oracle's sequential cascade (the paper's CPU method, Sec. 6 and 7.1: LB_MV, then LB_PC
        # and LB_TI behind their triggers, DTW with row-wise early abandoning) beside its exhaustive
        # search, on all the cores used above and on one core: the paper's speedup T(default) / T(X)
        # and share of skipped DTWs on this data
        note("cpu_cascade")
        n1 = min(8, nq)
        cpu = {"cores_all": th, "sample_all_cores": nsamp, "sample_one_core": n1}
        t0 = time.perf_counter()
        O.knn_exhaustive(Q[:n1], Cs, num=frac[0], den=frac[1], threads=1)
        t_ex1 = time.perf_counter() - t0
        cpu["exhaustive"] = {"all_cores_queries_per_s": round(nsamp / tc, 3),
                             "one_core_queries_per_s": round(n1 / t_ex1, 3)}
        for name, bits in (("LB_MV", 0), ("LB_MV+LB_PC+LB_TI", 6)):
            rec = {}
            for label, nqs, thr in (("all_cores", nsamp, th), ("one_core", n1, 1)):
                t0 = time.perf_counter()
                ci, cd, cs = O.knn_cascade(Q[:nqs], Cs, num=frac[0], den=frac[1], bounds=bits, threads=thr)
                tcs = time.perf_counter() - t0
                if not (np.array_equal(ci, ri[:nqs]) and np.array_equal(cd, rd[:nqs])):
                    raise AssertionError("the oracle's cascade differs from its exhaustive search")
                rec[label + "_queries_per_s"] = round(nqs / tcs, 3)
                if label == "all_cores":
                    pairs_ = float(cs["pairs"].sum())
                    rec["pct_dtw_skipped"] = round(100.0 * (1 - cs["dtw_started"].sum() / pairs_), 3)
                    rec["skipped_by"] = {"mv": int(cs["pruned_mv"].sum()), "pc": int(cs["pruned_pc"].sum()),
                                         "ti": int(cs["pruned_ti"].sum())}
                    rec["speedup_vs_exhaustive_all_cores"] = round(tc / tcs, 3)
                else:
                    rec["speedup_vs_exhaustive_one_core"] = round(t_ex1 / tcs, 3)
            cpu[name] = rec
        out["cpu_cascade"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
