"""Benchmark of the 1-NN DTW search with the lower-bound cascade on one MI355X.

One step = one tc_dtw_knn call over the whole query batch (query
envelopes, LB_MV, best-so-far seeding, compaction, advanced bounds when
enabled, DTW of the survivors with early abandoning, float64 re-scoring of
near-tie finalists).  Inputs and the candidate index are resident in HBM
before the timed region; the index build is timed separately.

Prints one JSON line ("Measurement") with:
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
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (generator kwargs, window fraction, description)
    "cascade": (dict(nq=1000, nc=10000, T=256, D=8), (1, 10),
                "pruned 1-NN: 1000 queries x 10000 references, length 256, d=8, "
                "correlated walks with 8 warped prototypes, window 10% (W=25)"),
    "plain": (dict(nq=64, nc=256, T=64, D=3), (1, 10),
              "plain 1-NN: 64 queries x 256 references, length 64, d=3, random walks, window 10% (W=6)"),
}

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cascade", choices=sorted(WORKLOADS))
    ap.add_argument("--bounds", default="mv")
    ap.add_argument("--frac", default=None, help="window fraction num/den, e.g. 1/10")
    ap.add_argument("--cpu-queries", type=int, default=24, help="queries in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extras", action="store_true", help="also time the plain GPU search")
    return ap.parse_args()


def cpu_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md, 'More than one GPU'); use --gpus 1", file=sys.stderr)
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

    nq, nc, T, D = Q.shape[0], Cs.shape[0], Q.shape[1], Q.shape[2]
    W = min(max(T * frac[0] // frac[1], 0), T - 1)
    band = sum(min(T - 1, i + W) - max(0, i - W) + 1 for i in range(T))
    ms_step = wall * 1e3 / args.steps
    qps = nq / (wall / args.steps)
    st = steps[-1]
    dtw_ms = float(np.mean([s["stage_ms"][5] for s in steps]))
    cells = float(np.mean([s["cells"] for s in steps]))
    alu_ops_per_cell = 2 * D + 2
    peak_gcells = VALU_LANE_OPS / alu_ops_per_cell / 1e9
    achieved_gcells = cells / (dtw_ms * 1e-3) / 1e9
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
            "kernel": "k_knn_dtw_diag" if W <= 63 else "k_knn_dtw_rows",
            "bound": "alu",
            "achieved": round(achieved_gcells, 2),
            "peak": round(peak_gcells, 2),
            "unit": "Gcell/s",
            "frac": round(achieved_gcells / peak_gcells, 4),
            "traffic": None,
            "per_unit": "%d VALU lane-ops per band cell (d subtractions, d fused multiply-adds, "
                        "a 3-way min, an add)" % alu_ops_per_cell,
        },
    }

    if args.extras:
        kwp = dict(frac=frac, bounds="plain")
        search.knn(ix, Qd, **kwp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, sp = search.knn(ix, Qd, stats=True, **kwp)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        out["plain_gpu"] = {"queries_per_s": round(nq / tp, 2),
                            "dtw_kernel_gcups": round(sp["cells"] / (sp["stage_ms"][5] * 1e-3) / 1e9, 2),
                            "cascade_speedup": round(tp / (wall / args.steps), 3)}

    if not args.no_cpu:
        import oracle as O
        nsamp = min(args.cpu_queries, nq)
        th = cpu_threads()
        t0 = time.perf_counter()
        ri, rd = O.knn_exhaustive(Q[:nsamp], Cs, num=frac[0], den=frac[1], threads=th)
        tc = time.perf_counter() - t0
        ok = bool(np.array_equal(ri, idx.cpu().numpy()[:nsamp]) and
                  np.array_equal(rd.astype(np.float32), dist.cpu().numpy()[:nsamp]))
        out["cpu_baseline"] = {"value": round(nsamp / tc, 3), "unit": "queries/s", "cores": th,
                               "kind": "oracle",
                               "sample": "first %d of %d queries against all %d references, exhaustive "
                                         "FP64 banded DTW (%.1f s)" % (nsamp, nq, nc, tc),
                               "matches_gpu": ok}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
