"""1-NN search and dense lower bounds on the GPU against the FP64 oracle.

Bar: identical nearest-neighbour indices (ties to the lowest index) and
distances equal to the oracle's float64 value rounded to float32 (the
finalists are re-scored in float64 in the oracle's operation order).
Bounds: never above the oracle's FP64 bound (they are rounded down) and
within the documented deflation (n*D + 4) 2^-24 of it.
"""
import sys

import numpy as np
import pytest

import oracle as O
from ti_allowance import ti_lower_allowance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_07731_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


def run_knn(dev, Q, Cs, **kw):
    from paper_2101_07731_amd import search
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    idx, dist, st = search.knn(ix, torch.from_numpy(Q).to(dev), stats=True, **kw)
    return idx.cpu().numpy(), dist.cpu().numpy(), st


def check_against_oracle(idx, dist, Q, Cs, num, den):
    ri, rd = O.knn_exhaustive(Q, Cs, num=num, den=den)
    np.testing.assert_array_equal(idx, ri)
    np.testing.assert_array_equal(dist, rd.astype(np.float32))


def test_plain_config_shape(dev):
    """Plain 1-NN: 64 queries x 256 references, length 64, d=3, window 10%."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.plain_knn()
    for bounds in ("plain", "mv"):
        say("knn plain shape", bounds)
        idx, dist, st = run_knn(dev, Q, Cs, frac=(1, 10), bounds=bounds)
        check_against_oracle(idx, dist, Q, Cs, 1, 10)
        assert st["pairs"] == 64 * 256
        if bounds == "plain":
            assert st["dtw_started"] == 64 * 256 and st["pruned_mv"] == 0
        else:
            assert st["pruned_mv"] + st["dtw_started"] == 64 * 256


@pytest.mark.parametrize("frac", [(1, 20), (1, 10), (1, 5)])
def test_cascade_prototypes_with_ties(dev, frac):
    """Prototype data (near neighbours exist) plus exact duplicate references
    so that ties must go to the lowest index."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.cascade_knn(nq=40, nc=600, T=96, D=8, seed=21)
    Cs = np.concatenate([Cs, Cs[::7]])                    # duplicates at higher indices
    Q = np.concatenate([Q, Cs[[3, 100, 599]]])            # queries equal to a reference: distance 0
    say("knn cascade", frac, Q.shape, Cs.shape)
    for seed_r in (1, 4, 8):
        idx, dist, st = run_knn(dev, Q, Cs, frac=frac, bounds="mv", seed_r=seed_r)
        check_against_oracle(idx, dist, Q, Cs, *frac)
        assert st["pruned_mv"] + st["dtw_started"] == st["pairs"]
    assert idx[-3] == 3 and dist[-3] == 0.0


@pytest.mark.parametrize("D", [20, 33, 64])
def test_wide_dimensions(dev, D):
    """d > 16: the diagonal kernel runs two rounds per iteration without
    prefetching (six chunks and more); both window parities."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.cascade_knn(nq=6, nc=90, T=48, D=D, seed=27)
    say("knn wide", D)
    for frac in ((1, 10), (1, 9)):     # W = 4 and 5 at length 48
        idx, dist, st = run_knn(dev, Q, Cs, frac=frac, bounds="mv")
        check_against_oracle(idx, dist, Q, Cs, *frac)
        assert st["pruned_mv"] + st["dtw_started"] == st["pairs"]


@pytest.mark.parametrize("k", [2, 5, 16, 32])
def test_k_nearest_against_oracle(dev, k):
    """k > 1: the k nearest in (distance, index) order, with duplicate
    references (ties) and queries equal to a reference, for the plain
    method, LB_MV and the full cascade."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.cascade_knn(nq=10, nc=280, T=64, D=4, seed=28)
    Cs = np.concatenate([Cs, Cs[::9]])
    Q = np.concatenate([Q, Cs[[5, 250]]])
    ri, rd = O.knn_exhaustive_k(Q, Cs, k, num=1, den=10)
    for bounds in ("plain", "mv", "mv+pc+ti"):
        say("knn k", k, bounds)
        idx, dist, st = run_knn(dev, Q, Cs, frac=(1, 10), bounds=bounds, k=k)
        assert idx.shape == (len(Q), k)
        np.testing.assert_array_equal(idx, ri)
        np.testing.assert_array_equal(dist, rd.astype(np.float32))
        assert st["pruned_mv"] + st["pruned_pc"] + st["pruned_ti"] + st["dtw_started"] == st["pairs"]
    assert idx[-2][0] == 5 and dist[-2][0] == 0.0


def test_k_nearest_row_mapping(dev):
    """k > 1 with a band wider than 63 (row-systolic DTW)."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.long_knn(nq=3, nc=40, T=700, D=3, seed=29)
    ri, rd = O.knn_exhaustive_k(Q, Cs, 4, num=1, den=10)
    idx, dist, _ = run_knn(dev, Q, Cs, frac=(1, 10), bounds="mv", k=4)
    np.testing.assert_array_equal(idx, ri)
    np.testing.assert_array_equal(dist, rd.astype(np.float32))


def test_k_nearest_full_size_sampled(dev):
    """k = 10 on the benchmark's workload (1000 x 10000, length 256, d = 8,
    window 10%), sampled queries against the oracle."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.cascade_knn()
    idx, dist, st = run_knn(dev, Q, Cs, frac=(1, 10), bounds="mv", k=10)
    say("knn k=10 full size", st)
    sample = np.array([0, 421, 999])
    ri, rd = O.knn_exhaustive_k(Q[sample], Cs, 10, num=1, den=10)
    np.testing.assert_array_equal(idx[sample], ri)
    np.testing.assert_array_equal(dist[sample], rd.astype(np.float32))
    assert np.all(np.diff(dist, axis=1) >= 0)


@pytest.mark.parametrize("case", [(1, (1, 10)), (3, (1, 9)), (8, (1, 10)), (13, (1, 9))],
                         ids=["d1_W6", "d3_W7", "d8_W6", "d13_W7"])
def test_independent_dtw_against_oracle(dev, case):
    """Independent DTW (DTW_I, Sec. 2): 1 and 3 nearest against the oracle's
    exhaustive DTW_I, plain and with LB_MV, with duplicate references."""
    from paper_2101_07731_amd import synth
    D, frac = case
    Q, Cs = synth.cascade_knn(nq=8, nc=200, T=64, D=D, seed=32)
    Cs = np.concatenate([Cs, Cs[::11]])
    Q = np.concatenate([Q, Cs[[17]]])
    for k in (1, 3):
        ri, rd = O.knn_exhaustive_k(Q, Cs, k, num=frac[0], den=frac[1], independent=True)
        for bounds in ("plain", "mv"):
            say("knn independent", case, k, bounds)
            idx, dist, st = run_knn(dev, Q, Cs, frac=frac, bounds=bounds, k=k, independent=1)
            if k == 1:
                idx, dist = idx[:, None], dist[:, None]
            np.testing.assert_array_equal(idx, ri)
            np.testing.assert_array_equal(dist, rd.astype(np.float32))
            assert st["pruned_mv"] + st["dtw_started"] == st["pairs"]


def test_independent_dtw_full_size_sampled(dev):
    """DTW_I on the benchmark's workload (1000 x 10000, length 256, d = 8,
    W = 25), sampled queries against the oracle."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.cascade_knn()
    idx, dist, st = run_knn(dev, Q, Cs, frac=(1, 10), bounds="mv", independent=1)
    say("knn independent full size", st)
    sample = np.array([3, 500])
    ri, rd = O.knn_exhaustive_k(Q[sample], Cs, 1, num=1, den=10, independent=True)
    np.testing.assert_array_equal(idx[sample], ri[:, 0])
    np.testing.assert_array_equal(dist[sample], rd[:, 0].astype(np.float32))


def test_cascade_repeatable(dev):
    from paper_2101_07731_amd import synth
    Q, Cs = synth.cascade_knn(nq=30, nc=500, T=64, D=4, seed=22)
    a = run_knn(dev, Q, Cs, frac=(1, 10))
    b = run_knn(dev, Q, Cs, frac=(1, 10))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("case", [(5, 60, 700, 3, (1, 10)), (4, 40, 300, 16, (1, 4))],
                         ids=["W70_d3", "W75_d16"])
def test_row_mapping_search(dev, case):
    """Bands wider than 63 use the row-systolic DTW."""
    from paper_2101_07731_amd import synth
    nq, nc, T, D, frac = case
    Q, Cs = synth.long_knn(nq=nq, nc=nc, T=T, D=D, seed=23)
    say("knn rows", case)
    for bounds in ("plain", "mv"):
        idx, dist, _ = run_knn(dev, Q, Cs, frac=frac, bounds=bounds)
        check_against_oracle(idx, dist, Q, Cs, *frac)


def test_unequal_query_and_candidate_lengths(dev):
    rng = np.random.default_rng(24)
    Q = np.cumsum(rng.standard_normal((12, 50, 3)), 1).astype(np.float32)
    Cs = np.cumsum(rng.standard_normal((200, 70, 3)), 1).astype(np.float32)
    idx, dist, _ = run_knn(dev, Q, Cs, window=5, frac=None)
    ri, rd = O.knn_exhaustive(Q, Cs, window=5)
    np.testing.assert_array_equal(idx, ri)
    np.testing.assert_array_equal(dist, rd.astype(np.float32))


@pytest.mark.parametrize("case", [
    (19, 150, 80, 8),   # three query tiles, ten element segments
    (1, 300, 64, 3),    # one query slot, three segments
    (3, 200, 20, 3),    # four query slots, E = 60 (not a multiple of 4), one segment
    (2, 130, 33, 5),    # two query slots, E = 165, two segments, ragged last tile
], ids=lambda c: "nq%d_nc%d_T%d_D%d" % c)
def test_lb_mv_dense_matrix(dev, case):
    from paper_2101_07731_amd import search, synth
    nq, nc, T, D = case
    Q, Cs = synth.cascade_knn(nq=nq, nc=nc, T=T, D=D, seed=25)
    say("lb_mv dense", case)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    lb = search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="mv", frac=(1, 10)).cpu().numpy()
    W = O.window_eff(T, T, 0, 1, 10)
    ref = np.array([[O.lb_mv(q, c, W) for c in Cs] for q in Q])
    assert np.all(lb.astype(np.float64) <= ref * (1 + 1e-12))
    # deflation (E+3) u plus the float32 accumulation error (at most E+2 roundings), E = n*D
    slack = 2 * (T * D + 4) * 2.0 ** -24 * 1.01 + 2e-7
    assert np.all(lb.astype(np.float64) >= ref * (1 - slack) - 1e-30)
    # the same matrix again: the segment sums are added in a fixed order
    lb2 = search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="mv", frac=(1, 10)).cpu().numpy()
    np.testing.assert_array_equal(lb, lb2)


def test_lb_mv_streaming_size_sampled(dev):
    """LB_MV at the streaming size (40000 references of length 256, d = 8,
    one and eight queries, the launch the streaming benchmark times):
    sampled columns against the oracle."""
    from paper_2101_07731_amd import search, synth
    Q, Cs = synth.cascade_knn(nq=8, nc=40000, T=256, D=8, seed=7)
    say("lb_mv streaming size", Cs.shape)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    W = O.window_eff(256, 256, 0, 1, 10)
    cols = np.random.default_rng(5).choice(40000, 64, replace=False)
    cols = np.concatenate([cols, [0, 63, 64, 39999]])
    slack = 2 * (256 * 8 + 4) * 2.0 ** -24 * 1.01 + 2e-7
    for nq in (1, 8):
        lb = search.lower_bounds(ix, torch.from_numpy(Q[:nq]).to(dev), kind="mv", frac=(1, 10)).cpu().numpy()
        ref = np.array([[O.lb_mv(q, Cs[c], W) for c in cols] for q in Q[:nq]])
        got = lb[:, cols].astype(np.float64)
        assert np.all(got <= ref * (1 + 1e-12))
        assert np.all(got >= ref * (1 - slack) - 1e-30)


@pytest.mark.parametrize("frac", [(1, 20), (1, 10), (1, 5)], ids=["W12", "W25", "W51"])
def test_full_size_sampled(dev, frac):
    """The benchmark's workload (1000 queries x 10000 references, length 256,
    d=8) at windows 5%, 10% and 20% in the launch configuration the
    benchmark times; every query's result is checked for a sample of queries
    against the exhaustive FP64 oracle."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.cascade_knn()
    say("knn full size", frac, Q.shape, Cs.shape)
    idx, dist, st = run_knn(dev, Q, Cs, frac=frac, bounds="mv")
    say("stats", st)
    sample = np.array([0, 1, 2, 137, 500, 998, 999])
    ri, rd = O.knn_exhaustive(Q[sample], Cs, num=frac[0], den=frac[1])
    np.testing.assert_array_equal(idx[sample], ri)
    np.testing.assert_array_equal(dist[sample], rd.astype(np.float32))
    assert np.all((idx >= 0) & (idx < len(Cs)))
    assert st["pruned_mv"] + st["dtw_started"] == 1000 * 10000


def _pc_floor(Cs):
    """The smallest cell length the library derives from the index: 1e-5 of the
    float32 value range, computed as float32(1e-5 * float64(max - min))."""
    rng = np.float32(Cs.max()) - np.float32(Cs.min())
    return float(np.float32(1e-5 * np.float64(rng)))


@pytest.mark.parametrize("case", [(8, 3, (1, 10), 2, 6, 6), (16, 4, (1, 5), 3, 4, 6), (33, 2, (1, 10), 2, 16, 3)],
                         ids=["d8_W8_L2_K6", "d16_W16_L3_K4", "d33_W8_L2_K16_w3"])
def test_lb_pc_dense_matrix(dev, case):
    from paper_2101_07731_amd import search, synth
    D, seed, frac, Lv, K, w = case
    T = 80 if D != 2 else 33
    Q, Cs = synth.cascade_knn(nq=11, nc=90, T=T, D=D, seed=30 + seed)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    say("lb_pc dense", case)
    lb = search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="pc", frac=frac, pc_levels=Lv,
                             pc_clusters=K, pc_group=w).cpu().numpy().astype(np.float64)
    W = O.window_eff(T, T, 0, *frac)
    fl = _pc_floor(Cs)
    ref = np.array([[O.lb_pc(q, c, W, Lv=Lv, K=K, w=w, floor_len=fl) for c in Cs] for q in Q])
    assert np.all(lb <= ref * (1 + 1e-12))
    slack = 2 * (T + D + 5) * 2.0 ** -24 * 1.01 + 1e-7
    np.testing.assert_array_less(ref * (1 - slack) - 1e-30, lb + 1e-30)


@pytest.mark.parametrize("D", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("w", [6, 3, 4])
def test_lb_pc_narrow_points(dev, D, w):
    """The query-side LB_PC kernel with every point width up to 7 fixed at
    compile time and the group lengths that select six, three and two points
    per step (a ragged last group: 77 = 12 * 6 + 5 positions), per element
    against the oracle."""
    from paper_2101_07731_amd import search, synth
    T = 77
    Q, Cs = synth.cascade_knn(nq=5, nc=70, T=T, D=D, seed=60 + D)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    say("lb_pc narrow", D, w)
    lb = search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="pc", frac=(1, 10), pc_levels=2,
                             pc_clusters=4, pc_group=w).cpu().numpy().astype(np.float64)
    W = O.window_eff(T, T, 0, 1, 10)
    fl = _pc_floor(Cs)
    ref = np.array([[O.lb_pc(q, c, W, Lv=2, K=4, w=w, floor_len=fl) for c in Cs] for q in Q])
    assert np.all(lb <= ref * (1 + 1e-12))
    slack = 2 * (T + D + 5) * 2.0 ** -24 * 1.01 + 1e-7
    np.testing.assert_array_less(ref * (1 - slack) - 1e-30, lb + 1e-30)


@pytest.mark.parametrize("K", [1, 5, 8])
@pytest.mark.parametrize("T", [192, 193])
def test_lb_pc_points_kernel_edges(dev, K, T):
    """Narrow points (d = 3, w = 6) at the series length where the search
    switches from lanes over the candidate's points (T <= 192) to lanes over
    candidates, with box counts below, between and at the register sets
    (K = 1, 5, 8): per element against the oracle."""
    from paper_2101_07731_amd import search, synth
    D = 3
    Q, Cs = synth.cascade_knn(nq=3, nc=40, T=T, D=D, seed=80 + K)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    say("lb_pc points kernel edges", K, T)
    lb = search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="pc", frac=(1, 10), pc_levels=2,
                             pc_clusters=K, pc_group=6).cpu().numpy().astype(np.float64)
    W = O.window_eff(T, T, 0, 1, 10)
    fl = _pc_floor(Cs)
    ref = np.array([[O.lb_pc(q, c, W, Lv=2, K=K, w=6, floor_len=fl) for c in Cs] for q in Q])
    assert np.all(lb <= ref * (1 + 1e-12))
    slack = 2 * (T + D + 5) * 2.0 ** -24 * 1.01 + 1e-7
    np.testing.assert_array_less(ref * (1 - slack) - 1e-30, lb + 1e-30)


@pytest.mark.parametrize("case", [(8, 3, (1, 10), 2, 6, 6, 80), (16, 4, (1, 5), 3, 4, 6, 80),
                                  (33, 2, (1, 10), 2, 16, 3, 33), (5, 5, (1, 10), 2, 6, 6, 71)],
                         ids=["d8_W8_L2_K6", "d16_W16_L3_K4", "d33_W8_L2_K16_w3", "d5_m71_n80"])
def test_lb_pc_candidate_boxes_dense_matrix(dev, case):
    """LB_PC with the roles swapped (boxes of the candidates, built once per
    index) against oracle.lb_pc(c, q): same rounding bar as the query-side
    bound, the points now the query's (m of them)."""
    from paper_2101_07731_amd import search, synth
    D, seed, frac, Lv, K, w, m = case
    n = 80 if D != 2 else 33
    Q, Cs = synth.cascade_knn(nq=11, nc=90, T=n, D=D, seed=50 + seed)
    Q = np.ascontiguousarray(Q[:, :m])
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    say("lb_pc candidate boxes dense", case)
    kw = dict(frac=frac, pc_levels=Lv, pc_clusters=K, pc_group=w)
    cb = search.CandBoxes(ix, m, **kw)
    lb = search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="pc", pc_cand=cb,
                             **kw).cpu().numpy().astype(np.float64)
    W = O.window_eff(m, n, 0, *frac)
    fl = _pc_floor(Cs)
    ref = np.array([[O.lb_pc(c, q, W, Lv=Lv, K=K, w=w, floor_len=fl) for c in Cs] for q in Q])
    assert np.all(lb <= ref * (1 + 1e-12))
    slack = 2 * (m + D + 5) * 2.0 ** -24 * 1.01 + 1e-7
    np.testing.assert_array_less(ref * (1 - slack) - 1e-30, lb + 1e-30)
    # a descriptor built for another query length is refused
    from paper_2101_07731_amd import _lib as L
    with pytest.raises(L.TcDtwError):
        search.lower_bounds(ix, torch.from_numpy(np.ascontiguousarray(Q[:, :m - 1])).to(dev), kind="pc",
                            pc_cand=cb, **kw)


@pytest.mark.parametrize("frac", [(1, 10), (1, 5)])
def test_cascade_with_candidate_boxes(dev, frac):
    """The search with LB_PC on candidate-side boxes returns the oracle's
    neighbours (1-NN and k = 4)."""
    from paper_2101_07731_amd import search, synth
    Q, Cs = synth.cascade_knn(nq=30, nc=700, T=96, D=8, seed=27)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    cb = search.CandBoxes(ix, 96, frac=frac)
    Qd = torch.from_numpy(Q).to(dev)
    say("knn candidate boxes", frac)
    for e in (0.0, 0.1, 0.5):
        idx, dist, st = search.knn(ix, Qd, stats=True, frac=frac, bounds="mv+pc", trigger_pc=e, pc_cand=cb)
        check_against_oracle(idx.cpu().numpy(), dist.cpu().numpy(), Q, Cs, *frac)
        assert st["pruned_mv"] + st["pruned_pc"] + st["dtw_started"] == st["pairs"], st
    idx, dist = search.knn(ix, Qd, k=4, frac=frac, bounds="mv+pc+ti", pc_cand=cb)
    ri, rd = O.knn_exhaustive_k(Q, Cs, 4, num=frac[0], den=frac[1])
    np.testing.assert_array_equal(idx.cpu().numpy(), ri)
    np.testing.assert_array_equal(dist.cpu().numpy(), rd.astype(np.float32))


@pytest.mark.parametrize("P,top", [(5, 1), (0, 0), (3, 0), (0, 1), (1, 0)])
@pytest.mark.parametrize("frac", [(1, 10), (1, 5)])
def test_lb_ti_dense_matrix(dev, P, top, frac):
    from paper_2101_07731_amd import search, synth
    T, D = 100, 6
    Q, Cs = synth.cascade_knn(nq=9, nc=70, T=T, D=D, seed=40)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    say("lb_ti dense", P, top, frac)
    lb = search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="ti", frac=frac, ti_period=P,
                             ti_top=top).cpu().numpy().astype(np.float64)
    W = O.window_eff(T, T, 0, *frac)
    ref = np.array([[O.lb_ti(q, c, W, P=P, top=top) for c in Cs] for q in Q])
    assert np.all(lb <= ref * (1 + 1e-12) + 1e-30)
    lo = np.array([[ti_lower_allowance(q, c, W, P, top) for c in Cs] for q in Q])
    np.testing.assert_array_less(lo - 1e-30, lb + 1e-30)


@pytest.mark.parametrize("bounds", ["mv+pc", "mv+pc+ti"])
def test_trajectory_workload_advanced_bounds(dev, bounds):
    """The trajectory workload (smooth curves across d = 3, length 182): the
    cascade with LB_PC behind LB_MV equals the oracle's exhaustive search, and
    LB_PC prunes pairs there (the oracle's own sequential cascade prunes with
    it on the same data)."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.trajectory_knn(nq=40, nc=1500)
    idx, dist, st = run_knn(dev, Q, Cs, frac=(1, 10), bounds=bounds)
    say("trajectory", bounds, st)
    check_against_oracle(idx, dist, Q, Cs, 1, 10)
    assert st["pruned_mv"] + st["pruned_pc"] + st["pruned_ti"] + st["dtw_started"] == st["pairs"], st
    assert st["pruned_pc"] > 0
    _, _, cs = O.knn_cascade(Q[:8], Cs, num=1, den=10, bounds=2)
    assert cs["pruned_pc"].sum() > 0


TI_SHAPES = [(40, 40, 0, 3), (40, 40, 1, 6), (50, 64, 7, 6), (64, 50, 3, 13), (12, 12, 5, 6), (8, 8, 7, 4),
             (96, 96, 31, 8), (96, 96, 32, 8), (150, 150, 63, 5)]


@pytest.mark.parametrize("P,top", [(5, 1), (5, 0), (1, 0), (0, 0), (0, 1), (2, 1), (7, 0)])
@pytest.mark.parametrize("shape", TI_SHAPES, ids=["m%d_n%d_w%d_d%d" % s for s in TI_SHAPES])
def test_lb_ti_band_offset_shapes(dev, P, top, shape):
    """The one-wave LB_TI kernel (bands of up to 127 offsets) over the shapes
    that decide its row phases: W = 0 and 1, m < n and m > n (W_eff = |m - n|),
    series too short for rows with every offset inside the candidate, one and
    two offsets per lane, and point widths of one to four chunks; against the
    oracle, never above it and never below the per-cell allowance."""
    from paper_2101_07731_amd import search, synth
    m, n, w, D = shape
    Q, Cs = synth.cascade_knn(nq=4, nc=12, T=max(m, n), D=D, seed=43 + m + n + w)
    Q = np.ascontiguousarray(Q[:, :m])
    Cs = np.ascontiguousarray(Cs[:, :n])
    W = O.window_eff(m, n, w)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    say("lb_ti shapes", P, top, shape, "W", W)
    lb = search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="ti", window=w, frac=None, ti_period=P,
                             ti_top=top).cpu().numpy().astype(np.float64)
    ref = np.array([[O.lb_ti(q, c, W, P=P, top=top) for c in Cs] for q in Q])
    assert np.all(lb <= ref * (1 + 1e-12) + 1e-30)
    lo = np.array([[ti_lower_allowance(q, c, W, P, top) for c in Cs] for q in Q])
    np.testing.assert_array_less(lo - 1e-30, lb + 1e-30)


@pytest.mark.parametrize("bounds", ["mv+pc", "mv+ti", "mv+pc+ti"])
@pytest.mark.parametrize("frac", [(1, 20), (1, 10), (1, 5)])
def test_cascade_with_advanced_bounds(dev, bounds, frac):
    from paper_2101_07731_amd import synth
    Q, Cs = synth.cascade_knn(nq=30, nc=700, T=96, D=8, seed=26)
    Cs = np.concatenate([Cs, Cs[::9]])
    say("knn", bounds, frac)
    for e in (0.0, 0.1, 0.5):
        idx, dist, st = run_knn(dev, Q, Cs, frac=frac, bounds=bounds, trigger_pc=e, trigger_ti=e)
        check_against_oracle(idx, dist, Q, Cs, *frac)
        assert st["pruned_mv"] + st["pruned_pc"] + st["pruned_ti"] + st["dtw_started"] == st["pairs"], st
        if "pc" not in bounds:
            assert st["pruned_pc"] == 0
        if "ti" not in bounds:
            assert st["pruned_ti"] == 0


def test_full_size_sampled_full_cascade(dev):
    """The benchmark workload with LB_MV, LB_PC and LB_TI deployed."""
    from paper_2101_07731_amd import synth
    Q, Cs = synth.cascade_knn()
    idx, dist, st = run_knn(dev, Q, Cs, frac=(1, 10), bounds="mv+pc+ti")
    say("stats full cascade", st)
    sample = np.array([3, 400, 777])
    ri, rd = O.knn_exhaustive(Q[sample], Cs, num=1, den=10)
    np.testing.assert_array_equal(idx[sample], ri)
    np.testing.assert_array_equal(dist[sample], rd.astype(np.float32))
    assert st["pruned_mv"] + st["pruned_pc"] + st["pruned_ti"] + st["dtw_started"] == 1000 * 10000


@pytest.mark.parametrize("P,top", [(5, 1), (0, 0), (3, 0), (1, 0), (5, 0)])
@pytest.mark.parametrize("case", [(150, 150, (1, 2)), (300, 300, (1, 2)), (180, 300, (1, 4))],
                         ids=["T150_W74", "T300_W150", "m180_n300_W120"])
def test_lb_ti_dense_matrix_wide_band(dev, P, top, case):
    """LB_TI for bands wider than 63 (the column mapping), against the oracle:
    never above it and never below the per-cell allowance."""
    from paper_2101_07731_amd import search, synth
    m, n, frac = case
    D = 5
    Q, Cs = synth.cascade_knn(nq=5, nc=24, T=max(m, n), D=D, seed=41)
    Q = np.ascontiguousarray(Q[:, :m])
    Cs = np.ascontiguousarray(Cs[:, :n])
    W = O.window_eff(m, n, 0, *frac)
    assert 2 * W + 1 > 128
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    say("lb_ti dense wide", P, top, case, "W", W)
    lb = search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="ti", frac=frac, ti_period=P,
                             ti_top=top).cpu().numpy().astype(np.float64)
    ref = np.array([[O.lb_ti(q, c, W, P=P, top=top) for c in Cs] for q in Q])
    assert np.all(lb <= ref * (1 + 1e-12) + 1e-30)
    lo = np.array([[ti_lower_allowance(q, c, W, P, top) for c in Cs] for q in Q])
    np.testing.assert_array_less(lo - 1e-30, lb + 1e-30)


def test_tune_cascade_picks_a_runnable_choice(dev):
    """Setup-stage choice over the paper's grids (bounds, Lv, triggers), also
    with a band wider than 63; the choice is cached by shape and parameters."""
    from paper_2101_07731_amd import search, synth
    Q, Cs = synth.cascade_knn(nq=20, nc=400, T=96, D=8, seed=31)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    Qd = torch.from_numpy(Q).to(dev)
    best, times = search.tune_cascade(ix, Qd, reps=1, frac=(1, 10))
    assert search.choice_name(best) in times and len(times) == len(search.CASCADE_CHOICES)
    assert search.tune_cascade(ix, Qd, reps=1, frac=(1, 10))[0] == best      # cached
    idx, dist = search.knn(ix, Qd, frac=(1, 10), **best)
    check_against_oracle(idx.cpu().numpy(), dist.cpu().numpy(), Q, Cs, 1, 10)
    Ql, Cl = synth.long_knn(nq=3, nc=20, T=300, D=4)
    ixl = search.Index(torch.from_numpy(Cl).to(dev))
    bl, tl = search.tune_cascade(ixl, torch.from_numpy(Ql).to(dev), reps=1, frac=(1, 2), pc_clusters=16)   # W = 150
    assert len(tl) == len(search.CASCADE_CHOICES)
    idx, dist = search.knn(ixl, torch.from_numpy(Ql).to(dev), frac=(1, 2), pc_clusters=16, **bl)
    check_against_oracle(idx.cpu().numpy(), dist.cpu().numpy(), Ql, Cl, 1, 2)


@pytest.mark.parametrize("k", [1, 4])
def test_graphed_search_replays_match_eager(dev, k):
    """The whole cascade captured in a HIP graph (search.GraphedSearch): three
    replays, with eager searches and synchronisations between them and new
    queries copied in before the last, each equal to the eager result."""
    from paper_2101_07731_amd import search, synth
    Q, Cs = synth.cascade_knn(nq=24, nc=500, T=80, D=6, seed=70)
    Q2, _ = synth.cascade_knn(nq=24, nc=1, T=80, D=6, seed=71)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    for bounds in ("mv", "mv+pc+ti"):
        say("graphed search", bounds, "k", k)
        g = search.GraphedSearch(ix, torch.from_numpy(Q).to(dev), k=k, frac=(1, 10), bounds=bounds)
        ei, ed = search.knn(ix, torch.from_numpy(Q).to(dev), k=k, frac=(1, 10), bounds=bounds)
        for rep in range(3):
            if rep == 2:
                g.queries_flat.copy_(torch.from_numpy(Q2).to(dev).reshape(g.queries_flat.shape))
                ei, ed = search.knn(ix, torch.from_numpy(Q2).to(dev), k=k, frac=(1, 10), bounds=bounds)
            gi, gd = g.replay()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(gi.cpu().numpy(), ei.cpu().numpy())
            np.testing.assert_array_equal(gd.cpu().numpy(), ed.cpu().numpy())
            search.knn(ix, torch.from_numpy(Q[:5]).to(dev), frac=(1, 10))   # eager work between replays
            torch.cuda.synchronize()
    if k == 1:
        check_against_oracle(gi.cpu().numpy(), gd.cpu().numpy(), Q2, Cs, 1, 10)
    else:
        ri, rd = O.knn_exhaustive_k(Q2, Cs, k, num=1, den=10)
        np.testing.assert_array_equal(gi.cpu().numpy(), ri)
        np.testing.assert_array_equal(gd.cpu().numpy(), rd.astype(np.float32))
