"""1-NN over reference banks of uneven lengths on the GPU against the FP64
oracle: per-pair windows (W = 10% of the longer series, W_eff >= |m - n|),
LB_MV through query sparse tables, DTW on the row mapping, float64
re-scoring.  The returned index must equal the oracle's exhaustive search
(ties to the lowest index) and the distance its float64 value rounded to
float32."""
import sys

import numpy as np
import pytest

import oracle as O

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


def bank(rng, count, lo, hi, D):
    from paper_2101_07731_amd import synth
    return [synth._f32(synth.znorm(synth.correlated_walks(rng, 1, int(rng.integers(lo, hi + 1)), D))[0])
            for _ in range(count)]


def run(dev, Q, Cs, frac=(1, 10), bounds="mv", **kw):
    from paper_2101_07731_amd import search
    ix = search.Index([torch.from_numpy(c).to(dev) for c in Cs])
    Qd = [torch.from_numpy(q).to(dev) for q in Q] if isinstance(Q, list) else torch.from_numpy(Q).to(dev)
    idx, dist, st = search.knn(ix, Qd, frac=frac, bounds=bounds, stats=True, **kw)
    return idx.cpu().numpy(), dist.cpu().numpy(), st, ix


@pytest.mark.parametrize("D", [1, 3, 8, 13])
@pytest.mark.parametrize("bounds", ["mv", "plain"])
def test_ragged_banks_match_exhaustive(dev, D, bounds):
    rng = np.random.default_rng(100 + D)
    Cs = bank(rng, 70, 4, 180, D)
    Cs += [Cs[5].copy(), Cs[17].copy()]          # exact duplicates: ties go to the lowest index
    Q = bank(rng, 12, 4, 180, D) + [Cs[17].copy()]
    say("ragged knn", D, bounds)
    idx, dist, st, _ = run(dev, Q, Cs, bounds=bounds)
    ri, rd = O.knn_exhaustive(Q, Cs, num=1, den=10)
    np.testing.assert_array_equal(idx, ri)
    np.testing.assert_array_equal(dist, rd.astype(np.float32))
    assert st["pruned_mv"] + st["dtw_started"] == st["pairs"]
    if bounds == "plain":
        assert st["dtw_started"] == len(Q) * len(Cs)


def test_uniform_queries_against_ragged_bank(dev):
    rng = np.random.default_rng(7)
    Cs = bank(rng, 50, 20, 130, 4)
    from paper_2101_07731_amd import synth
    Q = synth._f32(synth.znorm(synth.correlated_walks(rng, 9, 77, 4)))
    idx, dist, _, _ = run(dev, Q, Cs, frac=(1, 5))
    ri, rd = O.knn_exhaustive(Q, Cs, num=1, den=5)
    np.testing.assert_array_equal(idx, ri)
    np.testing.assert_array_equal(dist, rd.astype(np.float32))


@pytest.mark.parametrize("D", [5, 8])      # scalar and float4 paths
def test_ragged_lb_mv_sound_and_tight(dev, D):
    from paper_2101_07731_amd import search
    rng = np.random.default_rng(8)
    Cs = bank(rng, 40, 3, 150, D)
    Q = bank(rng, 7, 3, 150, D)
    ix = search.Index([torch.from_numpy(c).to(dev) for c in Cs])
    lb = search.lower_bounds(ix, [torch.from_numpy(q).to(dev) for q in Q], kind="mv", frac=(1, 10))
    lb = lb.cpu().numpy().astype(np.float64)
    for qi, q in enumerate(Q):
        for ci, c in enumerate(Cs):
            W = O.window_eff(q.shape[0], c.shape[0], 0, 1, 10)
            ref = O.lb_mv(q, c, W)
            assert lb[qi, ci] <= ref * (1 + 1e-12) + 1e-30
            slack = 2 * (c.shape[0] * D + 9) * 2.0 ** -24 * 1.01 + 1e-7
            assert lb[qi, ci] >= ref * (1 - slack) - 1e-30, (qi, ci, lb[qi, ci], ref)


@pytest.fixture(scope="module")
def bank_workload():
    from paper_2101_07731_amd import synth
    return synth.ragged_banks()


@pytest.mark.parametrize("D", [2, 4, 8, 16, 32])
def test_bank_workload_sampled(dev, bank_workload, D):
    """Each of the five banks of the uneven 1-NN workload (4096 references of
    lengths U[64, 2048], d = 2, 4, 8, 16, 32) with its queries; the bank's
    shortest query against the oracle's exhaustive search."""
    banks, queries = bank_workload
    Cs = banks[D]
    Q = [q for d, q in queries if d == D]
    say("bank", D, len(Q), len(Cs))
    idx, dist, st, _ = run(dev, Q, Cs)
    assert st["pruned_mv"] + st["dtw_started"] == st["pairs"]
    k = int(np.argmin([q.shape[0] for q in Q]))          # the shortest query keeps the oracle quick
    ri, rd = O.knn_exhaustive([Q[k]], Cs, num=1, den=10, threads=16)
    assert idx[k] == ri[0]
    assert dist[k] == np.float32(rd[0])


def _banked(rng, dims, per_bank, lo, hi):
    refs, first = [], {}
    for D in dims:
        first[D] = len(refs)
        refs += bank(rng, per_bank, lo, hi, D)
    return refs, first


@pytest.mark.parametrize("bounds", ["mv", "plain"])
def test_banks_of_several_dims_in_one_call(dev, bounds):
    """An index over banks of d = 1, 3, 4, 8 (each a contiguous run, lengths
    uneven) and queries of mixed d in ONE search call: every query gets the
    oracle's nearest neighbour within the bank of its d (index in the whole
    set), ties to the lowest index; the pair count covers query-bank pairs."""
    from paper_2101_07731_amd import search
    rng = np.random.default_rng(140)
    dims = (1, 3, 4, 8)
    refs, first = _banked(rng, dims, 40, 6, 120)
    refs[first[3] + 9] = refs[first[3] + 2].copy()            # a tie inside a bank
    Q, Qd = [], []
    for k in range(14):
        D = dims[k % len(dims)]
        Q += bank(rng, 1, 6, 120, D)
        Qd.append(D)
    Q.append(refs[first[4] + 5].copy())                         # distance 0 to a reference
    Qd.append(4)
    say("banks one call", bounds)
    ix = search.Index([torch.from_numpy(c).to(dev) for c in refs])
    assert ix.ix.nbanks == len(dims)
    idx, dist, st = search.knn(ix, [torch.from_numpy(q).to(dev) for q in Q], frac=(1, 10), bounds=bounds,
                               stats=True)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    assert st["pairs"] == len(Q) * 40
    assert st["pruned_mv"] + st["dtw_started"] == st["pairs"]
    for qi, (q, D) in enumerate(zip(Q, Qd)):
        members = refs[first[D]:first[D] + 40]
        ri, rd = O.knn_exhaustive([q], members, num=1, den=10)
        assert idx[qi] == first[D] + ri[0], (qi, D)
        assert dist[qi] == np.float32(rd[0])
    assert dist[-1] == 0.0 and idx[-1] == first[4] + 5


def test_banks_lower_bounds(dev):
    """The LB_MV matrix over banks: +inf outside a query's bank, the bank's
    own bound inside (as a search of that bank alone)."""
    from paper_2101_07731_amd import search
    rng = np.random.default_rng(141)
    refs, first = _banked(rng, (2, 5), 30, 10, 90)
    Q = bank(rng, 3, 10, 90, 2) + bank(rng, 2, 10, 90, 5)
    ix = search.Index([torch.from_numpy(c).to(dev) for c in refs])
    lb = search.lower_bounds(ix, [torch.from_numpy(q).to(dev) for q in Q], kind="mv", frac=(1, 10)).cpu().numpy()
    for qi, q in enumerate(Q):
        D = q.shape[1]
        lo = first[D]
        assert np.all(np.isinf(np.delete(lb[qi], np.arange(lo, lo + 30))))
        ixb = search.Index([torch.from_numpy(c).to(dev) for c in refs[lo:lo + 30]])
        lbb = search.lower_bounds(ixb, [torch.from_numpy(q).to(dev)], kind="mv", frac=(1, 10)).cpu().numpy()
        np.testing.assert_array_equal(lb[qi, lo:lo + 30], lbb[0])


def test_bank_workload_one_call_sampled(dev, bank_workload):
    """The uneven workload's five banks (4096 references each, d = 2 ... 32)
    in one index and its 256 queries of mixed d in one search call: the same
    neighbours as the per-bank searches for every query, and the oracle's for
    the shortest query of each bank."""
    from paper_2101_07731_amd import search
    banks, queries = bank_workload
    order = sorted(banks)
    refs, first = [], {}
    for D in order:
        first[D] = len(refs)
        refs += banks[D]
    ix = search.Index([torch.from_numpy(c).to(dev) for c in refs])
    Qs = [q for _, q in queries]
    say("bank workload one call", len(refs), len(Qs))
    idx, dist, st = search.knn(ix, [torch.from_numpy(q).to(dev) for q in Qs], frac=(1, 10), stats=True)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    assert st["pairs"] == 256 * 4096
    for D in order:
        sel = [k for k, (d, _) in enumerate(queries) if d == D]
        ixb = search.Index([torch.from_numpy(c).to(dev) for c in banks[D]])
        ib, db = search.knn(ixb, [torch.from_numpy(Qs[k]).to(dev) for k in sel], frac=(1, 10))
        np.testing.assert_array_equal(idx[sel], ib.cpu().numpy() + first[D])
        np.testing.assert_array_equal(dist[sel], db.cpu().numpy())
        k = sel[int(np.argmin([Qs[t].shape[0] for t in sel]))]
        ri, rd = O.knn_exhaustive([Qs[k]], banks[D], num=1, den=10, threads=16)
        assert idx[k] == first[D] + ri[0] and dist[k] == np.float32(rd[0])


def test_graphed_bank_search_replays_match_eager(dev):
    """The one-call search over banks of several dims (queries of uneven
    lengths and mixed d) captured in a HIP graph: the captured call reuses the
    query metadata the warm-up call wrote; three replays equal the eager
    result."""
    from paper_2101_07731_amd import search
    rng = np.random.default_rng(142)
    refs, first = _banked(rng, (2, 8), 30, 10, 90)
    Q = bank(rng, 4, 10, 90, 2) + bank(rng, 3, 10, 90, 8)
    ix = search.Index([torch.from_numpy(c).to(dev) for c in refs])
    Qd = [torch.from_numpy(q).to(dev) for q in Q]
    g = search.GraphedSearch(ix, Qd, frac=(1, 10), bounds="mv")
    ei, ed = search.knn(ix, Qd, frac=(1, 10), bounds="mv")
    for _ in range(3):
        gi, gd = g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(gi.cpu().numpy(), ei.cpu().numpy())
        np.testing.assert_array_equal(gd.cpu().numpy(), ed.cpu().numpy())
        search.knn(ix, Qd[:2], frac=(1, 10))
        torch.cuda.synchronize()
