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
