"""Batched pairs of uneven lengths and dims on the GPU: the direct ragged
path, reusable plans (every tuning choice), the backward through a plan,
HIP-graph replay, and a sampled check of the 4096-pair workload.

Every tuning choice evaluates the same per-cell arithmetic (the mapping
only changes which lane computes a cell), so float32 results must agree
bit for bit between choices and with the direct call; against the FP64
oracle the float32 bar is 1e-5 relative and the float64 mode is exact.
"""
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


def oracle_mixed(xs, ys, frac):
    """FP64 DTW of each pair, grouped by dim for the oracle's batched call."""
    out = np.zeros(len(xs))
    dims = np.array([x.shape[1] for x in xs])
    for D in np.unique(dims):
        idx = np.nonzero(dims == D)[0]
        out[idx] = O.dtw_pairs([xs[k] for k in idx], [ys[k] for k in idx], num=frac[0], den=frac[1])
    return out


def small_mixed(seed, npairs=60, tmin=1, tmax=300, dims=(1, 2, 3, 4, 5, 8, 13, 16, 32)):
    from paper_2101_07731_amd import synth
    xs, ys = synth.ragged_pairs(npairs=npairs, tmin=tmin, tmax=tmax, dims=dims, seed=seed)
    return xs, ys


def to_dev(arrs, dev):
    return [torch.from_numpy(a).to(dev) for a in arrs]


def test_direct_mixed_dims(dev):
    from paper_2101_07731_amd import pairs
    xs, ys = small_mixed(11)
    say("batch direct mixed", len(xs))
    ref = oracle_mixed(xs, ys, (1, 10))
    X, Y = to_dev(xs, dev), to_dev(ys, dev)
    d32 = pairs.banded(X, Y, frac=(1, 10)).cpu().numpy()
    np.testing.assert_allclose(d32, ref, rtol=1e-5, atol=0)
    d64 = pairs.banded(X, Y, frac=(1, 10), f64=True).cpu().numpy()
    np.testing.assert_array_equal(d64, ref.astype(np.float32))


@pytest.mark.parametrize("diag_max_w", [-1, 7, 31, 63])
@pytest.mark.parametrize("waves", [0, 1, 5])
@pytest.mark.parametrize("per_pair", [1, 8])
def test_plan_every_tuning_matches(dev, diag_max_w, waves, per_pair):
    from paper_2101_07731_amd import pairs
    xs, ys = small_mixed(12, npairs=48, tmax=1200)
    say("batch plan", diag_max_w, waves, per_pair)
    X, Y = to_dev(xs, dev), to_dev(ys, dev)
    direct = pairs.banded(X, Y, frac=(1, 10)).cpu().numpy()
    plan = pairs.Plan(X, Y, frac=(1, 10), diag_max_w=diag_max_w, waves_per_cu=waves, waves_per_pair=per_pair)
    got = plan.forward().cpu().numpy()
    np.testing.assert_array_equal(got, direct)
    got64 = plan.forward(f64=True).cpu().numpy()
    np.testing.assert_array_equal(got64, oracle_mixed(xs, ys, (1, 10)).astype(np.float32))
    if diag_max_w == -1:
        assert all(c[0] == "rows" for c in plan.classes())
    if per_pair == 8:
        assert any(c[6] > 1 for c in plan.classes())


def test_plan_backward_matches_oracle_path_gradient(dev):
    from paper_2101_07731_amd import pairs
    rng = np.random.default_rng(21)
    xs, ys = [], []
    for k in range(14):
        D = int(rng.choice([1, 3, 4, 8, 12]))
        m, n = int(rng.integers(2, 700)), int(rng.integers(2, 700))
        # jitter breaks ties between predecessors
        xs.append((np.cumsum(rng.standard_normal((m, D)), 0) + 1e-3 * rng.standard_normal((m, D))).astype(np.float32))
        ys.append((np.cumsum(rng.standard_normal((n, D)), 0) + 1e-3 * rng.standard_normal((n, D))).astype(np.float32))
    say("batch plan backward", len(xs))
    X, Y = to_dev(xs, dev), to_dev(ys, dev)
    g = torch.from_numpy(rng.uniform(0.5, 2.0, size=len(xs)).astype(np.float32)).to(dev)
    for dm, wp in ((63, 1), (-1, 8)):
        # a float64 forward takes the oracle's path, so the gradients agree to float32 rounding
        plan = pairs.Plan(X, Y, frac=(1, 10), diag_max_w=dm, waves_per_pair=wp)
        saved = plan.saved_buffer()
        dist = plan.forward(saved=saved, f64=True).cpu().numpy()
        gx, gy = plan.backward(saved, g)
        gxs, gys = plan.X.split(gx), plan.Y.split(gy)
        for k in range(len(xs)):
            m, n = xs[k].shape[0], ys[k].shape[0]
            W = O.window_eff(m, n, 0, 1, 10)
            v, rq, rc, _ = O.path_grad(xs[k], ys[k], W, gbar=float(g[k]))
            assert np.float32(v) == dist[k]
            scale = max(1.0, np.abs(rq).max(), np.abs(rc).max())
            np.testing.assert_allclose(gxs[k].cpu().numpy(), rq, rtol=1e-6, atol=1e-6 * scale)
            np.testing.assert_allclose(gys[k].cpu().numpy(), rc, rtol=1e-6, atol=1e-6 * scale)


def test_graph_replay_with_new_data(dev):
    from paper_2101_07731_amd import pairs
    xs, ys = small_mixed(13, npairs=40)
    say("batch graph", len(xs))
    X, Y = to_dev(xs, dev), to_dev(ys, dev)
    plan = pairs.Plan(X, Y, frac=(1, 10))
    gf = pairs.GraphedForward(plan)
    rng = np.random.default_rng(14)
    for rep in range(4):
        # new data of the same layout, then eager work between replays
        newx = torch.from_numpy(rng.standard_normal(gf.x_flat.numel()).astype(np.float32)).to(dev)
        newy = torch.from_numpy(rng.standard_normal(gf.y_flat.numel()).astype(np.float32)).to(dev)
        gf.x_flat.copy_(newx)
        gf.y_flat.copy_(newy)
        got = gf.replay().clone()
        eager = plan.forward(newx, newy)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), eager.cpu().numpy())
        xs2 = [a.cpu().numpy() for a in plan.X.split(newx)]
        ys2 = [a.cpu().numpy() for a in plan.Y.split(newy)]
        if rep == 0:
            np.testing.assert_allclose(got.cpu().numpy(), oracle_mixed(xs2, ys2, (1, 10)), rtol=1e-5)


def test_autotune_picks_a_choice(dev):
    from paper_2101_07731_amd import pairs
    xs, ys = small_mixed(15, npairs=64, tmax=200)
    X, Y = to_dev(xs, dev), to_dev(ys, dev)
    say("batch autotune")
    best, times = pairs.autotune(X, Y, frac=(1, 10), reps=2, diag_choices=(-1, 63), wave_choices=(4, 16),
                                 pair_choices=(1, 4))
    assert best in times and len(times) == 8
    plan = pairs.tuned_plan(X, Y, frac=(1, 10))
    np.testing.assert_allclose(plan.forward().cpu().numpy(), oracle_mixed(xs, ys, (1, 10)), rtol=1e-5)


def test_full_batch_sampled(dev):
    """The 4096-pair workload (lengths 64..2048, d in {2,4,8,16,32}): 48 sampled pairs against the oracle."""
    from paper_2101_07731_amd import pairs, synth
    xs, ys = synth.ragged_pairs()
    say("batch full", len(xs))
    X, Y = to_dev(xs, dev), to_dev(ys, dev)
    plan = pairs.Plan(X, Y, frac=(1, 10))
    dist = plan.forward().cpu().numpy()
    assert np.all(np.isfinite(dist))
    sample = np.random.default_rng(16).choice(len(xs), 48, replace=False)
    ref = oracle_mixed([xs[k] for k in sample], [ys[k] for k in sample], (1, 10))
    np.testing.assert_allclose(dist[sample], ref, rtol=1e-5, atol=0)
