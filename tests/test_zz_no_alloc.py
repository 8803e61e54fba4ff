"""tc_dtw_banded_noalloc (the static-scratch variant of tc_dtw_banded, for
callers that cannot allocate) against tc_dtw_banded: the same distances,
and the same gradients from the recorded argmin codes, bit for bit (same
kernels and plan; the classes only run in turn on one stream), on two
calls in a row, the second with a smaller
batch, for pairs of uneven lengths and dims (which use the scratch) and
uniform pairs (which need none), in float32 and float64."""
import sys

import numpy as np
import pytest

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


def _ragged(rng, count, lo, hi, dims):
    from paper_2101_07731_amd import synth
    xs, ys = [], []
    for _ in range(count):
        D = int(rng.choice(dims))
        xs.append(synth._f32(synth.znorm(synth.correlated_walks(rng, 1, int(rng.integers(lo, hi + 1)), D))[0]))
        ys.append(synth._f32(synth.znorm(synth.correlated_walks(rng, 1, int(rng.integers(lo, hi + 1)), D))[0]))
    return xs, ys


def _compare(dev, xs, ys, frac, f64):
    from paper_2101_07731_amd import pairs
    X = [torch.from_numpy(a).to(dev) for a in xs] if isinstance(xs, list) else torch.from_numpy(xs).to(dev)
    Y = [torch.from_numpy(a).to(dev) for a in ys] if isinstance(ys, list) else torch.from_numpy(ys).to(dev)
    ref, ref_saved = pairs.banded(X, Y, frac=frac, f64=f64, save=True)
    sb = pairs.saved_bytes(X, Y, frac=frac)
    saved = torch.full((max(sb, 4),), 0x5A, dtype=torch.uint8, device=dev)
    dist = torch.full_like(ref, float("nan"))
    pairs.banded_noalloc(X, Y, frac=frac, f64=f64, saved=saved, dist=dist)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dist.cpu().numpy(), ref.cpu().numpy())
    # the recorded argmin codes, as the backward reads them (words past a pair's record are never
    # written by either call): the same gradients bit for bit
    g = torch.linspace(0.5, 2.0, ref.numel(), device=dev)
    rx, ry = pairs.backward(X, Y, ref_saved, g, frac=frac)
    nx, ny = pairs.backward(X, Y, saved, g, frac=frac)
    rx = rx if isinstance(rx, list) else [rx]
    nx = nx if isinstance(nx, list) else [nx]
    ry = ry if isinstance(ry, list) else [ry]
    ny = ny if isinstance(ny, list) else [ny]
    for a, b in zip(rx + ry, nx + ny):
        np.testing.assert_array_equal(b.cpu().numpy(), a.cpu().numpy())


@pytest.mark.parametrize("f64", [False, True], ids=["f32", "f64"])
def test_noalloc_matches_banded_two_calls(dev, f64):
    from paper_2101_07731_amd import _lib as L
    assert L.lib().tc_dtw_banded_noalloc is not None
    rng = np.random.default_rng(71)
    xs, ys = _ragged(rng, 300, 16, 700, (2, 4, 8, 16, 32))      # both mappings, several classes
    say("noalloc ragged", len(xs), "f64" if f64 else "f32")
    _compare(dev, xs, ys, (1, 10), f64)
    xs2, ys2 = _ragged(rng, 37, 8, 300, (3, 8))                   # second call, smaller batch
    _compare(dev, xs2, ys2, (1, 10), f64)
    # uniform pairs (no scratch used), then ragged again after them
    xu = np.cumsum(rng.standard_normal((20, 96, 6)), 1).astype(np.float32)
    yu = np.cumsum(rng.standard_normal((20, 96, 6)), 1).astype(np.float32)
    _compare(dev, xu, yu, (1, 10), f64)
    _compare(dev, xs2[:5], ys2[:5], (1, 5), f64)


def test_noalloc_rejects_a_plan_beyond_the_scratch(dev):
    """A batch whose pair plan exceeds the static scratch is refused with
    UNSUPPORTED on the host, before any work is enqueued."""
    import ctypes as C
    from paper_2101_07731_amd import _lib as L
    lib = L.lib()
    cap = lib.tc_dtw_noalloc_scratch_bytes()
    n = cap // 48 + 10
    lens = np.full(n, 5, dtype=np.int32)
    lens[::2] = 6
    offs = np.zeros(n, dtype=np.int64)
    offs[1:] = np.cumsum(lens[:-1].astype(np.int64) * 2)
    buf = torch.zeros(int(offs[-1] + lens[-1] * 2), dtype=torch.float32, device=dev)
    b = L.Batch(buf.data_ptr(), offs.ctypes.data_as(C.POINTER(C.c_int64)),
                lens.ctypes.data_as(C.POINTER(C.c_int32)), n, 2, 0, None)
    dist = torch.full((n,), -1.0, device=dev)
    st = lib.tc_dtw_banded_noalloc(C.byref(b), C.byref(b), L.Window(0, 1, 10), 0, C.c_void_p(dist.data_ptr()),
                                   None, None)
    assert st == L.ERR_UNSUPPORTED
    assert b"static scratch" in lib.tc_dtw_last_error()
    torch.cuda.synchronize()
    assert torch.all(dist == -1.0)
