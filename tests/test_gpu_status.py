"""The device status word and tc_dtw_sync_status on the GPU: conditions the
asynchronous kernels detect (non-finite reference or query values) are
reported by the next tc_dtw_sync_status and then cleared; the
TC_DTW_FAKE_NO_DEVICE test hook turns calls into ERR_DEVICE."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2101_07731_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


def _sync():
    from paper_2101_07731_amd import _lib as L
    from paper_2101_07731_amd.pairs import _stream
    lib = L.lib()
    st = lib.tc_dtw_sync_status(_stream())
    return st, lib.tc_dtw_last_error().decode()


def test_clean_calls_leave_the_status_clear(dev):
    from paper_2101_07731_amd import search, synth
    _sync()
    Q, Cs = synth.cascade_knn(nq=4, nc=100, T=40, D=4, seed=60)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    search.knn(ix, torch.from_numpy(Q).to(dev), frac=(1, 10))
    st, msg = _sync()
    assert st == 0, msg


def test_non_finite_reference_reported_once(dev):
    from paper_2101_07731_amd import _lib as L, search, synth
    _sync()
    _, Cs = synth.cascade_knn(nq=1, nc=50, T=40, D=4, seed=61)
    Cs[7, 3, 2] = np.nan
    search.Index(torch.from_numpy(Cs).to(dev))
    st, msg = _sync()
    assert st == L.ERR_DEVICE and "reference value is not finite" in msg, msg
    assert _sync()[0] == 0          # read and cleared


def test_non_finite_query_reported(dev):
    from paper_2101_07731_amd import _lib as L, search, synth
    _sync()
    Q, Cs = synth.cascade_knn(nq=3, nc=60, T=40, D=4, seed=62)
    ix = search.Index(torch.from_numpy(Cs).to(dev))
    Q[1, 5, 0] = np.inf
    search.lower_bounds(ix, torch.from_numpy(Q).to(dev), kind="mv", frac=(1, 10))
    st, msg = _sync()
    assert st == L.ERR_DEVICE and "query value is not finite" in msg, msg
    # uneven query lengths (query tables)
    ixr = search.Index([torch.from_numpy(c[:30 + (k % 7)]).to(dev) for k, c in enumerate(Cs)])
    search.lower_bounds(ixr, [torch.from_numpy(q).to(dev) for q in Q], kind="mv", frac=(1, 10))
    st, msg = _sync()
    assert st == L.ERR_DEVICE and "query value is not finite" in msg, msg
    assert _sync()[0] == 0


def test_fake_no_device_hook(dev, monkeypatch):
    from paper_2101_07731_amd import _lib as L, pairs
    x = torch.randn(2, 16, 3, device=dev)
    monkeypatch.setenv("TC_DTW_FAKE_NO_DEVICE", "1")
    with pytest.raises(L.TcDtwError) as err:
        pairs.banded(x, x, frac=(1, 10))
    assert err.value.status == L.ERR_DEVICE
    monkeypatch.delenv("TC_DTW_FAKE_NO_DEVICE")
    d = pairs.banded(x, x, frac=(1, 10))
    assert torch.all(d == 0)
