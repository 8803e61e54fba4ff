"""The C ABI without a GPU: the library loads, exports every function that
include/*.h declares, and rejects invalid arguments on the host before any
HIP call (no compute call is made here)."""
import ctypes as C
import glob
import os
import re

import pytest

from paper_2101_07731_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(tc_dtw_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tc_dtw_banded", "tc_dtw_backward", "tc_dtw_abi_version", "tc_dtw_last_error"):
        assert required in names


def test_library_exports_every_declared_function():
    lib = L.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.tc_dtw_abi_version() == 7


def _batch(count=2, dim=3, ulen=8, data=0x1000):
    return L.Batch(data, None, None, count, dim, ulen, None)


def test_invalid_arguments_rejected_before_any_device_call():
    lib = L.lib()
    w = L.Window(2, 0, 0)
    x, y = _batch(), _batch()
    d = C.c_void_p(0x2000)
    cases = [
        (L.Batch(0, None, None, 2, 3, 8, None), y, w, d, L.ERR_INVALID),  # null data
        (_batch(count=0), y, w, d, L.ERR_INVALID),                       # empty set
        (_batch(count=3), y, w, d, L.ERR_INVALID),                       # count mismatch
        (_batch(dim=4), y, w, d, L.ERR_INVALID),                         # dim mismatch
        (_batch(ulen=0), y, w, d, L.ERR_INVALID),                        # zero length
        (_batch(dim=65), _batch(dim=65), w, d, L.ERR_UNSUPPORTED),       # dim > 64
        (x, y, L.Window(-1, 0, 0), d, L.ERR_INVALID),                    # negative window
        (x, y, L.Window(0, 1, -10), d, L.ERR_INVALID),                   # negative fraction
        (x, y, w, None, L.ERR_INVALID),                                  # null output
    ]
    for xb, yb, wb, out, expect in cases:
        st = lib.tc_dtw_banded(C.byref(xb), C.byref(yb), wb, 0, out, None, None, 0, None)
        assert st == expect, (st, lib.tc_dtw_last_error())
        assert lib.tc_dtw_last_error()
    st = lib.tc_dtw_banded(C.byref(x), C.byref(y), w, 0x80, d, None, None, 0, None)
    assert st == L.ERR_INVALID
    st = lib.tc_dtw_backward(C.byref(x), C.byref(y), w, None, d, d, d, None, 0, None)
    assert st == L.ERR_INVALID


def test_ragged_batches_need_a_workspace():
    lib = L.lib()
    lens = (C.c_int32 * 3)(5, 9, 7)
    x = L.Batch(0x1000, None, lens, 3, 2, 0, None)
    y = L.Batch(0x1000, None, lens, 3, 2, 0, None)
    w = L.Window(0, 1, 10)
    need = lib.tc_dtw_banded_workspace_bytes(C.byref(x), C.byref(y), w, 0)
    assert need > 0
    st = lib.tc_dtw_banded(C.byref(x), C.byref(y), w, 0, C.c_void_p(0x2000), None, None, 0, None)
    assert st == L.ERR_WORKSPACE
    assert lib.tc_dtw_saved_bytes(C.byref(x), C.byref(y), w) > 0
    # uniform pairs need none
    xu = _batch()
    assert lib.tc_dtw_banded_workspace_bytes(C.byref(xu), C.byref(xu), w, 0) == 0


def test_status_strings():
    lib = L.lib()
    for s in range(5):
        assert lib.tc_dtw_status_string(s)


def test_mixed_dims_and_plans_validated_on_the_host():
    lib = L.lib()
    lens = (C.c_int32 * 3)(5, 9, 7)
    dx = (C.c_int32 * 3)(2, 8, 3)
    dy_bad = (C.c_int32 * 3)(2, 8, 4)
    dz = (C.c_int32 * 3)(2, 0, 3)
    x = L.Batch(0x1000, None, lens, 3, 0, 0, dx)
    y = L.Batch(0x1000, None, lens, 3, 0, 0, dx)
    w = L.Window(0, 1, 10)
    assert lib.tc_dtw_banded_workspace_bytes(C.byref(x), C.byref(y), w, 0) > 0
    assert lib.tc_dtw_saved_bytes(C.byref(x), C.byref(y), w) > 0
    ybad = L.Batch(0x1000, None, lens, 3, 0, 0, dy_bad)
    st = lib.tc_dtw_banded(C.byref(x), C.byref(ybad), w, 0, C.c_void_p(0x2000), None, None, 0, None)
    assert st == L.ERR_INVALID and b"same dim" in lib.tc_dtw_last_error()
    z = L.Batch(0x1000, None, lens, 3, 0, 0, dz)
    assert lib.tc_dtw_banded(C.byref(z), C.byref(z), w, 0, C.c_void_p(0x2000), None, None, 0, None) == L.ERR_INVALID
    # plans: size query, tuning validation, null plan / buffer
    t = L.Tuning(63, 0, 0)
    assert lib.tc_dtw_pairs_plan_bytes(C.byref(x), C.byref(y), w, C.byref(t)) > 0
    assert lib.tc_dtw_pairs_plan_bytes(C.byref(x), C.byref(y), w, None) > 0
    for bad in (L.Tuning(64, 0, 0), L.Tuning(-2, 0, 0), L.Tuning(63, 33, 0), L.Tuning(63, -1, 0),
                L.Tuning(63, 0, 3), L.Tuning(63, 0, 16)):
        assert lib.tc_dtw_pairs_plan_bytes(C.byref(x), C.byref(y), w, C.byref(bad)) == 0
        st = lib.tc_dtw_pairs_plan_build(C.byref(x), C.byref(y), w, C.byref(bad), C.c_void_p(0x3000), 1 << 20,
                                         C.byref(L.PairsPlan()), None)
        assert st == L.ERR_INVALID
    st = lib.tc_dtw_pairs_plan_build(C.byref(x), C.byref(y), w, None, C.c_void_p(0x3000), 1 << 20, None, None)
    assert st == L.ERR_INVALID
    st = lib.tc_dtw_banded_run(None, C.c_void_p(0x1000), C.c_void_p(0x1000), 0, C.c_void_p(0x2000), None, None)
    assert st == L.ERR_INVALID
    st = lib.tc_dtw_backward_run(None, None, None, None, None, None, None, None)
    assert st == L.ERR_INVALID


def test_index_banks_validated_on_the_host():
    """References of several dims form banks: each dim one contiguous run,
    at most eight banks; queries of a dim without a bank are refused."""
    lib = L.lib()
    lens = (C.c_int32 * 3)(5, 9, 7)
    dx = (C.c_int32 * 3)(2, 3, 2)                  # dim 2 in two runs
    refs = L.Batch(0x1000, None, lens, 3, 0, 0, dx)
    assert lib.tc_dtw_index_bytes(C.byref(refs)) == 0
    st = lib.tc_dtw_build_index(C.byref(refs), C.c_void_p(0x2000), 1 << 20, C.byref(L.Index()), None)
    assert st == L.ERR_UNSUPPORTED
    n = 9
    lens9 = (C.c_int32 * n)(*([5] * n))
    d9 = (C.c_int32 * n)(*range(1, n + 1))          # nine banks
    refs9 = L.Batch(0x1000, None, lens9, n, 0, 0, d9)
    assert lib.tc_dtw_index_bytes(C.byref(refs9)) == 0
    dok = (C.c_int32 * 3)(2, 2, 3)
    assert lib.tc_dtw_index_bytes(C.byref(L.Batch(0x1000, None, lens, 3, 0, 0, dok))) > 0
    # a hand-made index description with banks of dims 2 and 3: a query of dim 4 has no bank
    ix = L.Index()
    ix.buf, ix.bytes, ix.count, ix.dim, ix.uniform_len, ix.max_len = 0x3000, 1 << 20, 3, 3, 0, 9
    ix.nbanks = 2
    ix.bank_dim[0], ix.bank_first[0], ix.bank_count[0] = 2, 0, 2
    ix.bank_dim[1], ix.bank_first[1], ix.bank_count[1] = 3, 2, 1
    p = L.KnnParams()
    lib.tc_dtw_knn_params_default(C.byref(p))
    qd = (C.c_int32 * 2)(2, 4)
    ql = (C.c_int32 * 2)(6, 6)
    qb = L.Batch(0x4000, None, ql, 2, 0, 0, qd)
    assert lib.tc_dtw_knn_workspace_bytes(C.byref(ix), C.byref(qb), C.byref(p)) == 0
    st = lib.tc_dtw_knn(C.byref(ix), C.byref(qb), C.byref(p), C.c_void_p(0x5000), C.c_void_p(0x6000), None,
                        C.c_void_p(0x7000), 1 << 20, None)
    assert st == L.ERR_INVALID and b"no bank" in lib.tc_dtw_last_error()


def test_k_validated_on_the_host():
    """k-NN: k in 1..32 and at most the number of candidates; k > 1 needs
    uniform lengths.  Checked from the index description and the query
    shape alone (no device memory is touched)."""
    lib = L.lib()
    ix = L.Index()
    ix.buf = C.c_void_p(0x4000)
    ix.bytes = 1 << 20
    ix.count = 10
    ix.dim = 2
    ix.uniform_len = 8
    ix.max_len = 8
    ix.ntiles = 1
    Q = L.Batch(0x1000, None, None, 3, 2, 8, None)     # 3 queries of length 8, dim 2
    def ws(k):
        p = L.KnnParams()
        lib.tc_dtw_knn_params_default(C.byref(p))
        p.k = k
        return lib.tc_dtw_knn_workspace_bytes(C.byref(ix), C.byref(Q), C.byref(p)), p
    assert ws(1)[0] > 0 and ws(5)[0] > ws(1)[0] and ws(10)[0] > 0
    for bad in (0, -1, 11, 33):
        assert ws(bad)[0] == 0
    _, p = ws(33)
    st = lib.tc_dtw_knn(C.byref(ix), C.byref(Q), C.byref(p), C.c_void_p(0x100), C.c_void_p(0x200), None,
                        C.c_void_p(0x300), 1 << 20, None)
    assert st == L.ERR_UNSUPPORTED
    _, p = ws(11)
    st = lib.tc_dtw_knn(C.byref(ix), C.byref(Q), C.byref(p), C.c_void_p(0x100), C.c_void_p(0x200), None,
                        C.c_void_p(0x300), 1 << 20, None)
    assert st == L.ERR_INVALID
    # uneven query lengths (a ragged search) with k > 1
    lens = (C.c_int32 * 3)(8, 6, 7)
    offs = (C.c_int64 * 3)(0, 16, 28)
    Qr = L.Batch(0x1000, offs, lens, 3, 2, 0, None)
    _, p = ws(2)
    assert lib.tc_dtw_knn_workspace_bytes(C.byref(ix), C.byref(Qr), C.byref(p)) == 0


def test_independent_dtw_validated_on_the_host():
    """Independent DTW: LB_MV or no bounds, W_eff <= 63, up to 16 dimensions,
    uniform lengths; the flag is 0 or 1."""
    lib = L.lib()

    def index(dim, length):
        ix = L.Index()
        ix.buf = C.c_void_p(0x4000)
        ix.bytes = 1 << 20
        ix.count = 10
        ix.dim = dim
        ix.uniform_len = length
        ix.max_len = length
        ix.ntiles = 1
        return ix

    def ws(ix, Q, **kw):
        p = L.KnnParams()
        lib.tc_dtw_knn_params_default(C.byref(p))
        for k, v in kw.items():
            setattr(p, k, v)
        return lib.tc_dtw_knn_workspace_bytes(C.byref(ix), C.byref(Q), C.byref(p))

    ix = index(8, 64)
    Q = L.Batch(0x1000, None, None, 3, 8, 64, None)
    assert ws(ix, Q, independent=1) > 0
    assert ws(ix, Q, independent=1, bounds=0) > 0
    assert ws(ix, Q, independent=2) == 0
    assert ws(ix, Q, independent=1, bounds=L.LB_MV | L.LB_PC) == 0
    assert ws(ix, Q, independent=1, bounds=L.LB_MV | L.LB_TI) == 0
    ixw = index(20, 64)
    Qw = L.Batch(0x1000, None, None, 3, 20, 64, None)
    assert ws(ixw, Qw) > 0 and ws(ixw, Qw, independent=1) == 0          # 20 dimensions
    ixl = index(8, 1000)
    Ql = L.Batch(0x1000, None, None, 3, 8, 1000, None)
    assert ws(ixl, Ql) > 0 and ws(ixl, Ql, independent=1) == 0          # W = 100
    lens = (C.c_int32 * 3)(64, 60, 62)
    offs = (C.c_int64 * 3)(0, 512, 992)
    Qr = L.Batch(0x1000, offs, lens, 3, 8, 0, None)
    assert ws(ix, Qr) > 0 and ws(ix, Qr, independent=1) == 0            # uneven lengths


def test_candidate_boxes_validated_on_the_host():
    """Candidate-side LB_PC boxes: sized from the index, the query length and
    the LB_PC parameters; a search rejects a descriptor built for another
    query length, window or parameter set before any device call."""
    lib = L.lib()
    ix = L.Index()
    ix.buf = C.c_void_p(0x4000)
    ix.bytes = 1 << 20
    ix.count = 10
    ix.dim = 2
    ix.uniform_len = 64
    ix.max_len = 64
    ix.ntiles = 1
    p = L.KnnParams()
    lib.tc_dtw_knn_params_default(C.byref(p))
    nb = lib.tc_dtw_cand_boxes_bytes(C.byref(ix), 64, C.byref(p))
    groups = (64 + p.pc_group - 1) // p.pc_group
    boxes = 10 * groups * p.pc_clusters * 2 * 2 * 4
    assert nb == (boxes + 255) // 256 * 256 + 10 * groups * 4
    assert lib.tc_dtw_cand_boxes_bytes(C.byref(ix), 0, C.byref(p)) == 0
    assert lib.tc_dtw_cand_boxes_bytes(C.byref(ix), 64, None) == 0
    out = L.CandBoxes()
    st = lib.tc_dtw_build_cand_boxes(C.byref(ix), 64, C.byref(p), C.c_void_p(0x8000), nb - 1, C.byref(out), None)
    assert st == L.ERR_INVALID
    ixr = L.Index()
    C.memmove(C.byref(ixr), C.byref(ix), C.sizeof(ix))
    ixr.uniform_len = 0
    assert lib.tc_dtw_cand_boxes_bytes(C.byref(ixr), 64, C.byref(p)) == 0
    # a descriptor as tc_dtw_build_cand_boxes fills it for query length 64, W = 6
    d = L.CandBoxes(0x8000, (boxes + 255) // 256 * 256, 10, 2, 64, 64, 6, groups, p.pc_levels, p.pc_clusters,
                    p.pc_group, p.pc_min_cell)
    Q = L.Batch(0x1000, None, None, 3, 2, 64, None)

    def ws(**kw):
        q = L.KnnParams()
        lib.tc_dtw_knn_params_default(C.byref(q))
        q.bounds = L.LB_MV | L.LB_PC
        q.pc_cand = C.pointer(d)
        for k, v in kw.items():
            setattr(q, k, v)
        return lib.tc_dtw_knn_workspace_bytes(C.byref(ix), C.byref(Q), C.byref(q))

    assert ws() > 0
    assert ws(pc_clusters=5) == 0
    assert ws(pc_group=4) == 0
    assert ws(window=L.Window(0, 1, 5)) == 0
    Q32 = L.Batch(0x1000, None, None, 3, 2, 60, None)
    q = L.KnnParams()
    lib.tc_dtw_knn_params_default(C.byref(q))
    q.pc_cand = C.pointer(d)
    assert lib.tc_dtw_knn_workspace_bytes(C.byref(ix), C.byref(Q32), C.byref(q)) == 0


def test_noalloc_rejects_a_plan_beyond_its_scratch_on_the_host():
    """tc_dtw_banded_noalloc refuses a batch whose pair plan exceeds its static
    scratch with UNSUPPORTED before any HIP call (no device here), and its
    other argument checks are tc_dtw_banded's."""
    import numpy as np
    lib = L.lib()
    cap = lib.tc_dtw_noalloc_scratch_bytes()
    assert cap == 8 << 20
    n = cap // 48 + 10
    lens = np.full(n, 5, dtype=np.int32)
    lens[::2] = 6
    b = L.Batch(0x1000, None, lens.ctypes.data_as(C.POINTER(C.c_int32)), n, 2, 0, None)
    st = lib.tc_dtw_banded_noalloc(C.byref(b), C.byref(b), L.Window(0, 1, 10), 0, C.c_void_p(0x2000), None, None)
    assert st == L.ERR_UNSUPPORTED
    assert b"static scratch" in lib.tc_dtw_last_error()
    x = _batch()
    st = lib.tc_dtw_banded_noalloc(C.byref(x), C.byref(x), L.Window(2, 0, 0), 0, None, None, None)
    assert st == L.ERR_INVALID


def test_fake_no_device_and_sync_status(monkeypatch):
    """With TC_DTW_FAKE_NO_DEVICE set, calls that pass the host checks fail
    with ERR_DEVICE (named in the message) instead of touching a device;
    tc_dtw_sync_status reports the same."""
    lib = L.lib()
    monkeypatch.setenv("TC_DTW_FAKE_NO_DEVICE", "1")
    x = _batch()
    st = lib.tc_dtw_banded(C.byref(x), C.byref(x), L.Window(2, 0, 0), 0, C.c_void_p(0x2000), None, None, 0, None)
    assert st == L.ERR_DEVICE
    assert b"TC_DTW_FAKE_NO_DEVICE" in lib.tc_dtw_last_error()
    assert lib.tc_dtw_sync_status(None) == L.ERR_DEVICE
    # the host checks still come first
    st = lib.tc_dtw_banded(C.byref(x), C.byref(x), L.Window(-1, 0, 0), 0, C.c_void_p(0x2000), None, None, 0, None)
    assert st == L.ERR_INVALID


def test_reuse_query_meta_validated_on_the_host():
    """tc_dtw_knn_params.reuse_query_meta is 0 (copy the per-query metadata) or
    1 (reuse what an earlier call left in the workspace); anything else is
    refused before any device call, by the workspace query and the search."""
    lib = L.lib()
    ix = L.Index()
    ix.buf = C.c_void_p(0x4000)
    ix.bytes = 1 << 20
    ix.count = 10
    ix.dim = 2
    ix.uniform_len = 8
    ix.max_len = 8
    ix.ntiles = 1
    Q = L.Batch(0x1000, None, None, 3, 2, 8, None)
    p = L.KnnParams()
    lib.tc_dtw_knn_params_default(C.byref(p))
    assert p.reuse_query_meta == 0
    assert lib.tc_dtw_knn_workspace_bytes(C.byref(ix), C.byref(Q), C.byref(p)) > 0
    p.reuse_query_meta = 1
    assert lib.tc_dtw_knn_workspace_bytes(C.byref(ix), C.byref(Q), C.byref(p)) > 0
    for bad in (2, -1):
        p.reuse_query_meta = bad
        assert lib.tc_dtw_knn_workspace_bytes(C.byref(ix), C.byref(Q), C.byref(p)) == 0
        st = lib.tc_dtw_knn(C.byref(ix), C.byref(Q), C.byref(p), C.c_void_p(0x100), C.c_void_p(0x200), None,
                            C.c_void_p(0x300), 1 << 20, None)
        assert st == L.ERR_INVALID
        assert b"reuse_query_meta" in lib.tc_dtw_last_error()
