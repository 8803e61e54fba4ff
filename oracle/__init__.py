"""FP64 reference oracle for TC-DTW (arXiv 2101.07731) -- TEST INFRASTRUCTURE.

Only the test-suite, the package smoke check and the CPU-baseline leg of
the benchmark may import this package.  The GPU library never calls it and
shares no code with it.  Every function takes float32 or float64 arrays,
promotes them exactly to float64 and runs the plain C implementation in
``tcdtw_oracle.c`` (see the comments there for the paper passage each
function follows).

Series layout: one series is an [T, D] array; a set of series is either a
3-D array [N, T, D] or a list of [T_k, D] arrays (ragged lengths).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib(path=None):
    """Load the oracle library (building it first if it is not there).
    `path` loads another build of the same source instead (used by the
    test that plants mistakes in a copy of the oracle)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    if path is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        path = _build.LIB
    L = C.CDLL(path)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    lp = C.POINTER(C.c_int64)
    i, d = C.c_int, C.c_double
    L.orc_window_eff.argtypes = [i, i, i, i, i]
    L.orc_window_eff.restype = i
    L.orc_dtw.argtypes = [dp, i, dp, i, i, i]
    L.orc_dtw.restype = d
    L.orc_dtw_ea.argtypes = [dp, i, dp, i, i, i, d, C.POINTER(C.c_int)]
    L.orc_dtw_ea.restype = d
    L.orc_dtw_pairs.argtypes = [dp, lp, ip, dp, lp, ip, i, i, i, i, i, i, dp]
    L.orc_dtw_pairs.restype = None
    L.orc_dtw_path_grad.argtypes = [dp, i, dp, i, i, i, d, dp, dp, ip, ip]
    L.orc_dtw_path_grad.restype = d
    L.orc_envelope.argtypes = [dp, i, i, i, i, dp, dp]
    L.orc_envelope.restype = None
    for name in ("orc_lb_mv", "orc_lb_ad"):
        getattr(L, name).argtypes = [dp, i, dp, i, i, i]
        getattr(L, name).restype = d
    L.orc_lb_ti.argtypes = [dp, i, dp, i, i, i, i, i]
    L.orc_lb_ti.restype = d
    L.orc_ti_cells.argtypes = [dp, i, dp, i, i, i, i, i, dp, dp]
    L.orc_ti_cells.restype = None
    L.orc_pc_boxes.argtypes = [dp, i, i, i, i, i, i, i, C.c_float, dp, dp, ip]
    L.orc_pc_boxes.restype = i
    L.orc_lb_pc.argtypes = [dp, i, dp, i, i, i, i, i, i, C.c_float]
    L.orc_lb_pc.restype = d
    L.orc_knn_exhaustive.argtypes = [dp, lp, ip, i, dp, lp, ip, i, i, i, i, i, i, ip, dp]
    L.orc_knn_exhaustive.restype = None
    L.orc_knn_cascade.argtypes = [dp, lp, ip, i, dp, lp, ip, i, i, i, i, i, C.c_uint32,
                                  i, i, i, i, i, C.c_float, d, d, i, ip, dp,
                                  C.POINTER(CascadeStats)]
    L.orc_knn_cascade.restype = None
    _lib = L
    return L


class CascadeStats(C.Structure):
    _fields_ = [("pairs", C.c_int64), ("pruned_mv", C.c_int64), ("pruned_pc", C.c_int64),
                ("pruned_ti", C.c_int64), ("dtw_started", C.c_int64),
                ("dtw_abandoned", C.c_int64)]


def _f64(a):
    a = np.ascontiguousarray(np.asarray(a), dtype=np.float64)
    return a


def _ptr(a, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


def _series(x):
    x = _f64(x)
    if x.ndim == 1:
        x = x[:, None]
    assert x.ndim == 2, "a series is a [T, D] array"
    return x


def _set(xs):
    """Concatenate a set of series -> (flat float64, offsets int64, lengths int32, D)."""
    if isinstance(xs, np.ndarray) and xs.ndim == 3:
        N, T, D = xs.shape
        flat = _f64(xs).reshape(-1)
        off = (np.arange(N, dtype=np.int64) * T * D)
        lens = np.full(N, T, dtype=np.int32)
        return flat, off, lens, D
    arrs = [_series(s) for s in xs]
    D = arrs[0].shape[1]
    assert all(a.shape[1] == D for a in arrs), "one dimension per set"
    lens = np.array([a.shape[0] for a in arrs], dtype=np.int32)
    off = np.zeros(len(arrs), dtype=np.int64)
    if len(arrs) > 1:
        off[1:] = np.cumsum(lens[:-1].astype(np.int64) * D)
    flat = np.concatenate([a.reshape(-1) for a in arrs]) if arrs else np.zeros(0)
    return np.ascontiguousarray(flat), off, lens, D


def window_eff(m, n, window=0, num=0, den=0):
    """max(W, |m-n|) with W = floor(max(m,n)*num/den) if den > 0 else window."""
    return lib().orc_window_eff(int(m), int(n), int(window), int(num), int(den))


def dtw(q, c, weff):
    q, c = _series(q), _series(c)
    return lib().orc_dtw(_ptr(q), q.shape[0], _ptr(c), c.shape[0], q.shape[1], int(weff))


def dtw_ea(q, c, weff, bsf):
    q, c = _series(q), _series(c)
    ab = C.c_int(0)
    v = lib().orc_dtw_ea(_ptr(q), q.shape[0], _ptr(c), c.shape[0], q.shape[1], int(weff),
                         float(bsf), C.byref(ab))
    return v, bool(ab.value)


def dtw_pairs(xs, ys, window=0, num=0, den=0, threads=None):
    """DTW of pairs (xs[k], ys[k]); window per pair from (window, num, den)."""
    xf, xo, xl, D = _set(xs)
    yf, yo, yl, D2 = _set(ys)
    assert D == D2 and len(xl) == len(yl)
    out = np.zeros(len(xl), dtype=np.float64)
    threads = threads or os.cpu_count() or 1
    lib().orc_dtw_pairs(_ptr(xf), _ptr(xo, C.c_int64), _ptr(xl, C.c_int32),
                        _ptr(yf), _ptr(yo, C.c_int64), _ptr(yl, C.c_int32),
                        len(xl), D, int(window), int(num), int(den), int(threads), _ptr(out))
    return out


def path_grad(q, c, weff, gbar=1.0):
    """-> (dtw, grad_q [m,D], grad_c [n,D], path [(i,j), ...] from the end back to (0,0))."""
    q, c = _series(q), _series(c)
    m, n, D = q.shape[0], c.shape[0], q.shape[1]
    gq = np.zeros((m, D))
    gc = np.zeros((n, D))
    path = np.zeros(2 * (m + n), dtype=np.int32)
    plen = C.c_int32(0)
    v = lib().orc_dtw_path_grad(_ptr(q), m, _ptr(c), n, D, int(weff), float(gbar),
                                _ptr(gq), _ptr(gc), _ptr(path, C.c_int32), C.byref(plen))
    return v, gq, gc, path[:2 * plen.value].reshape(-1, 2)


def envelope(q, n, weff):
    q = _series(q)
    m, D = q.shape
    U = np.zeros((n, D))
    L = np.zeros((n, D))
    lib().orc_envelope(_ptr(q), m, int(n), D, int(weff), _ptr(U), _ptr(L))
    return U, L


def lb_mv(q, c, weff):
    q, c = _series(q), _series(c)
    return lib().orc_lb_mv(_ptr(q), q.shape[0], _ptr(c), c.shape[0], q.shape[1], int(weff))


def lb_ad(q, c, weff):
    q, c = _series(q), _series(c)
    return lib().orc_lb_ad(_ptr(q), q.shape[0], _ptr(c), c.shape[0], q.shape[1], int(weff))


def lb_ti(q, c, weff, P=5, top=1):
    q, c = _series(q), _series(c)
    return lib().orc_lb_ti(_ptr(q), q.shape[0], _ptr(c), c.shape[0], q.shape[1], int(weff),
                           int(P), int(top))


def ti_cells(q, c, weff, P=5, top=1):
    q, c = _series(q), _series(c)
    m, n = q.shape[0], c.shape[0]
    Lo = np.zeros((m, n))
    Hi = np.zeros((m, n))
    lib().orc_ti_cells(_ptr(q), m, _ptr(c), n, q.shape[1], int(weff), int(P), int(top),
                       _ptr(Lo), _ptr(Hi))
    return Lo, Hi


def pc_boxes(q, n, weff, Lv=2, K=6, w=6, floor_len=1e-5):
    """-> (box_lo [G,K,D], box_hi [G,K,D], nbox [G]); unused box slots hold +inf/-inf."""
    q = _series(q)
    m, D = q.shape
    G = (n + w - 1) // w
    lo = np.zeros((G, K, D))
    hi = np.zeros((G, K, D))
    nb = np.zeros(G, dtype=np.int32)
    r = lib().orc_pc_boxes(_ptr(q), m, int(n), D, int(weff), int(Lv), int(K), int(w),
                           float(floor_len), _ptr(lo), _ptr(hi), _ptr(nb, C.c_int32))
    if r < 0:
        raise ValueError("Lv**D does not fit in 63 bits")
    return lo, hi, nb


def lb_pc(q, c, weff, Lv=2, K=6, w=6, floor_len=1e-5):
    q, c = _series(q), _series(c)
    return lib().orc_lb_pc(_ptr(q), q.shape[0], _ptr(c), c.shape[0], q.shape[1], int(weff),
                           int(Lv), int(K), int(w), float(floor_len))


def knn_exhaustive(Q, Cs, window=0, num=0, den=0, threads=None):
    """Plain 1-NN: -> (nn_idx int32 [nq], nn_dist float64 [nq]); ties to the lowest index."""
    qf, qo, ql, D = _set(Q)
    cf, co, cl, D2 = _set(Cs)
    assert D == D2
    nq = len(ql)
    idx = np.zeros(nq, dtype=np.int32)
    dist = np.zeros(nq, dtype=np.float64)
    threads = threads or os.cpu_count() or 1
    lib().orc_knn_exhaustive(_ptr(qf), _ptr(qo, C.c_int64), _ptr(ql, C.c_int32), nq,
                             _ptr(cf), _ptr(co, C.c_int64), _ptr(cl, C.c_int32), len(cl),
                             D, int(window), int(num), int(den), int(threads),
                             _ptr(idx, C.c_int32), _ptr(dist))
    return idx, dist


def dtw_indep(q, c, weff):
    """Independent multivariate DTW (Sec. 2: DTW_I): the univariate banded
    DTW of every dimension with its own warping path, summed over the
    dimensions in increasing order."""
    q, c = _series(q), _series(c)
    total = 0.0
    for p in range(q.shape[1]):
        total = total + dtw(q[:, p:p + 1], c[:, p:p + 1], weff)
    return total


def knn_exhaustive_k(Q, Cs, k, window=0, num=0, den=0, threads=None, independent=False):
    """Plain k-NN (the 1-NN definition of Sec. 2 extended to the k nearest):
    the float64 banded DTW of every (query, reference) pair -- dependent
    (one warping path for all dimensions) or, with `independent`, DTW_I as
    in dtw_indep -- then per query the k references with the smallest
    distance, ordered by (distance, index) so that ties go to the lower
    index.  -> (idx int32 [nq, k], dist float64 [nq, k])."""
    Qs = [np.asarray(q) for q in Q]
    Rs = [np.asarray(c) for c in Cs]
    nq, nc = len(Qs), len(Rs)
    assert 1 <= k <= nc
    xs = [q for q in Qs for _ in range(nc)]
    ys = [c for _ in range(nq) for c in Rs]
    if independent:
        D = Qs[0].shape[1]
        d = np.zeros(nq * nc)
        for p in range(D):   # per-dimension DTWs added in increasing dimension order
            d = d + dtw_pairs([x[:, p:p + 1] for x in xs], [y[:, p:p + 1] for y in ys], window=window,
                              num=num, den=den, threads=threads)
        d = d.reshape(nq, nc)
    else:
        d = dtw_pairs(xs, ys, window=window, num=num, den=den, threads=threads).reshape(nq, nc)
    idx = np.zeros((nq, k), dtype=np.int32)
    dist = np.zeros((nq, k), dtype=np.float64)
    refs = np.arange(nc)
    for i in range(nq):
        order = np.lexsort((refs, d[i]))[:k]     # primary key: distance; then index
        idx[i] = order
        dist[i] = d[i, order]
    return idx, dist


def knn_cascade(Q, Cs, window=0, num=0, den=0, bounds=6, ti_P=5, ti_top=1, pc_Lv=2, pc_K=6,
                pc_w=6, pc_floor=1e-5, e_ti=0.1, e_pc=0.1, threads=None):
    """The paper's sequential cascade -> (nn_idx, nn_dist, per-query stats dict of arrays)."""
    qf, qo, ql, D = _set(Q)
    cf, co, cl, D2 = _set(Cs)
    assert D == D2
    nq = len(ql)
    idx = np.zeros(nq, dtype=np.int32)
    dist = np.zeros(nq, dtype=np.float64)
    st = (CascadeStats * nq)()
    threads = threads or os.cpu_count() or 1
    lib().orc_knn_cascade(_ptr(qf), _ptr(qo, C.c_int64), _ptr(ql, C.c_int32), nq,
                          _ptr(cf), _ptr(co, C.c_int64), _ptr(cl, C.c_int32), len(cl),
                          D, int(window), int(num), int(den), int(bounds), int(ti_P),
                          int(ti_top), int(pc_Lv), int(pc_K), int(pc_w), float(pc_floor),
                          float(e_ti), float(e_pc), int(threads),
                          _ptr(idx, C.c_int32), _ptr(dist), st)
    stats = {f: np.array([getattr(s, f) for s in st], dtype=np.int64)
             for f, _ in CascadeStats._fields_}
    return idx, dist, stats
