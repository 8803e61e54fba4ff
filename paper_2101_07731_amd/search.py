"""Python binding of the search calls of the C ABI: tc_dtw_build_index,
tc_dtw_lower_bounds and tc_dtw_knn (argument marshalling only; torch
provides device memory and the current stream)."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .pairs import SeriesSet, _stream, _workspace, window_spec

BOUNDS = {"plain": 0, "mv": L.LB_MV, "mv+pc": L.LB_MV | L.LB_PC, "mv+ti": L.LB_MV | L.LB_TI,
          "mv+pc+ti": L.LB_MV | L.LB_PC | L.LB_TI}


class Index:
    """A candidate set prepared for searches (device buffer owned by this object)."""

    def __init__(self, refs):
        self.refs = SeriesSet(refs)
        lib = L.lib()
        nbytes = lib.tc_dtw_index_bytes(C.byref(self.refs.batch))
        if nbytes == 0:
            L.check(L.ERR_INVALID)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.refs.flat.device)
        self.ix = L.Index()
        L.check(lib.tc_dtw_build_index(C.byref(self.refs.batch), C.c_void_p(self.buf.data_ptr()), nbytes,
                                       C.byref(self.ix), _stream()))

    @property
    def count(self):
        return self.ix.count


def params(window=None, frac=(1, 10), bounds="mv", **kw):
    """tc_dtw_knn_params from keyword arguments (names as in the C struct;
    pc_cand takes a CandBoxes object)."""
    p = L.KnnParams()
    L.lib().tc_dtw_knn_params_default(C.byref(p))
    p.window = window_spec(window, frac)
    p.bounds = BOUNDS[bounds] if isinstance(bounds, str) else int(bounds)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError("unknown search parameter " + k)
        if k == "pc_cand":
            v = C.pointer(v.desc) if v is not None else None
        setattr(p, k, v)
    return p


class CandBoxes:
    """Candidate-side LB_PC boxes of an index (tc_dtw_build_cand_boxes; the
    roles of Sec. 5 swapped, as Sec. 8 suggests), built once for a query
    length, window and LB_PC parameters, and passed to searches as
    pc_cand=... with the same parameters.  Owns its device buffer."""

    def __init__(self, index, query_len, **kw):
        p = params(**kw)
        lib = L.lib()
        nbytes = lib.tc_dtw_cand_boxes_bytes(C.byref(index.ix), int(query_len), C.byref(p))
        if nbytes == 0:
            L.check(lib.tc_dtw_build_cand_boxes(C.byref(index.ix), int(query_len), C.byref(p), None, 0,
                                                None, _stream()))
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=index.buf.device)
        self.desc = L.CandBoxes()
        L.check(lib.tc_dtw_build_cand_boxes(C.byref(index.ix), int(query_len), C.byref(p),
                                            C.c_void_p(self.buf.data_ptr()), nbytes, C.byref(self.desc),
                                            _stream()))


def lower_bounds(index, queries, kind="mv", **kw):
    """Dense bound matrix [nq, nc] of one kind ('mv', 'pc' or 'ti')."""
    Q = SeriesSet(queries)
    p = params(bounds="mv", **kw)
    k = {"mv": L.LB_MV, "pc": L.LB_PC, "ti": L.LB_TI}[kind]
    lib = L.lib()
    lb = torch.empty((Q.count, index.count), dtype=torch.float32, device=Q.flat.device)
    wsb = lib.tc_dtw_lower_bounds_workspace_bytes(C.byref(index.ix), C.byref(Q.batch), C.byref(p), k)
    if wsb == 0:
        L.check(L.ERR_INVALID)
    ws = _workspace(wsb, Q.flat.device)
    L.check(lib.tc_dtw_lower_bounds(C.byref(index.ix), C.byref(Q.batch), C.byref(p), k,
                                    C.c_void_p(lb.data_ptr()), C.c_void_p(ws.data_ptr()), wsb, _stream()))
    return lb


def knn(index, queries, stats=False, workspace=None, k=1, **kw):
    """k nearest neighbours of every query: (nn_idx int32, nn_dist float32
    [, stats dict]), shaped [nq] for k = 1 and [nq, k] otherwise (ascending
    distance, ties to the lower index)."""
    Q = SeriesSet(queries)
    p = params(k=k, **kw)
    lib = L.lib()
    dev = Q.flat.device
    shape = (Q.count,) if k == 1 else (Q.count, k)
    idx = torch.empty(shape, dtype=torch.int32, device=dev)
    dist = torch.empty(shape, dtype=torch.float32, device=dev)
    wsb = lib.tc_dtw_knn_workspace_bytes(C.byref(index.ix), C.byref(Q.batch), C.byref(p))
    if wsb == 0:
        L.check(lib.tc_dtw_knn(C.byref(index.ix), C.byref(Q.batch), C.byref(p), None, None, None, None, 0,
                               _stream()))
    ws = workspace if workspace is not None and workspace.numel() >= wsb else _workspace(wsb, dev)
    st = L.KnnStats() if stats else None
    L.check(lib.tc_dtw_knn(C.byref(index.ix), C.byref(Q.batch), C.byref(p), C.c_void_p(idx.data_ptr()),
                           C.c_void_p(dist.data_ptr()), C.byref(st) if st is not None else None,
                           C.c_void_p(ws.data_ptr()), wsb, _stream()))
    if not stats:
        return idx, dist
    sd = {f: getattr(st, f) for f, _ in L.KnnStats._fields_ if f != "stage_ms"}
    sd["stage_ms"] = list(st.stage_ms)
    return idx, dist, sd


class GraphedSearch:
    """A whole search (every stage of the cascade, tc_dtw_knn) captured once in
    a CUDA (HIP) graph for fixed shapes; `replay` reruns it with no host work.
    New queries of the same shapes go into `.queries_flat` (the flat buffer of
    the captured batch).  Queries of uneven lengths or dims work too: the
    warm-up call copies their metadata into the workspace and the captured
    call reuses it (params.reuse_query_meta)."""

    def __init__(self, index, queries, k=1, **kw):
        self.Q = SeriesSet(queries)
        self.queries_flat = self.Q.flat
        self.index = index
        lib = L.lib()
        dev = self.Q.flat.device
        p = params(k=k, **kw)
        wsb = lib.tc_dtw_knn_workspace_bytes(C.byref(index.ix), C.byref(self.Q.batch), C.byref(p))
        if wsb == 0:
            L.check(lib.tc_dtw_knn(C.byref(index.ix), C.byref(self.Q.batch), C.byref(p), None, None, None, None,
                                   0, _stream()))
        self.ws = _workspace(wsb, dev)
        shape = (self.Q.count,) if k == 1 else (self.Q.count, k)
        self.idx = torch.empty(shape, dtype=torch.int32, device=dev)
        self.dist = torch.empty(shape, dtype=torch.float32, device=dev)

        def call(reuse):
            p.reuse_query_meta = 1 if reuse else 0
            L.check(lib.tc_dtw_knn(C.byref(index.ix), C.byref(self.Q.batch), C.byref(p),
                                   C.c_void_p(self.idx.data_ptr()), C.c_void_p(self.dist.data_ptr()), None,
                                   C.c_void_p(self.ws.data_ptr()), wsb, _stream()))

        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):   # warm-up outside the capture (writes the query metadata)
            call(False)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            call(True)

    def replay(self):
        self.graph.replay()
        return self.idx, self.dist


def knn_workspace_bytes(index, queries, **kw):
    Q = SeriesSet(queries)
    p = params(**kw)
    return L.lib().tc_dtw_knn_workspace_bytes(C.byref(index.ix), C.byref(Q.batch), C.byref(p))


def _choices():
    """The setup-stage grid of Sec. 6 / Sec. 7.1: LB_MV alone; LB_PC with
    Lv in {2, 3} levels and e_PC in {0.1, 0.5}; LB_TI (P = 5 with TOP) with
    e_TI in {0.05, 0.1, 0.2}; both advanced bounds at two trigger pairs and
    both Lv.  Each choice is a dict of tc_dtw_knn_params fields plus
    'bounds'; the box count K (pc_clusters) is passed to tune_cascade."""
    out = [{"bounds": "mv"}]
    for lv in (2, 3):
        for e in (0.1, 0.5):
            out.append({"bounds": "mv+pc", "pc_levels": lv, "trigger_pc": e})
    for e in (0.05, 0.1, 0.2):
        out.append({"bounds": "mv+ti", "trigger_ti": e})
    for lv in (2, 3):
        for epc, eti in ((0.1, 0.1), (0.5, 0.2)):
            out.append({"bounds": "mv+pc+ti", "pc_levels": lv, "trigger_pc": epc, "trigger_ti": eti})
    return tuple(out)


CASCADE_CHOICES = _choices()

# setup-stage choices already made, by (index, query shape, window and other parameters)
_TUNED = {}


def choice_name(c):
    return " ".join("%s=%s" % (k, v) for k, v in sorted(c.items()))


def tune_cascade(index, queries, reps=2, choices=CASCADE_CHOICES, cache=True, **kw):
    """Setup-stage choice of the bounds and their parameters (Sec. 6: the
    triggering threshold and the bound are chosen per dataset during setup;
    Sec. 7.1 lists the grids): times the search of `queries` (a sample) for
    every choice and returns (best choice dict, {choice name: ms}).  Every
    choice returns the same neighbours; only the time differs.  The result
    is cached by the index, the query shape and the other parameters, so a
    later call with the same key returns it without timing (pass
    cache=False to time again); apply it with knn(index, q, **best, **kw)."""
    Q = SeriesSet(queries)
    key = (int(index.buf.data_ptr()), int(index.count), Q.shape, Q.count if Q.shape is None else None,
           tuple(sorted((k, str(v)) for k, v in kw.items())), tuple(choice_name(c) for c in choices))
    if cache and key in _TUNED:
        return _TUNED[key]
    times = {}
    for c in choices:
        args = dict(kw)
        args.update(c)
        try:
            knn(index, queries, **args)
        except L.TcDtwError as err:
            if err.status == L.ERR_UNSUPPORTED:
                continue
            raise
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            knn(index, queries, **args)
        e1.record()
        torch.cuda.synchronize()
        times[choice_name(c)] = e0.elapsed_time(e1) / reps
    by_name = {choice_name(c): c for c in choices}
    best = dict(by_name[min(times, key=times.get)])
    _TUNED[key] = (best, times)
    return best, times
