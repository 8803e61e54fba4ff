"""Python binding of the pair calls of the C ABI: tc_dtw_banded,
tc_dtw_backward, the reusable pair plans (tc_dtw_pairs_plan_*, with a
timing autotuner and HIP-graph replay), plus DTWLoss
(torch.autograd.Function).

Series sets are float32 CUDA tensors [B, T, D] (uniform lengths) or lists
of [T_k, D_k] tensors (ragged lengths and dims).  torch provides device
memory, the current stream and graph capture only; all arithmetic runs in
the library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def window_spec(window=None, frac=None):
    """Window as (W, num, den): an absolute half-width or a fraction num/den of max(m, n)."""
    if frac is not None:
        num, den = frac
        return L.Window(0, int(num), int(den))
    return L.Window(int(window or 0), 0, 0)


class SeriesSet:
    """A set of series on the device and its C-ABI batch descriptor (host metadata kept alive).

    A [B, T, D] tensor is a uniform set; a list of [T_k, D_k] tensors is a
    ragged one (lengths and dims may differ per series)."""

    def __init__(self, xs):
        self.dims = None
        if isinstance(xs, torch.Tensor):
            if xs.dim() != 3:
                raise ValueError("a uniform set is a [B, T, D] tensor")
            if xs.dtype != torch.float32 or not xs.is_cuda:
                raise ValueError("series must be float32 CUDA tensors")
            self.flat = xs.contiguous()
            self.shape = tuple(xs.shape)
            self.lens = None
            self.batch = L.Batch(self.flat.data_ptr(), None, None, xs.shape[0], xs.shape[2], xs.shape[1], None)
        else:
            xs = list(xs)
            if not xs:
                raise ValueError("empty series set")
            for t in xs:
                if t.dim() != 2 or t.dtype != torch.float32 or not t.is_cuda:
                    raise ValueError("ragged sets are lists of float32 CUDA [T, D] tensors")
            dims = np.array([t.shape[1] for t in xs], dtype=np.int32)
            self.flat = torch.cat([t.reshape(-1) for t in xs]).contiguous()
            self.lens = np.array([t.shape[0] for t in xs], dtype=np.int32)
            self.offs = np.zeros(len(xs), dtype=np.int64)
            if len(xs) > 1:
                self.offs[1:] = np.cumsum(self.lens[:-1].astype(np.int64) * dims[:-1])
            self.shape = None
            self.dimv = dims
            mixed = bool(np.any(dims != dims[0]))
            if mixed:
                self.dims = dims
            self.batch = L.Batch(self.flat.data_ptr(),
                                 self.offs.ctypes.data_as(C.POINTER(C.c_int64)),
                                 self.lens.ctypes.data_as(C.POINTER(C.c_int32)),
                                 len(xs), int(dims[0]), 0,
                                 self.dims.ctypes.data_as(C.POINTER(C.c_int32)) if mixed else None)

    @property
    def count(self):
        return self.batch.count

    def split(self, flat):
        """Reshape a flat tensor laid out like this set back into its shape."""
        if self.shape is not None:
            return flat.view(self.shape)
        return [flat[o:o + n * d].view(n, d)
                for o, n, d in zip(self.offs.tolist(), self.lens.tolist(), self.dimv.tolist())]


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def banded(x, y, window=None, frac=(1, 10), f64=False, save=False):
    """DTW of each pair (x[b], y[b]) within the Sakoe-Chiba band.

    Returns dist (float32 [B]) or (dist, saved) when save=True; `saved`
    holds the argmin codes that `backward` needs."""
    X, Y = SeriesSet(x), SeriesSet(y)
    win = window_spec(window, frac)
    lib = L.lib()
    flags = L.F64 if f64 else 0
    dev = X.flat.device
    dist = torch.empty(X.count, dtype=torch.float32, device=dev)
    wsb = lib.tc_dtw_banded_workspace_bytes(C.byref(X.batch), C.byref(Y.batch), win, flags)
    ws = _workspace(wsb, dev)
    saved = None
    if save:
        sb = lib.tc_dtw_saved_bytes(C.byref(X.batch), C.byref(Y.batch), win)
        saved = torch.empty(max(sb, 4), dtype=torch.uint8, device=dev)
    L.check(lib.tc_dtw_banded(C.byref(X.batch), C.byref(Y.batch), win, flags,
                              C.c_void_p(dist.data_ptr()),
                              C.c_void_p(saved.data_ptr()) if saved is not None else None,
                              C.c_void_p(ws.data_ptr()), wsb, _stream()))
    return (dist, saved) if save else dist


def banded_noalloc(x, y, window=None, frac=(1, 10), f64=False, saved=None, dist=None):
    """As banded, through tc_dtw_banded_noalloc: the library's static scratch
    instead of a workspace (the caller passes the outputs; `saved` may be a
    buffer of tc_dtw_saved_bytes() bytes to record the argmin codes)."""
    X, Y = SeriesSet(x), SeriesSet(y)
    win = window_spec(window, frac)
    dev = X.flat.device
    if dist is None:
        dist = torch.empty(X.count, dtype=torch.float32, device=dev)
    L.check(L.lib().tc_dtw_banded_noalloc(C.byref(X.batch), C.byref(Y.batch), win, L.F64 if f64 else 0,
                                          C.c_void_p(dist.data_ptr()),
                                          C.c_void_p(saved.data_ptr()) if saved is not None else None,
                                          _stream()))
    return dist


def saved_bytes(x, y, window=None, frac=(1, 10)):
    X, Y = SeriesSet(x), SeriesSet(y)
    return L.lib().tc_dtw_saved_bytes(C.byref(X.batch), C.byref(Y.batch), window_spec(window, frac))


def backward(x, y, saved, grad_dist, window=None, frac=(1, 10)):
    """Gradients (grad_x, grad_y) of sum_b grad_dist[b] * DTW(x[b], y[b]) along the saved paths."""
    X, Y = SeriesSet(x), SeriesSet(y)
    win = window_spec(window, frac)
    lib = L.lib()
    dev = X.flat.device
    gd = grad_dist.to(device=dev, dtype=torch.float32).contiguous()
    gx = torch.empty_like(X.flat)
    gy = torch.empty_like(Y.flat)
    wsb = lib.tc_dtw_backward_workspace_bytes(C.byref(X.batch), C.byref(Y.batch), win)
    ws = _workspace(wsb, dev)
    L.check(lib.tc_dtw_backward(C.byref(X.batch), C.byref(Y.batch), win,
                                C.c_void_p(saved.data_ptr()), C.c_void_p(gd.data_ptr()),
                                C.c_void_p(gx.data_ptr()), C.c_void_p(gy.data_ptr()),
                                C.c_void_p(ws.data_ptr()), wsb, _stream()))
    return X.split(gx), Y.split(gy)


class DTWLoss(torch.autograd.Function):
    """dist[b] = DTW(x[b], y[b]) for uniform [B, T, D] float32 CUDA tensors;
    the backward is the adjoint along each pair's optimal warping path."""

    @staticmethod
    def forward(ctx, x, y, window=None, frac=(1, 10), f64=False):
        dist, saved = banded(x.detach(), y.detach(), window=window, frac=frac, f64=f64, save=True)
        ctx.save_for_backward(x, y, saved)
        ctx.win = (window, frac)
        return dist

    @staticmethod
    def backward(ctx, grad_dist):
        x, y, saved = ctx.saved_tensors
        window, frac = ctx.win
        gx, gy = backward(x.detach(), y.detach(), saved, grad_dist, window=window, frac=frac)
        return gx, gy, None, None, None


class Plan:
    """A reusable plan of a batch of pairs (tc_dtw_pairs_plan_build).

    The plan fixes lengths, dims, windows and the mapping of every pair;
    `forward` / `backward` only enqueue kernels, so they may be captured in
    a CUDA (HIP) graph.  Data passed to them must be laid out like x and y
    (the flat buffers of SeriesSet)."""

    def __init__(self, x, y, window=None, frac=(1, 10), diag_max_w=63, waves_per_cu=0, waves_per_pair=0):
        self.X, self.Y = SeriesSet(x), SeriesSet(y)
        self.win = window_spec(window, frac)
        self.tuning = L.Tuning(int(diag_max_w), int(waves_per_cu), int(waves_per_pair))
        lib = L.lib()
        dev = self.X.flat.device
        nb = lib.tc_dtw_pairs_plan_bytes(C.byref(self.X.batch), C.byref(self.Y.batch), self.win,
                                         C.byref(self.tuning))
        if nb == 0:
            L.check(lib.tc_dtw_pairs_plan_build(C.byref(self.X.batch), C.byref(self.Y.batch), self.win,
                                                C.byref(self.tuning), None, 0, None, _stream()))
        self.buf = _workspace(nb, dev)
        self.plan = L.PairsPlan()
        L.check(lib.tc_dtw_pairs_plan_build(C.byref(self.X.batch), C.byref(self.Y.batch), self.win,
                                            C.byref(self.tuning), C.c_void_p(self.buf.data_ptr()), nb,
                                            C.byref(self.plan), _stream()))
        self.device = dev

    @property
    def count(self):
        return self.plan.npairs

    def saved_buffer(self):
        return torch.empty(max(int(self.plan.saved_bytes), 4), dtype=torch.uint8, device=self.device)

    def forward(self, x_flat=None, y_flat=None, dist=None, saved=None, f64=False):
        """dist[b] = DTW of pair b; records argmin codes into `saved` when given."""
        xf = self.X.flat if x_flat is None else x_flat
        yf = self.Y.flat if y_flat is None else y_flat
        if dist is None:
            dist = torch.empty(self.count, dtype=torch.float32, device=self.device)
        L.check(L.lib().tc_dtw_banded_run(C.byref(self.plan), C.c_void_p(xf.data_ptr()),
                                          C.c_void_p(yf.data_ptr()), L.F64 if f64 else 0,
                                          C.c_void_p(dist.data_ptr()),
                                          C.c_void_p(saved.data_ptr()) if saved is not None else None,
                                          _stream()))
        return dist

    def backward(self, saved, grad_dist, x_flat=None, y_flat=None, grad_x=None, grad_y=None):
        """Flat gradients (grad_x, grad_y) along the paths recorded in `saved`."""
        xf = self.X.flat if x_flat is None else x_flat
        yf = self.Y.flat if y_flat is None else y_flat
        gx = torch.empty_like(xf) if grad_x is None else grad_x
        gy = torch.empty_like(yf) if grad_y is None else grad_y
        L.check(L.lib().tc_dtw_backward_run(C.byref(self.plan), C.c_void_p(xf.data_ptr()),
                                            C.c_void_p(yf.data_ptr()), C.c_void_p(saved.data_ptr()),
                                            C.c_void_p(grad_dist.data_ptr()), C.c_void_p(gx.data_ptr()),
                                            C.c_void_p(gy.data_ptr()), _stream()))
        return gx, gy

    def classes(self):
        """The plan's launches: (mapping, dim class, pairs, max m, max n, max W_eff, waves per pair)."""
        return [("rows" if c.rows else "diag", c.dim, c.nitems, c.maxm, c.maxn, c.maxw, c.waves_per_pair)
                for c in self.plan.cls[:self.plan.nclasses]]


class GraphedForward:
    """A plan's forward captured once in a CUDA (HIP) graph; `replay` reruns it
    on the static buffers (copy new data into .x_flat / .y_flat first)."""

    def __init__(self, plan, save=False):
        self.plan = plan
        self.x_flat = plan.X.flat
        self.y_flat = plan.Y.flat
        self.dist = torch.empty(plan.count, dtype=torch.float32, device=plan.device)
        self.saved = plan.saved_buffer() if save else None
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):   # warm-up outside the capture
            plan.forward(self.x_flat, self.y_flat, self.dist, self.saved)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            plan.forward(self.x_flat, self.y_flat, self.dist, self.saved)

    def replay(self):
        self.graph.replay()
        return self.dist


_TUNED = {}

DIAG_CHOICES = (-1, 31, 63)
WAVE_CHOICES = (8, 16, 24)
PAIR_CHOICES = (1, 4, 8)


def shape_key(x, y, window=None, frac=(1, 10)):
    """Key of a batch's shapes (lengths and dims of every pair, and the window)."""
    X, Y = SeriesSet(x), SeriesSet(y)
    def desc(S):
        if S.shape is not None:
            return ("u",) + tuple(S.shape)
        return ("r", S.lens.tobytes(), S.dimv.tobytes())
    return (desc(X), desc(Y), window, frac)


def autotune(x, y, window=None, frac=(1, 10), reps=3, diag_choices=DIAG_CHOICES, wave_choices=WAVE_CHOICES,
             pair_choices=PAIR_CHOICES):
    """Times the plan's forward for every (diag_max_w, waves_per_cu,
    waves_per_pair) choice and returns (best choice, {choice: ms}); the best
    choice is remembered per shape key (see `tuned_plan`)."""
    key = shape_key(x, y, window, frac)
    times = {}
    for dm in diag_choices:
        for wv in wave_choices:
            for wp in pair_choices:
                plan = Plan(x, y, window=window, frac=frac, diag_max_w=dm, waves_per_cu=wv, waves_per_pair=wp)
                dist = torch.empty(plan.count, dtype=torch.float32, device=plan.device)
                plan.forward(dist=dist)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    plan.forward(dist=dist)
                e1.record()
                torch.cuda.synchronize()
                times[(dm, wv, wp)] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    _TUNED[key] = best
    return best, times


def tuned_plan(x, y, window=None, frac=(1, 10), **kw):
    """A Plan with the autotuned choice for this shape key (tuning on first use)."""
    key = shape_key(x, y, window, frac)
    if key not in _TUNED:
        autotune(x, y, window=window, frac=frac, **kw)
    dm, wv, wp = _TUNED[key]
    return Plan(x, y, window=window, frac=frac, diag_max_w=dm, waves_per_cu=wv, waves_per_pair=wp)
