"""Python binding of the pair calls of the C ABI: tc_dtw_banded and
tc_dtw_backward, plus DTWLoss (torch.autograd.Function).

Series sets are float32 CUDA tensors [B, T, D] (uniform lengths) or lists
of [T_k, D] tensors (ragged lengths).  torch provides device memory and the
current stream only; all arithmetic runs in the library's kernels.
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
    """A set of series on the device and its C-ABI batch descriptor (host metadata kept alive)."""

    def __init__(self, xs):
        if isinstance(xs, torch.Tensor):
            if xs.dim() != 3:
                raise ValueError("a uniform set is a [B, T, D] tensor")
            if xs.dtype != torch.float32 or not xs.is_cuda:
                raise ValueError("series must be float32 CUDA tensors")
            self.flat = xs.contiguous()
            self.shape = tuple(xs.shape)
            self.lens = None
            self.batch = L.Batch(self.flat.data_ptr(), None, None, xs.shape[0], xs.shape[2], xs.shape[1])
        else:
            xs = list(xs)
            if not xs:
                raise ValueError("empty series set")
            D = xs[0].shape[1]
            for t in xs:
                if t.dim() != 2 or t.shape[1] != D or t.dtype != torch.float32 or not t.is_cuda:
                    raise ValueError("ragged sets are lists of float32 CUDA [T, D] tensors with one D")
            self.flat = torch.cat([t.reshape(-1) for t in xs]).contiguous()
            self.lens = np.array([t.shape[0] for t in xs], dtype=np.int32)
            self.offs = np.zeros(len(xs), dtype=np.int64)
            if len(xs) > 1:
                self.offs[1:] = np.cumsum(self.lens[:-1].astype(np.int64) * D)
            self.shape = None
            self.batch = L.Batch(self.flat.data_ptr(),
                                 self.offs.ctypes.data_as(C.POINTER(C.c_int64)),
                                 self.lens.ctypes.data_as(C.POINTER(C.c_int32)),
                                 len(xs), D, 0)

    @property
    def count(self):
        return self.batch.count

    def split(self, flat):
        """Reshape a flat tensor laid out like this set back into its shape."""
        if self.shape is not None:
            return flat.view(self.shape)
        D = self.batch.dim
        return [flat[o:o + n * D].view(n, D) for o, n in zip(self.offs.tolist(), self.lens.tolist())]


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
