"""Thin Python binding of include/hmg_nn.h (argument marshalling only).

``Net`` wraps the network handle; ``conv3d_*`` expose the single layers used by
the parity tests.  Tensors are contiguous float32 CUDA tensors laid out
[batch][channel][z][y][x].
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .hmg import OK, HmgError


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()


def _f32(t, name):
    if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


def _check(st, what):
    if st != OK:
        raise HmgError(st, what)


class Net:
    """The warm-start encoder-decoder (hmg_nn_create ... hmg_nn_destroy)."""

    def __init__(self, levels=4, base_channels=8, in_channels=1, out_channels=18, seed=0,
                 stream: torch.cuda.Stream | None = None):
        self.lib = _lib.load()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.config = _lib.HmgNnConfig(levels, base_channels, in_channels, out_channels)
        h = ctypes.c_void_p()
        _check(self.lib.hmg_nn_create(ctypes.byref(self.config),
                                      ctypes.c_void_p(self.stream.cuda_stream), seed,
                                      ctypes.byref(h)), "hmg_nn_create")
        self._h = h
        n = ctypes.c_int64()
        _check(self.lib.hmg_nn_param_count(self._h, ctypes.byref(n)), "hmg_nn_param_count")
        self.param_count = n.value

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.hmg_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def get_params(self) -> np.ndarray:
        out = np.empty(self.param_count, np.float32)
        _check(self.lib.hmg_nn_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                          self.param_count), "hmg_nn_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.param_count:
            raise ValueError("parameter count mismatch")
        _check(self.lib.hmg_nn_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p),
                                          self.param_count), "hmg_nn_set_params")

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.param_count, np.float32)
        _check(self.lib.hmg_nn_get_grads(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                         self.param_count), "hmg_nn_get_grads")
        return out

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _f32(x, "x")
        B, C, D = x.shape[0], x.shape[1], x.shape[2]
        if C != self.config.in_channels or x.shape[2:] != (D, D, D):
            raise ValueError("x must be [batch][in_channels][D][D][D]")
        if out is None:
            out = torch.empty((B, self.config.out_channels, D, D, D), dtype=torch.float32,
                              device=x.device)
        _check(self.lib.hmg_nn_forward(self._h, _ptr(x), B, D, _ptr(_f32(out, "out"))),
               "hmg_nn_forward")
        return out

    def backward(self, dy: torch.Tensor):
        _check(self.lib.hmg_nn_backward(self._h, _ptr(_f32(dy, "dy"))), "hmg_nn_backward")

    def zero_grad(self):
        _check(self.lib.hmg_nn_zero_grad(self._h), "hmg_nn_zero_grad")

    def adam_step(self, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(self.lib.hmg_nn_adam_step(self._h, lr, beta1, beta2, eps, step), "hmg_nn_adam_step")

    def mse(self, y: torch.Tensor, t: torch.Tensor, dy: torch.Tensor) -> float:
        loss = ctypes.c_double()
        _check(self.lib.hmg_nn_mse(self._h, _ptr(_f32(y, "y")), _ptr(_f32(t, "t")), y.numel(),
                                   _ptr(_f32(dy, "dy")), ctypes.byref(loss)), "hmg_nn_mse")
        return loss.value

    def save(self, path):
        np.save(path, self.get_params(), allow_pickle=False)

    def load(self, path):
        self.set_params(np.load(path, allow_pickle=False))


def warm_start(ctx, net: Net, accept_relres=0.5):
    """hmg_warm_start: returns (worst relative residual of the guess, used)."""
    rr, used = ctypes.c_double(), ctypes.c_int32()
    st = ctx.lib.hmg_warm_start(ctx._h, net.handle, accept_relres, ctypes.byref(rr),
                                ctypes.byref(used))
    ctx._check(st)
    return rr.value, bool(used.value)


def _dims(x):
    B, C, D, H, W = x.shape
    return B, C, D, H, W


def conv3d_forward(x, w, bias, relu=False, stream=None):
    lib = _lib.load()
    B, Cin, D, H, W = _dims(_f32(x, "x"))
    Cout = w.shape[0]
    y = torch.empty((B, Cout, D, H, W), dtype=torch.float32, device=x.device)
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib.hmg_conv3d_forward(ctypes.c_void_p(s), _ptr(x), _ptr(_f32(w, "w")),
                                  _ptr(bias), _ptr(y), B, Cin, Cout, D, H, W, int(relu)),
           "hmg_conv3d_forward")
    return y


def conv3d_backward_data(dz, w, dx, stream=None):
    lib = _lib.load()
    B, Cout, D, H, W = _dims(_f32(dz, "dz"))
    Cin = w.shape[1]
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib.hmg_conv3d_backward_data(ctypes.c_void_p(s), _ptr(dz), _ptr(_f32(w, "w")),
                                        _ptr(_f32(dx, "dx")), B, Cin, Cout, D, H, W),
           "hmg_conv3d_backward_data")
    return dx


def conv3d_backward_weight(x, dz, dw, dbias, stream=None):
    lib = _lib.load()
    B, Cin, D, H, W = _dims(_f32(x, "x"))
    Cout = dz.shape[1]
    work = torch.empty(lib.hmg_conv3d_workspace(B, Cin, Cout, D, H, W), dtype=torch.float32,
                       device=x.device)
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib.hmg_conv3d_backward_weight(ctypes.c_void_p(s), _ptr(x), _ptr(_f32(dz, "dz")),
                                          _ptr(_f32(dw, "dw")), _ptr(dbias), _ptr(work),
                                          B, Cin, Cout, D, H, W), "hmg_conv3d_backward_weight")
    return dw, dbias


def conv3d_backward_weight_noalloc(x, dz, dw, dbias, stream=None):
    """hmg_conv3d_backward_weight_noalloc: the same gradient with the library's
    fixed device scratch instead of a workspace (nothing is allocated)."""
    lib = _lib.load()
    B, Cin, D, H, W = _dims(_f32(x, "x"))
    Cout = dz.shape[1]
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(lib.hmg_conv3d_backward_weight_noalloc(ctypes.c_void_p(s), _ptr(x), _ptr(_f32(dz, "dz")),
                                                  _ptr(_f32(dw, "dw")), _ptr(dbias),
                                                  B, Cin, Cout, D, H, W),
           "hmg_conv3d_backward_weight_noalloc")
    return dw, dbias
