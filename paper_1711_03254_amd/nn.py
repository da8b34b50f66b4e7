"""Python binding of the surrogate kernels, the C ABI of include/lbm_nn.h
(exported by liblbm.so).  Argument marshalling only.

Tensors are torch tensors on the GPU used as device memory.  A `View` is a
tensor with a channel offset and a channel stride (ld): element (p, c) is
t.flatten()[p * ld + off + c], the layout of include/lbm_nn.h; bf16 data
lives in int16 tensors (bit patterns).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import lbm

NN_EXPORTED = ("nn_conv3d_fwd", "nn_weights_flip", "nn_bwd_weight_work", "nn_conv3d_bwd_weight",
               "nn_relu_bwd_cast", "nn_pool2_fwd", "nn_pool2_bwd", "nn_up2_fwd", "nn_up2_bwd", "nn_mse",
               "nn_adam", "nn_to_bf16", "nn_solid_distance", "nn_features", "nn_decode_fields")

_lib = None
_P, _I, _L, _F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float


def load():
    global _lib
    if _lib is not None:
        return _lib
    lib = lbm.load_library()
    sig = {
        "nn_conv3d_fwd": [_P, _I, _P, _P, _P, _I, _I, _I, _I, _I, _I, _I, _I, _I, _P],
        "nn_weights_flip": [_P, _P, _I, _I, _P],
        "nn_bwd_weight_work": [_I, _I, _I, _I, _I, _I],
        "nn_conv3d_bwd_weight": [_P, _I, _P, _I, _P, _P, _P, _L, _I, _I, _I, _I, _I, _I, _P],
        "nn_relu_bwd_cast": [_P, _I, _P, _I, _P, _I, _L, _I, _I, _P],
        "nn_pool2_fwd": [_P, _I, _P, _I, _I, _I, _I, _I, _I, _P],
        "nn_pool2_bwd": [_P, _I, _P, _I, _I, _I, _I, _I, _I, _I, _P],
        "nn_up2_fwd": [_P, _I, _P, _I, _I, _I, _I, _I, _I, _P],
        "nn_up2_bwd": [_P, _I, _P, _I, _I, _I, _I, _I, _I, _P],
        "nn_mse": [_P, _I, _P, _I, _P, _P, _I, _P, _L, _I, _P],
        "nn_adam": [_P, _P, _P, _P, _P, _L, _F, _F, _F, _F, _I, _P],
        "nn_to_bf16": [_P, _P, _L, _P],
        "nn_solid_distance": [_P, _P, _P, _I, _I, _I, _I, _P],
        "nn_features": [_P, _P, _P, _P, _F, _P, _I, _I, _L, _P],
        "nn_decode_fields": [_P, _I, _P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _F, _F,
                             ctypes.c_double, _P, _P, _P, _P, _L, _P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int64 if name == "nn_bwd_weight_work" else ctypes.c_int
    _lib = lib
    return lib


class NNError(RuntimeError):
    pass


def _ok(name, rc):
    if rc != 0:
        raise NNError(f"{name} failed with code {rc}")


@dataclass
class View:
    t: torch.Tensor
    ld: int
    off: int = 0

    @property
    def ptr(self):
        return self.t.data_ptr() + self.off * self.t.element_size()

    def sub(self, off):
        return View(self.t, self.ld, self.off + off)


def _s(stream):
    return (stream if stream is not None else torch.cuda.current_stream()).cuda_stream


def conv3d_fwd(x: View, w, bias, y: View, relu, dims, ci, co, stream=None):
    nb, d, h, wd = dims
    y_fp32 = 1 if y.t.dtype == torch.float32 else 0
    _ok("nn_conv3d_fwd", load().nn_conv3d_fwd(x.ptr, x.ld, w.data_ptr(), bias.data_ptr() if bias is not None else None,
                                              y.ptr, y.ld, y_fp32, int(relu), nb, d, h, wd, ci, co, _s(stream)))


def weights_flip(w, wt, ci, co, stream=None):
    _ok("nn_weights_flip", load().nn_weights_flip(w.data_ptr(), wt.data_ptr(), ci, co, _s(stream)))


def bwd_weight_work(dims, ci, co):
    return int(load().nn_bwd_weight_work(*dims, ci, co))


def conv3d_bwd_weight(x: View, dy: View, dw, db, work, dims, ci, co, stream=None):
    _ok("nn_conv3d_bwd_weight", load().nn_conv3d_bwd_weight(x.ptr, x.ld, dy.ptr, dy.ld, dw.data_ptr(), db.data_ptr(),
                                                            work.data_ptr(), work.numel(), *dims, ci, co, _s(stream)))


def relu_bwd_cast(dy: View, y: View, out: View, p, c, relu, stream=None):
    _ok("nn_relu_bwd_cast", load().nn_relu_bwd_cast(dy.ptr, dy.ld, y.ptr if y is not None else None,
                                                    y.ld if y is not None else 0, out.ptr, out.ld, p, c, int(relu),
                                                    _s(stream)))


def pool2_fwd(x: View, y: View, dims, c, stream=None):
    _ok("nn_pool2_fwd", load().nn_pool2_fwd(x.ptr, x.ld, y.ptr, y.ld, *dims, c, _s(stream)))


def pool2_bwd(dy: View, dx: View, accumulate, dims, c, stream=None):
    _ok("nn_pool2_bwd", load().nn_pool2_bwd(dy.ptr, dy.ld, dx.ptr, dx.ld, int(accumulate), *dims, c, _s(stream)))


def up2_fwd(x: View, y: View, dims, c, stream=None):
    _ok("nn_up2_fwd", load().nn_up2_fwd(x.ptr, x.ld, y.ptr, y.ld, *dims, c, _s(stream)))


def up2_bwd(dy: View, dx: View, dims, c, stream=None):
    _ok("nn_up2_bwd", load().nn_up2_bwd(dy.ptr, dy.ld, dx.ptr, dx.ld, *dims, c, _s(stream)))


def mse(pred: View, target: View, cw, dpred: View, loss, p, c, stream=None):
    _ok("nn_mse", load().nn_mse(pred.ptr, pred.ld, target.ptr, target.ld, cw.data_ptr(), dpred.ptr, dpred.ld,
                                loss.data_ptr(), p, c, _s(stream)))


def adam(param, grad, m, v, param_bf16, lr, t, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    _ok("nn_adam", load().nn_adam(param.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                                  param_bf16.data_ptr() if param_bf16 is not None else None, param.numel(), lr, b1, b2,
                                  eps, t, _s(stream)))


def to_bf16(x, y, stream=None):
    _ok("nn_to_bf16", load().nn_to_bf16(x.data_ptr(), y.data_ptr(), x.numel(), _s(stream)))


def solid_distance(solid, work, dist, dims, radius, stream=None):
    """solid: uint8 tensor; work: float32 tensor of 2 P; dist: float32 [P]."""
    d, h, w = dims
    _ok("nn_solid_distance", load().nn_solid_distance(solid.data_ptr(), work.data_ptr(), dist.data_ptr(), d, h, w,
                                                      radius, _s(stream)))


def features(solid, rho_a, rho_b, dist, dist_scale, x: View, c, stream=None):
    _ok("nn_features", load().nn_features(solid.data_ptr(), rho_a.data_ptr(), rho_b.data_ptr(), dist.data_ptr(),
                                          dist_scale, x.ptr, x.ld, c, solid.numel(), _s(stream)))


def decode_fields(out: View, solid, rho_a0, rho_b0, nu_a, nu_b, g, u_scale, rho_scale, floor, u, rho_a, rho_b, work,
                  stream=None):
    _ok("nn_decode_fields", load().nn_decode_fields(out.ptr, out.ld, solid.data_ptr(), rho_a0.data_ptr(),
                                                    rho_b0.data_ptr(), nu_a, nu_b, g, u_scale, rho_scale, floor,
                                                    u.data_ptr(), rho_a.data_ptr(), rho_b.data_ptr(), work.data_ptr(),
                                                    solid.numel(), _s(stream)))
