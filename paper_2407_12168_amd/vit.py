"""Python binding of the ViT forecast surrogate (include/ensf_vit.h), argument marshalling
only; states are torch float32 GPU tensors of shape (batch, C, H, W)."""
import ctypes

import numpy as np

from .ensf import EnsfError, ENSF_EINVAL, _check, _lib, _ptr, _stream

EXPORTS = ("ensf_vit_create", "ensf_vit_num_params", "ensf_vit_set_params",
           "ensf_vit_get_params", "ensf_vit_forward", "ensf_vit_grad", "ensf_vit_train_step",
           "ensf_vit_destroy")


class ensf_vit_config(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32), ("patch", ctypes.c_int32),
                ("layers", ctypes.c_int32), ("heads", ctypes.c_int32),
                ("embed", ctypes.c_int32), ("mlp_hidden", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("device", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


_READY = False


def _L():
    global _READY
    L = _lib()
    if not _READY:
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        L.ensf_vit_create.argtypes = [ctypes.POINTER(ensf_vit_config), ctypes.POINTER(vp)]
        L.ensf_vit_num_params.argtypes = [vp]
        L.ensf_vit_num_params.restype = i64
        L.ensf_vit_set_params.argtypes = [vp, vp]
        L.ensf_vit_get_params.argtypes = [vp, vp]
        L.ensf_vit_forward.argtypes = [vp, vp, vp, i32, vp]
        L.ensf_vit_grad.argtypes = [vp, vp, vp, i32, vp, dp, vp]
        L.ensf_vit_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, dp, vp]
        L.ensf_vit_destroy.argtypes = [vp]
        for n in EXPORTS:
            if n != "ensf_vit_num_params":
                getattr(L, n).restype = ctypes.c_int
        _READY = True
    return L


def ensf_vit_create(channels, height, width, patch, layers, heads, embed, mlp_hidden, max_batch,
                    seed=0, device=0):
    c = ensf_vit_config(channels, height, width, patch, layers, heads, embed, mlp_hidden,
                        max_batch, device, seed)
    h = ctypes.c_void_p()
    _check(_L().ensf_vit_create(ctypes.byref(c), ctypes.byref(h)), "ensf_vit_create")
    return h


def ensf_vit_num_params(v):
    return int(_L().ensf_vit_num_params(v))


def ensf_vit_set_params(v, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.size != ensf_vit_num_params(v):
        raise EnsfError(ENSF_EINVAL, "parameter count")
    _check(_L().ensf_vit_set_params(v, a.ctypes.data), "ensf_vit_set_params")


def ensf_vit_get_params(v):
    a = np.empty(ensf_vit_num_params(v), dtype=np.float32)
    _check(_L().ensf_vit_get_params(v, a.ctypes.data), "ensf_vit_get_params")
    return a


def ensf_vit_forward(v, x, y, stream=None):
    import torch
    _check(_L().ensf_vit_forward(v, _ptr(x, torch.float32, "x"), _ptr(y, torch.float32, "y"),
                                 x.shape[0], _stream(stream)), "ensf_vit_forward")


def ensf_vit_grad(v, x, target, grad, stream=None):
    """Writes the flat parameter gradient into `grad` (GPU float32) and returns the loss."""
    import torch
    loss = ctypes.c_double(0.0)
    _check(_L().ensf_vit_grad(v, _ptr(x, torch.float32, "x"), _ptr(target, torch.float32, "target"),
                              x.shape[0], _ptr(grad, torch.float32, "grad"), ctypes.byref(loss),
                              _stream(stream)), "ensf_vit_grad")
    return loss.value


def ensf_vit_train_step(v, x, target, lr, stream=None, want_loss=True):
    import torch
    loss = ctypes.c_double(0.0)
    _check(_L().ensf_vit_train_step(v, _ptr(x, torch.float32, "x"),
                                    _ptr(target, torch.float32, "target"), x.shape[0],
                                    float(lr), ctypes.byref(loss) if want_loss else None,
                                    _stream(stream)), "ensf_vit_train_step")
    return loss.value if want_loss else None


def ensf_vit_destroy(v):
    if v is not None and v.value:
        _check(_L().ensf_vit_destroy(v), "ensf_vit_destroy")


class ViT:
    """Owns one ensf_vit; destroy() is idempotent."""

    def __init__(self, **cfg):
        self.handle = ensf_vit_create(**cfg)

    def destroy(self):
        h, self.handle = self.handle, None
        if h is not None:
            ensf_vit_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
