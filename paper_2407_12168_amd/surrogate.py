"""Python binding of the conv forecast surrogate (include/ensf_surrogate.h), argument
marshalling only; states are torch float32 GPU tensors of shape (batch, C0, H, W)."""
import ctypes

import numpy as np

from .ensf import EnsfError, ENSF_EINVAL, _check, _lib, _ptr, _stream

EXPORTS = ("ensf_surrogate_create", "ensf_surrogate_num_params", "ensf_surrogate_set_params",
           "ensf_surrogate_get_params", "ensf_surrogate_forward", "ensf_surrogate_grad",
           "ensf_surrogate_train_step", "ensf_surrogate_destroy")

_READY = False


def _L():
    global _READY
    L = _lib()
    if not _READY:
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.ensf_surrogate_create.argtypes = [i32, i32, i32, i32, i32, i32, u64, i32,
                                            ctypes.POINTER(vp)]
        L.ensf_surrogate_num_params.argtypes = [vp]
        L.ensf_surrogate_num_params.restype = i64
        L.ensf_surrogate_set_params.argtypes = [vp, vp]
        L.ensf_surrogate_get_params.argtypes = [vp, vp]
        L.ensf_surrogate_forward.argtypes = [vp, vp, vp, i32, vp]
        L.ensf_surrogate_grad.argtypes = [vp, vp, vp, i32, vp, ctypes.POINTER(ctypes.c_double), vp]
        L.ensf_surrogate_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float,
                                                ctypes.POINTER(ctypes.c_double), vp]
        L.ensf_surrogate_destroy.argtypes = [vp]
        for n in EXPORTS:
            if n != "ensf_surrogate_num_params":
                getattr(L, n).restype = ctypes.c_int
        _READY = True
    return L


def ensf_surrogate_create(c0, width, layers, h, w, max_batch, seed=0, device=0):
    hnd = ctypes.c_void_p()
    _check(_L().ensf_surrogate_create(c0, width, layers, h, w, max_batch, seed, device,
                                      ctypes.byref(hnd)), "ensf_surrogate_create")
    return hnd


def ensf_surrogate_num_params(s):
    return int(_L().ensf_surrogate_num_params(s))


def ensf_surrogate_set_params(s, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.size != ensf_surrogate_num_params(s):
        raise EnsfError(ENSF_EINVAL, "parameter count")
    _check(_L().ensf_surrogate_set_params(s, a.ctypes.data), "ensf_surrogate_set_params")


def ensf_surrogate_get_params(s):
    a = np.empty(ensf_surrogate_num_params(s), dtype=np.float32)
    _check(_L().ensf_surrogate_get_params(s, a.ctypes.data), "ensf_surrogate_get_params")
    return a


def ensf_surrogate_forward(s, x, y, stream=None):
    import torch
    _check(_L().ensf_surrogate_forward(s, _ptr(x, torch.float32, "x"), _ptr(y, torch.float32, "y"),
                                       x.shape[0], _stream(stream)), "ensf_surrogate_forward")


def ensf_surrogate_grad(s, x, target, grad, stream=None):
    import torch
    loss = ctypes.c_double(0.0)
    _check(_L().ensf_surrogate_grad(s, _ptr(x, torch.float32, "x"),
                                    _ptr(target, torch.float32, "target"), x.shape[0],
                                    _ptr(grad, torch.float32, "grad"), ctypes.byref(loss),
                                    _stream(stream)), "ensf_surrogate_grad")
    return loss.value


def ensf_surrogate_train_step(s, x, target, lr, want_loss=True, stream=None):
    import torch
    loss = ctypes.c_double(0.0)
    _check(_L().ensf_surrogate_train_step(s, _ptr(x, torch.float32, "x"),
                                          _ptr(target, torch.float32, "target"), x.shape[0],
                                          float(lr), ctypes.byref(loss) if want_loss else None,
                                          _stream(stream)), "ensf_surrogate_train_step")
    return loss.value if want_loss else None


def ensf_surrogate_destroy(s):
    if s is not None and s.value:
        _check(_L().ensf_surrogate_destroy(s), "ensf_surrogate_destroy")


class Surrogate:
    """Owns one ensf_surrogate; destroy() is idempotent."""

    def __init__(self, c0=2, width=64, layers=6, h=128, w=128, max_batch=64, seed=0, device=0):
        self.handle = ensf_surrogate_create(c0, width, layers, h, w, max_batch, seed, device)
        self.shape = (c0, h, w)

    def destroy(self):
        h, self.handle = self.handle, None
        if h is not None:
            ensf_surrogate_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
