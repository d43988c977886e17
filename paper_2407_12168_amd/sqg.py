"""Python binding of the GPU SQG model (include/ensf_sqg.h), argument marshalling only;
states are torch GPU tensors (batch, 2, n, n), float64 or float32."""
import ctypes
import math

from .ensf import _check, _lib, _ptr, _stream

EXPORTS = ("ensf_sqg_create", "ensf_sqg_run", "ensf_sqg_run_f32", "ensf_sqg_destroy")
_READY = False


def _L():
    global _READY
    L = _lib()
    if not _READY:
        vp, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.ensf_sqg_create.argtypes = [i32, d, d, d, i32, d, d, i32, i32, ctypes.POINTER(vp)]
        L.ensf_sqg_run.argtypes = [vp, vp, vp, i32, i32, vp]
        L.ensf_sqg_run_f32.argtypes = [vp, vp, vp, i32, i32, vp]
        L.ensf_sqg_destroy.argtypes = [vp]
        for n in EXPORTS:
            getattr(L, n).restype = ctypes.c_int
        _READY = True
    return L


def ensf_sqg_create(n=128, lx=20.0, shear=1.0, dt=0.025, diff_order=8, diff_efold=None,
                    relax_time=math.inf, max_batch=256, device=0):
    efold = 10.0 * dt if diff_efold is None else diff_efold
    h = ctypes.c_void_p()
    _check(_L().ensf_sqg_create(n, lx, shear, dt, diff_order, float(efold), float(relax_time),
                                max_batch, device, ctypes.byref(h)), "ensf_sqg_create")
    return h


def ensf_sqg_run(s, x, y, n_steps, stream=None):
    import torch
    if x.dtype == torch.float64:
        _check(_L().ensf_sqg_run(s, _ptr(x, torch.float64, "x"), _ptr(y, torch.float64, "y"),
                                 x.shape[0], int(n_steps), _stream(stream)), "ensf_sqg_run")
    else:
        _check(_L().ensf_sqg_run_f32(s, _ptr(x, torch.float32, "x"), _ptr(y, torch.float32, "y"),
                                     x.shape[0], int(n_steps), _stream(stream)),
               "ensf_sqg_run_f32")


def ensf_sqg_destroy(s):
    if s is not None and s.value:
        _check(_L().ensf_sqg_destroy(s), "ensf_sqg_destroy")


class SQGModel:
    """Owns one ensf_sqg; destroy() is idempotent."""

    def __init__(self, **kw):
        self.handle = ensf_sqg_create(**kw)

    def run(self, x, y, n_steps, stream=None):
        ensf_sqg_run(self.handle, x, y, n_steps, stream)

    def destroy(self):
        h, self.handle = self.handle, None
        if h is not None:
            ensf_sqg_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
