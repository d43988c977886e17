"""Isotropic Gaussian random fields with a red spectrum.

Recipe (one 2-D level): draw white noise, take its FFT, scale every coefficient by
|k|^(-p/2) with integer wavenumbers and the k = 0 coefficient zeroed, transform back and
divide by the sample standard deviation.  The power spectral density then falls as
|k|^(-p) (p = 3 by default) and each field has zero mean and exactly unit variance.
The paper's test state is a 2-level SQG temperature field (Sec. II-B, Sec. IV-A);
these fields stand in for it with the same shape and a turbulence-like spectrum.
"""
import os

import numpy as np
from scipy import fft as sfft

_WORKERS = 1  # callers parallelise over fields


def _wavenumber_magnitude(h, w):
    ky = np.fft.fftfreq(h) * h
    kx = np.fft.rfftfreq(w) * w
    return np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)


def smooth_fields(rng, count, h, w, slope=3.0):
    """`count` independent fields of shape (h, w), float64, zero mean, unit variance."""
    kmag = _wavenumber_magnitude(h, w)
    amp = np.zeros_like(kmag)
    nz = kmag > 0
    amp[nz] = kmag[nz] ** (-slope / 2.0)
    out = np.empty((count, h, w), dtype=np.float64)
    chunk = max(1, (1 << 24) // (h * w))
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        white = rng.standard_normal((e - s, h, w))
        spec = sfft.rfft2(white, workers=_WORKERS) * amp
        f = sfft.irfft2(spec, s=(h, w), workers=_WORKERS)
        f -= f.mean(axis=(1, 2), keepdims=True)
        f /= f.std(axis=(1, 2), keepdims=True)
        out[s:e] = f
    return out


def smooth_field(rng, levels, h, w, slope=3.0):
    """One state vector: `levels` independent fields, flattened level-major
    (element e = level*h*w + iy*w + ix)."""
    return smooth_fields(rng, levels, h, w, slope).reshape(-1)


def field_psd_slope(field2d):
    """Least-squares slope of log(PSD) against log|k| over 2 <= |k| <= min(h, w)/4."""
    h, w = field2d.shape
    psd = np.abs(np.fft.rfft2(field2d)) ** 2
    kmag = _wavenumber_magnitude(h, w)
    sel = (kmag >= 2) & (kmag <= min(h, w) / 4)
    return np.polyfit(np.log(kmag[sel]), np.log(psd[sel]), 1)[0]
