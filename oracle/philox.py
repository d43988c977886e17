"""Philox4x32-10 and Box-Muller normals, FP64 (oracle; test infrastructure only).

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11): a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1).  One round maps
    (c0, c1, c2, c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57; between rounds the key is bumped by the Weyl
constants (0x9E3779B9, 0xBB67AE85).  Ten rounds, the first with the unbumped key.

Counter convention of the filter's noise (the paper leaves the generator open):
    key     = (seed mod 2^32, seed >> 32)
    counter = (element_index // 4, particle, step, filter_id)
with step = 0xFFFFFFFF for the initial N(0, I) draw.  The four words of one call give
the normals of elements 4q .. 4q+3:
    u(r)       = ((r >> 8) + 1/2) * 2^-24                  (in (0, 1), exact in FP32)
    n[4q]      = sqrt(-2 ln u(r0)) * cos(2 pi u(r1))
    n[4q + 1]  = sqrt(-2 ln u(r0)) * sin(2 pi u(r1))
    n[4q + 2]  = sqrt(-2 ln u(r2)) * cos(2 pi u(r3))
    n[4q + 3]  = sqrt(-2 ln u(r2)) * sin(2 pi u(r3))
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
SH = np.uint64(32)
INIT_STEP = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Inputs are integer arrays (broadcastable) of 32-bit
    values; returns four uint64 arrays holding 32-bit words."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for rnd in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> SH) ^ c1 ^ k0, p1 & MASK, (p0 >> SH) ^ c3 ^ k1, p0 & MASK)
        if rnd < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def uniform24(r):
    """Map a 32-bit word to (0, 1) using its top 24 bits."""
    return ((np.asarray(r, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24


def box_muller(ra, rb):
    """Pair of standard normals from two words (Box & Muller, 1958)."""
    rad = np.sqrt(-2.0 * np.log(uniform24(ra)))
    ang = 2.0 * np.pi * uniform24(rb)
    return rad * np.cos(ang), rad * np.sin(ang)


def raw_words(seed, filter_id, step, particles, n_elements):
    """Raw words for each particle in `particles` over ceil(n/4) counters:
    array (P, ceil(n/4), 4) of uint64."""
    particles = np.asarray(particles, dtype=np.uint64)
    nq = (n_elements + 3) // 4
    q = np.arange(nq, dtype=np.uint64)
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    r = philox4x32_10(q[None, :], particles[:, None], np.uint64(step), np.uint64(filter_id),
                      k0, k1)
    return np.stack(r, axis=-1)


def normals(seed, filter_id, step, particles, n_elements):
    """Standard normals (P, n) for the given particles at one pseudo-time step."""
    w = raw_words(seed, filter_id, step, particles, n_elements)
    a, b = box_muller(w[..., 0], w[..., 1])
    c, d = box_muller(w[..., 2], w[..., 3])
    out = np.stack([a, b, c, d], axis=-1).reshape(w.shape[0], -1)
    return out[:, :n_elements]
