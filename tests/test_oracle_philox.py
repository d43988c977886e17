"""Pins of the oracle's counter-based generator: published known answers and the
distribution of the normals it yields."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(x, 16) for x in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_known_answers(row):
    c0, c1, c2, c3, k0, k1, *want = row
    got = philox.philox4x32_10(c0, c1, c2, c3, k0, k1)
    assert [int(x) for x in got] == want


def test_vectorised_matches_scalar_calls():
    q = np.arange(7)
    r = philox.philox4x32_10(q, 3, 5, 9, 0x1234, 0x5678)
    for i in range(7):
        s = philox.philox4x32_10(i, 3, 5, 9, 0x1234, 0x5678)
        assert all(int(r[w][i]) == int(s[w]) for w in range(4))


def test_uniform_range_and_resolution():
    u = philox.uniform24(np.array([0, 0xFF, 0x100, 0xFFFFFFFF], dtype=np.uint64))
    assert u[0] == 0.5 * 2.0 ** -24 and u[1] == u[0]
    assert u[2] == 1.5 * 2.0 ** -24
    assert u[3] == 1.0 - 0.5 * 2.0 ** -24
    assert np.all((u > 0) & (u < 1))


def test_box_muller_geometry():
    # radius^2 of each normal pair is -2 ln u(ra); angle is 2 pi u(rb)
    ra = np.array([0x80000000, 0x12345678], dtype=np.uint64)
    rb = np.array([0x40000000, 0xdeadbeef], dtype=np.uint64)
    a, b = philox.box_muller(ra, rb)
    np.testing.assert_allclose(a * a + b * b, -2 * np.log(philox.uniform24(ra)), rtol=1e-14)
    np.testing.assert_allclose(np.arctan2(b, a) % (2 * np.pi),
                               (2 * np.pi * philox.uniform24(rb)) % (2 * np.pi), rtol=1e-12)


def test_normals_distribution():
    z = philox.normals(seed=12168, filter_id=3, step=7, particles=np.arange(64), n_elements=16384)
    z = z.reshape(-1)
    assert abs(z.mean()) < 4.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4.0 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_counters_independent():
    a = philox.normals(1, 0, 0, [0, 1], 64)
    b = philox.normals(1, 0, 1, [0, 1], 64)
    c = philox.normals(1, 1, 0, [0, 1], 64)
    d = philox.normals(2, 0, 0, [0, 1], 64)
    for o in (b, c, d):
        assert not np.allclose(a, o)
    assert not np.allclose(a[0], a[1])
    np.testing.assert_array_equal(a, philox.normals(1, 0, 0, [0, 1], 64))
    # a prefix of the elements does not depend on the length requested
    np.testing.assert_array_equal(a[:, :10], philox.normals(1, 0, 0, [0, 1], 10))
