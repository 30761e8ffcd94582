"""Seeded input generators: the published SplitMix64 outputs, determinism,
ranges and the disc coverage rule."""
import numpy as np

from conftest import read_golden
from paper_0906_3611_amd import inputs


def test_splitmix64_published_outputs():
    for row in read_golden("splitmix64_seed0.txt"):
        k, hexv = row.split()
        assert int(inputs.splitmix64(0, [int(k)])[0]) == int(hexv, 16)


def test_noise_fields_range_and_determinism():
    a, b = inputs.noise_fields(67, 61, 1, 0.5, 0.5, 0.01)
    a2, b2 = inputs.noise_fields(67, 61, 1, 0.5, 0.5, 0.01)
    assert np.array_equal(a, a2) and np.array_equal(b, b2)
    assert a.shape == (61, 67)
    assert 0.49 <= a.min() and a.max() < 0.51
    assert not np.array_equal(a, b)
    assert abs(a.mean() - 0.5) < 1e-3
    c, _ = inputs.noise_fields(67, 61, 2, 0.5, 0.5, 0.01)
    assert not np.array_equal(a, c)


def test_disc_fields_cover_requested_fraction():
    a, b = inputs.disc_fields(128, 96, 2, 0.7)
    inside = a == 1.2
    assert 0.7 <= inside.mean() < 0.72
    assert np.all(b[inside] == 0.05) and np.all(a[~inside] == 0.05) and np.all(b[~inside] == 1.2)


def test_noise_window_is_a_periodic_slice_of_the_lattice():
    nx, ny, seed = 37, 23, 11
    ra, rb = inputs.noise_fields(nx, ny, seed, 0.5, 0.4, 0.02)
    for x0, y0, w, h in ((0, 0, 37, 23), (-6, -6, 13, 13), (30, 20, 13, 13), (5, 7, 3, 4)):
        wa, wb = inputs.noise_window(nx, ny, seed, 0.5, 0.4, 0.02, x0, y0, w, h)
        ys = (y0 + np.arange(h)) % ny
        xs = (x0 + np.arange(w)) % nx
        assert np.array_equal(wa, ra[np.ix_(ys, xs)])
        assert np.array_equal(wb, rb[np.ix_(ys, xs)])
