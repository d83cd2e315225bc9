"""Pins of the oracle's HEALPix RING geometry (Gorski et al. 2005)."""
import math
import os

import numpy as np
import pytest

from oracle import healpix

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("nside", [1, 2, 3, 4, 8, 16, 64, 256])
def test_pixel_count_and_contiguity(nside):
    r = healpix.rings(nside)
    assert r.nrings == 4 * nside - 1
    assert int(r.nphi.sum()) == 12 * nside * nside
    # rings tile the pixel range contiguously, in order
    assert r.first[0] == 0
    assert np.all(r.first[1:] == r.first[:-1] + r.nphi[:-1])
    # z strictly decreasing and antisymmetric about the equator
    assert np.all(np.diff(r.z) < 0)
    assert np.max(np.abs(r.z + r.z[::-1])) < 1e-15
    assert abs(r.z.sum()) < 1e-12
    assert np.allclose(r.sin_theta ** 2 + r.z ** 2, 1.0, rtol=0, atol=1e-15)


def test_nside1_base_pixels_golden():
    tab = np.loadtxt(os.path.join(GOLD, "healpix_nside1.txt"))
    z, phi = healpix.pixel_coords(1)
    assert np.allclose(z, tab[:, 1], atol=1e-15)
    assert np.allclose(phi / math.pi, tab[:, 2], atol=1e-15)


@pytest.mark.parametrize("nside", [2, 4, 16])
def test_equal_area_ring_boundaries(nside):
    # Equal-area property: the pixels north of the boundary between ring i and
    # ring i+1 cover a fraction N_i/Npix of the sphere, i.e. the boundary sits
    # at z_b = 1 - 2 N_i / Npix. Boundaries lie strictly between ring centres.
    r = healpix.rings(nside)
    cum = np.cumsum(r.nphi)[:-1]
    zb = 1.0 - 2.0 * cum / r.npix
    assert np.all(zb < r.z[:-1]) and np.all(zb > r.z[1:])
    # in the belt, centres are midway between boundaries (uniform z spacing)
    belt = slice(nside, 3 * nside - 1)
    assert np.allclose(np.diff(r.z[belt]), -2.0 / (3.0 * nside), atol=1e-15)


@pytest.mark.parametrize("nside,expected", [(16, 22), (256, 494), (512, 1004), (1024, 2026)])
def test_non_power_of_two_ring_counts(nside, expected):
    r = healpix.rings(nside)
    n = r.nphi
    assert int(np.sum((n & (n - 1)) != 0)) == expected


def test_phi_within_ring_uniform():
    z, phi = healpix.pixel_coords(8)
    r = healpix.rings(8)
    for k in range(r.nrings):
        f, n = int(r.first[k]), int(r.nphi[k])
        d = np.diff(phi[f:f + n])
        assert np.allclose(d, 2 * math.pi / n)
        assert 0.0 <= phi[f] < 2 * math.pi / n
