"""HEALPix RING geometry (Gorski et al. 2005, ApJ 622, 759), the pixelisation
the paper's maps use (acknowledgements; Sect. 3).

Rings are numbered i = 1 .. 4 Nside - 1 from the north pole.

* North polar cap, i < Nside: z = 1 - i^2 / (3 Nside^2), 4 i pixels,
  phi_j = pi / (2 i) (j - 1/2), j = 1 .. 4 i; the ring starts at pixel 2 i (i - 1).
* Equatorial belt, Nside <= i <= 3 Nside: z = 4/3 - 2 i / (3 Nside),
  4 Nside pixels, phi_j = pi / (2 Nside) (j - f), with f = 1 when i + Nside is
  odd and f = 1/2 when it is even (HEALPix numbering: the first pixel of an
  unshifted ring sits at phi = 0); the ring starts at pixel
  2 Nside (Nside - 1) + 4 Nside (i - Nside).
* South polar cap: ring i mirrors ring 4 Nside - i (z -> -z, same phi).

Parity unpinned? No: pinned by tests/test_oracle_geometry.py (pixel count,
z antisymmetry, equal-area ring boundaries, the 12 base pixels of Nside 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Rings:
    nside: int
    z: np.ndarray        # cos(theta) of each ring, float64
    sin_theta: np.ndarray
    nphi: np.ndarray     # pixels per ring, int64
    phi0: np.ndarray     # azimuth of the first pixel, float64
    first: np.ndarray    # index of the first pixel, int64

    @property
    def nrings(self) -> int:
        return self.z.size

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside


def rings(nside: int) -> Rings:
    if nside < 1:
        raise ValueError("nside must be >= 1")
    ns = nside
    npix = 12 * ns * ns
    nr = 4 * ns - 1
    z = np.empty(nr)
    st = np.empty(nr)
    nphi = np.empty(nr, dtype=np.int64)
    phi0 = np.empty(nr)
    first = np.empty(nr, dtype=np.int64)
    for k in range(nr):
        i = k + 1
        inorth = i if i <= 2 * ns else 4 * ns - i      # mirror ring in the north
        if inorth < ns:
            one_minus_z = inorth * inorth / (3.0 * ns * ns)
            zn = 1.0 - one_minus_z
            s = math.sqrt(one_minus_z * (2.0 - one_minus_z))
            n = 4 * inorth
            p0 = math.pi / (4.0 * inorth)
            fn = 2 * inorth * (inorth - 1)
        else:
            zn = 4.0 / 3.0 - 2.0 * inorth / (3.0 * ns)
            s = math.sqrt((1.0 - zn) * (1.0 + zn))
            n = 4 * ns
            p0 = 0.0 if ((inorth + ns) % 2 == 1) else math.pi / (4.0 * ns)
            fn = 2 * ns * (ns - 1) + 4 * ns * (inorth - ns)
        if i <= 2 * ns:
            z[k], first[k] = zn, fn
        else:
            z[k] = -zn
            first[k] = npix - fn - n
        st[k], nphi[k], phi0[k] = s, n, p0
    return Rings(ns, z, st, nphi, phi0, first)


def pixel_coords(nside: int):
    """(z, phi) of every pixel centre, RING order."""
    r = rings(nside)
    z = np.empty(r.npix)
    phi = np.empty(r.npix)
    for k in range(r.nrings):
        n, f = int(r.nphi[k]), int(r.first[k])
        z[f:f + n] = r.z[k]
        phi[f:f + n] = r.phi0[k] + 2.0 * math.pi * np.arange(n) / n
    return z, phi
