"""Spin-2 (polarisation) transforms of the oracle (test infrastructure).

The paper's temperature-and-polarisation data (T, E, B spectra and the 3x3
covariance of the joint move, Sect. 2.2.2) need the spin-weighted harmonics
+-2Y_lm; the paper does not define them, so the HEALPix / COSMO convention is
taken (Zaldarriaga & Seljak 1997; Gorski et al. 2005):

    Q +- iU = sum_lm  (+-2 a_lm) (+-2 Y_lm),   +-2 a_lm = -(a_E +- i a_B),
    +2Y_lm = d^2 Y_lm / sqrt((l-1) l (l+1) (l+2)),  -2Y_lm = dbar^2 Y_lm / sqrt(...)

with the spin-raising / lowering operators of Goldberg et al. (1967) acting on
a spin-s function f(theta) e^{i m phi}:

    d f    = -(d/dtheta - m / sin - s cot) f,    dbar f = -(d/dtheta + m / sin + s cot) f.

Writing +-2Y_lm = (W_lm +- X_lm) e^{i m phi}, the scalar Legendre equation
and s dlambda_l/dtheta = l c lambda_l - F_lm lambda_{l-1} (c = cos, s = sin,
F_lm = sqrt((2l+1)/(2l-1) (l^2 - m^2))) give, with N_l = sqrt((l-1)l(l+1)(l+2)),

    W_lm = ( -2 ((l - m^2)/s^2 + l(l-1)/2) lambda_l + 2 c F_lm / s^2 lambda_{l-1} ) / N_l
    X_lm = -2 m / s^2 ( (l-1) c lambda_l - F_lm lambda_{l-1} ) / N_l        (l >= 2; 0 below)

and the maps of a real (E, B) pair follow from the per-ring spectra

    G_Q(m) = -sum_l (a_E W + i a_B X),   G_U(m) = -sum_l (a_B W - i a_E X),

each synthesised like a spin-0 field (F(-m) = conj F(m)). The transpose
(real-field inner product on both sides) is a_E = sum_r (-W G^_Q - i X G^_U),
a_B = sum_r (i X G^_Q - W G^_U) with G^ the azimuthal adjoint of the maps.

Pins (tests/test_oracle_spin2.py): W +- X against d^2 Y and dbar^2 Y computed
by 50-digit numerical differentiation of the scalar harmonic; orthonormality
of +-2Y on an exact Gauss-Legendre grid; adjointness; pure-E / pure-B m = 0
fields giving U = 0 / Q = 0.
"""
from __future__ import annotations

import math

import numpy as np

from .legendre import lambda_rows
from .sht import SHT


def wx_rows(lmax: int, mmax: int, z: np.ndarray, sin_theta: np.ndarray):
    """Generator over l = 0..lmax yielding (l, W, X), arrays of shape
    (min(l, mmax)+1, nz) (zero for l < 2)."""
    z = np.asarray(z, dtype=np.float64)
    st = np.asarray(sin_theta, dtype=np.float64)
    s2 = st * st
    prev = None
    for l, lam in lambda_rows(lmax, mmax, z, st):
        top = lam.shape[0] - 1
        if l < 2:
            prev = lam
            yield l, np.zeros_like(lam), np.zeros_like(lam)
            continue
        m = np.arange(top + 1, dtype=np.float64)[:, None]
        lm1 = np.zeros_like(lam)
        lm1[:prev.shape[0]] = prev               # lambda_{l-1,m} (0 for m = l)
        F = np.sqrt((2.0 * l + 1.0) / (2.0 * l - 1.0) * (l * l - m * m))
        nl = math.sqrt((l - 1.0) * l * (l + 1.0) * (l + 2.0))
        W = (-2.0 * ((l - m * m) / s2 + 0.5 * l * (l - 1.0)) * lam + 2.0 * z * F / s2 * lm1) / nl
        X = -2.0 * m / s2 * ((l - 1.0) * z * lam - F * lm1) / nl
        prev = lam
        yield l, W, X


class PolSHT:
    """(a_E, a_B) -> (Q, U) and its transpose for one (nside, lmax)."""

    def __init__(self, nside: int, lmax: int, mmax: int | None = None):
        self.s = SHT(nside, lmax, mmax)
        self.nside, self.lmax, self.mmax = nside, lmax, self.s.mmax
        self.npix, self.nalm = self.s.npix, self.s.nalm

    def spectra(self, aE: np.ndarray, aB: np.ndarray, ring_idx=None):
        R = self.s.rings
        rows = np.arange(R.nrings) if ring_idx is None else np.asarray(list(ring_idx))
        GQ = np.zeros((self.mmax + 1, rows.size), dtype=np.complex128)
        GU = np.zeros_like(GQ)
        for l, W, X in wx_rows(self.lmax, self.mmax, R.z[rows], R.sin_theta[rows]):
            if l < 2:
                continue
            top = W.shape[0] - 1
            e = aE[self.s._idx(l, top)][:, None]
            b = aB[self.s._idx(l, top)][:, None]
            GQ[:top + 1] -= W * e + 1j * X * b
            GU[:top + 1] -= W * b - 1j * X * e
        return GQ, GU

    def synth(self, aE: np.ndarray, aB: np.ndarray):
        GQ, GU = self.spectra(np.asarray(aE, dtype=np.complex128), np.asarray(aB, dtype=np.complex128))
        return self.s.phi_synth(GQ), self.s.phi_synth(GU)

    def synth_rings(self, aE: np.ndarray, aB: np.ndarray, ring_idx) -> dict:
        """(Q, U) pixel values on selected rings only (ring index -> pair of
        arrays): the same spectra restricted to those rings, each synthesised
        like a spin-0 field."""
        R = self.s.rings
        ring_idx = list(ring_idx)
        GQ, GU = self.spectra(np.asarray(aE, dtype=np.complex128), np.asarray(aB, dtype=np.complex128), ring_idx)
        m = np.arange(self.mmax + 1)
        wm = np.where(m == 0, 1.0, 2.0)
        out = {}
        for j, k in enumerate(ring_idx):
            n = int(R.nphi[k])
            maps = []
            for G in (GQ, GU):
                c = np.zeros(n, dtype=np.complex128)
                np.add.at(c, m % n, wm * G[:, j] * np.exp(1j * m * R.phi0[k]))
                maps.append((n * np.fft.ifft(c)).real)
            out[k] = tuple(maps)
        return out

    def adjoint(self, Q: np.ndarray, U: np.ndarray):
        R = self.s.rings
        GQ = self.s.phi_adjoint(np.asarray(Q, dtype=np.float64))
        GU = self.s.phi_adjoint(np.asarray(U, dtype=np.float64))
        aE = np.zeros(self.nalm, dtype=np.complex128)
        aB = np.zeros(self.nalm, dtype=np.complex128)
        for l, W, X in wx_rows(self.lmax, self.mmax, R.z, R.sin_theta):
            if l < 2:
                continue
            top = W.shape[0] - 1
            i = self.s._idx(l, top)
            aE[i] = np.sum(-W * GQ[:top + 1] - 1j * X * GU[:top + 1], axis=1)
            aB[i] = np.sum(1j * X * GQ[:top + 1] - W * GU[:top + 1], axis=1)
        return aE, aB
