"""Spherical-harmonic synthesis Y and its exact transpose Y^T on HEALPix.

Definitions (paper: a(n) = sum_lm a_lm Y_lm(n), Sect. 2.1; the pixel sums
sum_p Y*_lm(p) ... of App. A, which fix Y^T as the plain transpose with no
quadrature weight):

    (Y a)_p   = sum_l [ a_l0 lambda_l0(z_p) + 2 Re sum_{m=1}^{min(l,mmax)} a_lm lambda_lm(z_p) e^{i m phi_p} ]
    (Y^T x)_lm = sum_p x_p lambda_lm(z_p) e^{-i m phi_p}

for a real field stored as m >= 0 (a_l0 real). Under the inner product
<a, c> = sum_l a_l0 c_l0 + 2 sum_{m>0} Re(a_lm conj c_lm), Y^T is the adjoint
of Y.

Ring factorisation (exact, just a regrouping of the same sums):
Legendre step  F_r(m) = sum_l lambda_lm(z_r) a_lm,
azimuthal step (Y a)_{r,j} = Re sum_k c_k e^{2 pi i j k / n_r}, with
c_k = sum_{m = k mod n_r} w_m F_r(m) e^{i m phi0_r}, w_0 = 1, w_m = 2,
evaluated with numpy's FFT; the transpose runs the same two steps backwards.
"""
from __future__ import annotations

import math

import numpy as np

from . import healpix
from .legendre import lambda_rows


def nalm(lmax: int, mmax: int) -> int:
    return (mmax + 1) * (lmax + 1) - (mmax * (mmax + 1)) // 2


def mstart(lmax: int, mmax: int) -> np.ndarray:
    """Index of a_{m,m} in the m-major layout, for m = 0..mmax."""
    m = np.arange(mmax + 1)
    return m * (lmax + 1) - (m * (m - 1)) // 2


def lm_arrays(lmax: int, mmax: int):
    ls, ms = [], []
    for m in range(mmax + 1):
        ls.append(np.arange(m, lmax + 1))
        ms.append(np.full(lmax + 1 - m, m))
    return np.concatenate(ls), np.concatenate(ms)


def real_weight(lmax: int, mmax: int) -> np.ndarray:
    """w_m per stored coefficient: 1 for m = 0, 2 for m > 0."""
    _, ms = lm_arrays(lmax, mmax)
    return np.where(ms == 0, 1.0, 2.0)


def dot(a: np.ndarray, c: np.ndarray, lmax: int, mmax: int) -> float:
    """Real-field inner product <a, c>."""
    w = real_weight(lmax, mmax)
    return float(np.sum(w * (a.real * c.real + a.imag * c.imag)))


class SHT:
    """Y and Y^T for one (nside, lmax, mmax).

    fast=True evaluates the two Legendre sums with the plain-C loops of
    ``clegendre`` (the same recurrence and sums, for the large workloads);
    the azimuthal step is numpy's FFT either way."""

    def __init__(self, nside: int, lmax: int, mmax: int | None = None, fast: bool = False):
        self.fast = fast
        self.nside, self.lmax = nside, lmax
        self.mmax = lmax if mmax is None else mmax
        if self.mmax > lmax:
            raise ValueError("mmax > lmax")
        self.rings = healpix.rings(nside)
        self.npix = self.rings.npix
        self.nalm = nalm(lmax, self.mmax)
        self.ms = mstart(lmax, self.mmax)

    # -- Legendre step ---------------------------------------------------
    def _idx(self, l: int, top: int) -> np.ndarray:
        m = np.arange(top + 1)
        return self.ms[:top + 1] + l - m

    def legendre_synth(self, alm: np.ndarray) -> np.ndarray:
        """F[m, r] = sum_l lambda_lm(z_r) a_lm (complex)."""
        R = self.rings
        if self.fast:
            from . import clegendre
            return clegendre.legendre_synth(self.lmax, self.mmax, R.z, R.sin_theta, alm)
        F = np.zeros((self.mmax + 1, R.nrings), dtype=np.complex128)
        for l, lam in lambda_rows(self.lmax, self.mmax, R.z, R.sin_theta):
            top = lam.shape[0] - 1
            F[:top + 1] += lam * alm[self._idx(l, top)][:, None]
        return F

    def legendre_adjoint(self, G: np.ndarray, square: bool = False) -> np.ndarray:
        """out_lm = sum_r lambda_lm(z_r) G[m, r] (lambda^2 if square)."""
        R = self.rings
        if self.fast:
            from . import clegendre
            return clegendre.legendre_adjoint(self.lmax, self.mmax, R.z, R.sin_theta, G, square)
        out = np.zeros(self.nalm, dtype=np.complex128)
        for l, lam in lambda_rows(self.lmax, self.mmax, R.z, R.sin_theta):
            top = lam.shape[0] - 1
            w = lam * lam if square else lam
            out[self._idx(l, top)] = np.sum(w * G[:top + 1], axis=1)
        return out

    # -- azimuthal step --------------------------------------------------
    def phi_synth(self, F: np.ndarray) -> np.ndarray:
        R = self.rings
        out = np.empty(self.npix)
        m = np.arange(self.mmax + 1)
        wm = np.where(m == 0, 1.0, 2.0)
        for k in range(R.nrings):
            n, f0 = int(R.nphi[k]), int(R.first[k])
            c = np.zeros(n, dtype=np.complex128)
            np.add.at(c, m % n, wm * F[:, k] * np.exp(1j * m * R.phi0[k]))
            out[f0:f0 + n] = (n * np.fft.ifft(c)).real
        return out

    def phi_adjoint(self, x: np.ndarray) -> np.ndarray:
        R = self.rings
        G = np.empty((self.mmax + 1, R.nrings), dtype=np.complex128)
        m = np.arange(self.mmax + 1)
        for k in range(R.nrings):
            n, f0 = int(R.nphi[k]), int(R.first[k])
            X = np.fft.fft(x[f0:f0 + n])
            G[:, k] = np.exp(-1j * m * R.phi0[k]) * X[m % n]
        return G

    # -- full transforms -------------------------------------------------
    def synth(self, alm: np.ndarray) -> np.ndarray:
        return self.phi_synth(self.legendre_synth(np.asarray(alm, dtype=np.complex128)))

    def adjoint(self, x: np.ndarray) -> np.ndarray:
        return self.legendre_adjoint(self.phi_adjoint(np.asarray(x, dtype=np.float64)))

    def analysis(self, x: np.ndarray, n_iter: int = 0) -> np.ndarray:
        """a = (4 pi / Npix) Y^T x, then n_iter Jacobi corrections
        a += (4 pi / Npix) Y^T (x - Y a)."""
        wq = 4.0 * math.pi / self.npix
        a = wq * self.adjoint(x)
        for _ in range(n_iter):
            a = a + wq * self.adjoint(x - self.synth(a))
        return a

    def ring_weights(self, ninv: np.ndarray) -> np.ndarray:
        """W_r = sum of ninv over the pixels of ring r."""
        R = self.rings
        return np.array([ninv[int(R.first[k]):int(R.first[k]) + int(R.nphi[k])].sum()
                         for k in range(R.nrings)])


def synth_rings(sht: SHT, alm: np.ndarray, ring_idx) -> dict:
    """Map values on selected rings only (ring index -> pixel values), the
    same two sums as SHT.synth restricted to those rings."""
    R = sht.rings
    ring_idx = list(ring_idx)
    z, st = R.z[ring_idx], R.sin_theta[ring_idx]
    F = np.zeros((sht.mmax + 1, len(ring_idx)), dtype=np.complex128)
    for l, lam in lambda_rows(sht.lmax, sht.mmax, z, st):
        top = lam.shape[0] - 1
        F[:top + 1] += lam * alm[sht._idx(l, top)][:, None]
    m = np.arange(sht.mmax + 1)
    wm = np.where(m == 0, 1.0, 2.0)
    out = {}
    for j, k in enumerate(ring_idx):
        n = int(R.nphi[k])
        c = np.zeros(n, dtype=np.complex128)
        np.add.at(c, m % n, wm * F[:, j] * np.exp(1j * m * R.phi0[k]))
        out[k] = (n * np.fft.ifft(c)).real
    return out
