"""Pins of the oracle's ring-factored Y / Y^T: the dense SciPy matrix (an
independent implementation), single-mode synthesis, adjointness, aliasing,
and planted mistakes that the pins must catch."""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import crinputs as ci
from oracle import dense, healpix, sht


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("nside,lmax", [(1, 2), (2, 5), (4, 11), (8, 23), (4, 20), (2, 9)])
def test_ring_factored_matches_dense(nside, lmax):
    # includes lmax > 3 nside - 1, where m folds onto ring lengths (aliasing)
    S = sht.SHT(nside, lmax)
    D = dense.DenseY(nside, lmax)
    rng = np.random.default_rng(nside * 100 + lmax)
    a = ci.white_alm(rng, lmax)
    x = rng.standard_normal(S.npix)
    assert _rel(S.synth(a), D.synth(a)) < 1e-12
    assert _rel(S.adjoint(x), D.adjoint(x)) < 1e-12


@pytest.mark.parametrize("l,m", [(0, 0), (3, 0), (5, 2), (9, 9), (20, 13)])
def test_single_mode_synthesis(l, m):
    nside, lmax = 8, 23
    S = sht.SHT(nside, lmax)
    a = np.zeros(S.nalm, dtype=np.complex128)
    a[S.ms[m] + l - m] = 1.0
    z, phi = healpix.pixel_coords(nside)
    y = sph_harm_y(l, m, np.arccos(z), phi)
    expect = y.real if m == 0 else 2.0 * y.real
    assert np.allclose(S.synth(a), expect, atol=1e-13)


@pytest.mark.parametrize("nside,lmax,mmax", [(16, 47, 47), (32, 95, 60), (8, 40, 40)])
def test_adjointness(nside, lmax, mmax):
    S = sht.SHT(nside, lmax, mmax)
    rng = np.random.default_rng(3)
    a = ci.white_alm(rng, lmax, mmax)
    y = rng.standard_normal(S.npix)
    lhs = float(np.dot(S.synth(a), y))
    rhs = sht.dot(a, S.adjoint(y), lmax, mmax)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + np.linalg.norm(y))


def test_analysis_recovers_bandlimited_alm():
    nside, lmax = 32, 40
    S = sht.SHT(nside, lmax)
    a = ci.white_alm(np.random.default_rng(9), lmax)
    a[S.ms[0]:S.ms[0] + lmax + 1] = a[S.ms[0]:S.ms[0] + lmax + 1].real
    got = S.analysis(S.synth(a), n_iter=4)
    assert _rel(got, a) < 1e-6


def test_sum_y00():
    S = sht.SHT(8, 0)
    x = np.ones(S.npix)
    assert abs(S.adjoint(x)[0] - S.npix / math.sqrt(4 * math.pi)) < 1e-10


# ---------------------------------------------------------------- planted mistakes
class _WrongPhase(sht.SHT):
    def phi_synth(self, F):            # e^{-i m phi0} instead of e^{+i m phi0}
        R = self.rings
        out = np.empty(self.npix)
        m = np.arange(self.mmax + 1)
        wm = np.where(m == 0, 1.0, 2.0)
        for k in range(R.nrings):
            n, f0 = int(R.nphi[k]), int(R.first[k])
            c = np.zeros(n, dtype=np.complex128)
            np.add.at(c, m % n, wm * F[:, k] * np.exp(-1j * m * R.phi0[k]))
            out[f0:f0 + n] = (n * np.fft.ifft(c)).real
        return out


class _NoWeightTwo(sht.SHT):
    def phi_synth(self, F):            # forgets the factor 2 of the m > 0 terms
        R = self.rings
        out = np.empty(self.npix)
        m = np.arange(self.mmax + 1)
        for k in range(R.nrings):
            n, f0 = int(R.nphi[k]), int(R.first[k])
            c = np.zeros(n, dtype=np.complex128)
            np.add.at(c, m % n, F[:, k] * np.exp(1j * m * R.phi0[k]))
            out[f0:f0 + n] = (n * np.fft.ifft(c)).real
        return out


class _NoFold(sht.SHT):
    def phi_adjoint(self, x):          # drops m >= n_phi instead of folding
        G = super().phi_adjoint(x)
        R = self.rings
        m = np.arange(self.mmax + 1)
        for k in range(R.nrings):
            G[m >= R.nphi[k], k] = 0
        return G


@pytest.mark.parametrize("cls", [_WrongPhase, _NoWeightTwo, _NoFold])
def test_planted_mistakes_are_caught(cls):
    nside, lmax = 4, 11
    bad = cls(nside, lmax)
    D = dense.DenseY(nside, lmax)
    rng = np.random.default_rng(1)
    a = ci.white_alm(rng, lmax)
    x = rng.standard_normal(bad.npix)
    err = max(_rel(bad.synth(a), D.synth(a)), _rel(bad.adjoint(x), D.adjoint(x)))
    assert err > 1e-3
