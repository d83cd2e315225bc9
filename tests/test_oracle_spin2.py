"""Pins of the spin-2 oracle (oracle/spin2.py): the spin-weighted functions
against the spin-raising / lowering operators applied to the scalar harmonic
(numerical differentiation in 50-digit arithmetic), exact orthonormality on
a Gauss-Legendre grid, adjointness of the polarised transforms and the
azimuthally symmetric special cases."""
import math

import mpmath
import numpy as np
import pytest

import crinputs as ci
from oracle import spin2
from oracle.sht import dot, lm_arrays


def _lam_mp(l, m, t):
    """lambda_lm(cos t) with one (-1)^m (no Condon-Shortley in P), from the
    terminating hypergeometric series of the Ferrers function (DLMF 14.3.1)."""
    x = mpmath.cos(t)
    u = (1 - x) / 2
    term, s = mpmath.mpf(1), mpmath.mpf(1)
    for k in range(l - m):
        term *= mpmath.mpf(m - l + k) * (m + l + 1 + k) / ((m + 1 + k) * (k + 1)) * u
        s += term
    P = mpmath.factorial(l + m) / (mpmath.factorial(l - m) * mpmath.mpf(2) ** m * mpmath.factorial(m)) \
        * mpmath.sin(t) ** m * s
    norm = mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l - m) / mpmath.factorial(l + m))
    return (-1) ** m * norm * P


def _wx_by_eth(l, m, theta):
    """(W, X) from +-2Y = eth^2 Y / N, ethbar^2 Y / N (Goldberg et al. 1967)."""
    mpmath.mp.dps = 50
    t = mpmath.mpf(theta)
    f = lambda tt: _lam_mp(l, m, tt)
    L0, L1, L2 = f(t), mpmath.diff(f, t, 1), mpmath.diff(f, t, 2)
    s, c = mpmath.sin(t), mpmath.cos(t)
    g = -(L1 - m / s * L0)
    gp = -(L2 - m / s * L1 + m * c / s ** 2 * L0)
    eth2 = -(gp - (m / s + c / s) * g)
    h = -(L1 + m / s * L0)
    hp = -(L2 + m / s * L1 - m * c / s ** 2 * L0)
    ethb2 = -(hp + (m / s - c / s) * h)
    n = mpmath.sqrt(mpmath.mpf((l - 1) * l * (l + 1) * (l + 2)))
    p2, m2 = eth2 / n, ethb2 / n
    return float((p2 + m2) / 2), float((p2 - m2) / 2)


@pytest.mark.parametrize("theta", [0.31, 1.1, 1.9, 2.95])
def test_wx_against_spin_raising_operators(theta):
    lmax = 14
    z = np.array([math.cos(theta)])
    st = np.array([math.sin(theta)])
    rows = {l: (W[:, 0], X[:, 0]) for l, W, X in spin2.wx_rows(lmax, lmax, z, st)}
    for l in (2, 3, 5, 9, 14):
        for m in sorted({0, 1, 2, l // 2, l - 1, l}):
            w, x = _wx_by_eth(l, m, theta)
            assert abs(rows[l][0][m] - w) <= 1e-12 * max(1.0, abs(w)), (l, m, rows[l][0][m], w)
            assert abs(rows[l][1][m] - x) <= 1e-12 * max(1.0, abs(x)), (l, m, rows[l][1][m], x)


def test_spin2_orthonormal_gauss_legendre():
    lmax = 24
    x, w = np.polynomial.legendre.leggauss(lmax + 8)
    st = np.sqrt((1 - x) * (1 + x))
    W = np.zeros((lmax + 1, lmax + 1, x.size))
    X = np.zeros_like(W)
    for l, Wl, Xl in spin2.wx_rows(lmax, lmax, x, st):
        W[l, :Wl.shape[0]] = Wl
        X[l, :Xl.shape[0]] = Xl
    for m in (0, 1, 2, 7, 20):
        for sgn in (1.0, -1.0):
            Ys = W[:, m] + sgn * X[:, m]              # [l, node]
            G = 2 * math.pi * (Ys * w) @ Ys.T
            lo = max(2, m)
            expect = np.zeros_like(G)
            expect[np.arange(lo, lmax + 1), np.arange(lo, lmax + 1)] = 1.0
            assert np.max(np.abs(G[lo:, lo:] - expect[lo:, lo:])) < 1e-12, (m, sgn)


def _proj(a, lmax):
    ls, ms = lm_arrays(lmax, lmax)
    a = np.where(ls >= 2, a, 0)
    a = a.astype(np.complex128)
    a[ms == 0] = a[ms == 0].real
    return a


@pytest.mark.parametrize("nside,lmax", [(4, 11), (8, 23), (6, 17)])
def test_polarised_transforms_adjoint(nside, lmax):
    P = spin2.PolSHT(nside, lmax)
    rng = np.random.default_rng(nside)
    aE, aB = _proj(ci.white_alm(rng, lmax), lmax), _proj(ci.white_alm(rng, lmax), lmax)
    Q2, U2 = rng.standard_normal(P.npix), rng.standard_normal(P.npix)
    Q, U = P.synth(aE, aB)
    e2, b2 = P.adjoint(Q2, U2)
    lhs = float(Q @ Q2 + U @ U2)
    rhs = dot(aE, e2, lmax, lmax) + dot(aB, b2, lmax, lmax)
    assert abs(lhs - rhs) <= 1e-12 * (np.linalg.norm(Q) * np.linalg.norm(Q2) + np.linalg.norm(U) * np.linalg.norm(U2))


def test_axisymmetric_e_and_b_modes():
    nside, lmax = 8, 23
    P = spin2.PolSHT(nside, lmax)
    ls, ms = lm_arrays(lmax, lmax)
    rng = np.random.default_rng(2)
    a0 = np.where((ms == 0) & (ls >= 2), rng.standard_normal(ls.size), 0.0).astype(np.complex128)
    Q, U = P.synth(a0, np.zeros_like(a0))
    assert np.max(np.abs(U)) < 1e-13 * np.max(np.abs(Q))
    Q, U = P.synth(np.zeros_like(a0), a0)
    assert np.max(np.abs(Q)) < 1e-13 * np.max(np.abs(U))


def test_synth_rings_equals_full_synthesis():
    nside, lmax = 8, 23
    P = spin2.PolSHT(nside, lmax)
    rng = np.random.default_rng(4)
    aE, aB = _proj(ci.white_alm(rng, lmax), lmax), _proj(ci.white_alm(rng, lmax), lmax)
    Q, U = P.synth(aE, aB)
    rings = [0, 3, 14, 15, 16, 30]
    got = P.synth_rings(aE, aB, rings)
    R = P.s.rings
    for k in rings:
        f, n = int(R.first[k]), int(R.nphi[k])
        assert np.allclose(got[k][0], Q[f:f + n], rtol=0, atol=1e-13 * np.abs(Q).max())
        assert np.allclose(got[k][1], U[f:f + n], rtol=0, atol=1e-13 * np.abs(U).max())
