"""Pins of the oracle's lambda_lm recurrence: closed forms, SciPy, an
arbitrary-precision library in the underflow region, the addition theorem,
parity and orthonormality on an exact quadrature."""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy.special import sph_harm_y, roots_legendre

from oracle import healpix
from oracle.legendre import lambda_rows, lambda_table, lambda_single, log10_abs_lambda

GOLD = os.path.join(os.path.dirname(__file__), "golden")

_TRIG = {
    "1": lambda c, s: np.ones_like(c),
    "cos": lambda c, s: c,
    "sin": lambda c, s: s,
    "3cos2-1": lambda c, s: 3 * c * c - 1,
    "sin*cos": lambda c, s: s * c,
    "sin2": lambda c, s: s * s,
    "5cos3-3cos": lambda c, s: 5 * c ** 3 - 3 * c,
    "sin3": lambda c, s: s ** 3,
}


def test_closed_forms_golden():
    r = healpix.rings(8)
    lam = lambda_table(3, 3, r.z, r.sin_theta)
    with open(os.path.join(GOLD, "ylm_closed_forms.txt")) as fh:
        rows = [ln.split("#")[0].split() for ln in fh if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 8
    for l, m, coef, form in rows:
        l, m, coef = int(l), int(m), float(coef)
        expect = coef * _TRIG[form](r.z, r.sin_theta)
        assert np.allclose(lam[l, m], expect, rtol=1e-14, atol=1e-15), (l, m)


def test_against_scipy_low_l():
    rng = np.random.default_rng(5)
    z = np.concatenate([rng.uniform(-1, 1, 40), [0.0, 0.999, -0.999]])
    st = np.sqrt((1 - z) * (1 + z))
    theta = np.arccos(z)
    lmax = 100
    lam = lambda_table(lmax, lmax, z, st)
    worst = 0.0
    for l in range(lmax + 1):
        for m in range(l + 1):
            ref = sph_harm_y(l, m, theta, 0.0).real
            worst = max(worst, np.max(np.abs(lam[l, m] - ref)) / math.sqrt((2 * l + 1) / (4 * math.pi)))
    assert worst < 1e-12


def _log10_abs_mp(l, m, z):
    # Ferrers function without the Condon-Shortley phase from its terminating
    # hypergeometric series (DLMF 14.3.1 with 15.2.1), in 80-digit arithmetic:
    # P_l^m(x) = (l+m)! / ((l-m)! 2^m m!) (1-x^2)^{m/2} 2F1(m-l, m+l+1; m+1; (1-x)/2)
    mpmath.mp.dps = 80
    x = mpmath.mpf(z)
    t = (1 - x) / 2
    term, s = mpmath.mpf(1), mpmath.mpf(1)
    for k in range(l - m):
        term *= mpmath.mpf(m - l + k) * (m + l + 1 + k) / ((m + 1 + k) * (k + 1)) * t
        s += term
    P = mpmath.factorial(l + m) / (mpmath.factorial(l - m) * mpmath.mpf(2) ** m * mpmath.factorial(m)) \
        * (1 - x * x) ** (mpmath.mpf(m) / 2) * s
    norm = mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l - m) / mpmath.factorial(l + m))
    return float(mpmath.log10(abs(P * norm)))


@pytest.mark.parametrize("l,m,ring", [(2047, 2000, 1), (2047, 1500, 1), (1535, 1535, 1), (300, 250, 3)])
def test_underflow_region_against_mpmath(l, m, ring):
    # polar-most rings of Nside 1024 / 512 where lambda ~ 10^-5000 underflows double
    nside = 1024 if l == 2047 else 512
    r = healpix.rings(nside)
    z = float(r.z[ring - 1])
    ours = log10_abs_lambda(l, m, z)
    ref = _log10_abs_mp(l, m, z)
    assert ref < -300 or l == 300
    assert abs(ours - ref) < 1e-10 * max(1.0, abs(ref))


@pytest.mark.parametrize("nside,lmax", [(512, 1535), (1024, 2047)])
def test_addition_theorem_polar_and_equator(nside, lmax):
    # sum_{m=-l}^{l} |Y_lm|^2 = (2l+1)/(4 pi) at every point, including rings
    # where the large-m terms underflow.
    r = healpix.rings(nside)
    idx = [0, 1, 2, 5, nside - 1, 2 * nside - 1]
    z, st = r.z[idx], r.sin_theta[idx]
    for l, lam in lambda_rows(lmax, lmax, z, st):
        if l in (0, 1, 2, 100, lmax // 2, lmax):
            s = lam[0] ** 2 + 2 * np.sum(lam[1:] ** 2, axis=0)
            assert np.allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-10), l


def test_parity():
    z = np.array([0.3, 0.77, 0.05])
    st = np.sqrt(1 - z * z)
    lp = lambda_table(40, 40, z, st)
    lm = lambda_table(40, 40, -z, st)
    for l in range(41):
        for m in range(l + 1):
            assert np.allclose(lm[l, m], (-1) ** (l + m) * lp[l, m], rtol=1e-13, atol=1e-16)


def test_orthonormality_gauss_legendre():
    # 2 pi sum_k w_k lambda_lm(x_k) lambda_l'm(x_k) = delta_ll' exactly for
    # l, l' <= lmax with lmax+1 Gauss-Legendre nodes (polynomial degree <= 2 lmax)
    lmax = 30
    x, w = roots_legendre(lmax + 1)
    lam = lambda_table(lmax, lmax, x, np.sqrt(1 - x * x))
    for m in range(lmax + 1):
        L = lam[m:, m, :]
        G = 2 * math.pi * (L * w[None, :]) @ L.T
        assert np.allclose(G, np.eye(lmax + 1 - m), atol=1e-13)


def test_single_point_helper():
    assert abs(lambda_single(1, 1, 0.0) + math.sqrt(3 / (8 * math.pi))) < 1e-15
