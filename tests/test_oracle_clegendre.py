"""Pins of the oracle's plain-C Legendre sums (``oracle/legendre_sums.c``,
used for the Nside 512 and 1024 parity cases) and of the remaining oracle
helpers: the C sums equal the numpy sums (themselves pinned to SciPy's dense
Y), the C lambda_lm equal SciPy's Y_lm at l <= 100 and satisfy the addition
theorem deep in the underflow region of the Nside 1024 polar ring; the
sampled-ring synthesis equals the full synthesis; ring-factored Y equals the
dense Y, and PCG equals the dense Cholesky solve, at Nside 16."""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import crinputs as ci
from oracle import clegendre, cr, dense, healpix, sht


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("nside,lmax,mmax", [(1, 2, None), (2, 5, None), (4, 11, None), (4, 20, None), (8, 23, None),
                                             (6, 17, None), (16, 47, None), (32, 95, None), (32, 60, 33)])
def test_c_sums_equal_numpy_sums(nside, lmax, mmax):
    S = sht.SHT(nside, lmax, mmax)
    C = sht.SHT(nside, lmax, mmax, fast=True)
    rng = np.random.default_rng(nside * 1000 + lmax)
    a = ci.white_alm(rng, lmax, mmax)
    G = rng.standard_normal((S.mmax + 1, S.rings.nrings)) + 1j * rng.standard_normal((S.mmax + 1, S.rings.nrings))
    assert _rel(C.legendre_synth(a), S.legendre_synth(a)) < 1e-13
    assert _rel(C.legendre_adjoint(G), S.legendre_adjoint(G)) < 1e-13
    assert _rel(C.legendre_adjoint(G, square=True), S.legendre_adjoint(G, square=True)) < 1e-13
    x = rng.standard_normal(S.npix)
    assert _rel(C.synth(a), S.synth(a)) < 1e-13
    assert _rel(C.adjoint(x), S.adjoint(x)) < 1e-13


@pytest.mark.parametrize("m", [0, 1, 7, 40, 100])
def test_c_lambda_equals_scipy(m):
    lmax = 100
    z = np.array([-0.97, -0.3, 0.0, 0.12, 0.5, 0.999])
    st = np.sqrt((1 - z) * (1 + z))
    lam = clegendre.lambda_m(lmax, m, z, st)
    theta = np.arccos(z)
    for l in range(m, lmax + 1):
        ref = sph_harm_y(l, m, theta, np.zeros_like(z)).real
        assert np.max(np.abs(lam[l - m] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), l


def test_c_lambda_addition_theorem_underflow_region():
    # sum_{m=-l}^{l} lambda_lm^2 = (2l+1)/(4 pi) at the first ring of Nside
    # 1024 (sin theta = 8e-4: lambda_mm underflows double for m above ~100)
    # and at the equator, every l up to 2047 checked through all m
    nside, lmax = 1024, 2047
    R = healpix.rings(nside)
    rings = [0, 5, 2 * nside - 1]
    z, st = R.z[rings], R.sin_theta[rings]
    tot = np.zeros((lmax + 1, len(rings)))
    for m in range(lmax + 1):
        lam = clegendre.lambda_m(lmax, m, z, st)
        tot[m:] += (1.0 if m == 0 else 2.0) * lam * lam
    ref = (2 * np.arange(lmax + 1) + 1)[:, None] / (4 * math.pi)
    err = np.abs(tot - ref) / ref
    # rounding of the m = 0 recurrence grows near z = 1 (1.1e-10 at l = 2047
    # on the first ring, 6e-13 on ring 5, 3e-15 at the equator); a wrong
    # coefficient or exponent gives errors of order one
    assert np.max(err[:, 0]) < 1e-9
    assert np.max(err[:, 1:]) < 1e-11
    # parity lambda(-z) = (-1)^(l+m) lambda(z) on a mirrored pair
    for m in (0, 3, 500):
        a = clegendre.lambda_m(lmax, m, z[:1], st[:1])[:, 0]
        b = clegendre.lambda_m(lmax, m, -z[:1], st[:1])[:, 0]
        sgn = (-1.0) ** (np.arange(m, lmax + 1) + m)
        assert np.max(np.abs(b - sgn * a)) <= 1e-13 * max(np.max(np.abs(a)), 1e-300)


@pytest.mark.parametrize("nside,lmax", [(16, 47), (32, 95)])
def test_synth_rings_equals_full_synthesis(nside, lmax):
    S = sht.SHT(nside, lmax)
    a = ci.white_alm(np.random.default_rng(nside), lmax)
    full = S.synth(a)
    R = S.rings
    rings = [0, 1, nside - 1, nside, 2 * nside - 1, 3 * nside, R.nrings - 2, R.nrings - 1]
    got = sht.synth_rings(S, a, rings)
    for k in rings:
        f, n = int(R.first[k]), int(R.nphi[k])
        assert _rel(got[k], full[f:f + n]) < 1e-13, k


def test_ring_factored_matches_dense_nside16():
    nside, lmax = 16, 47
    D = dense.DenseY(nside, lmax)
    rng = np.random.default_rng(1647)
    a = ci.white_alm(rng, lmax)
    x = rng.standard_normal(12 * nside * nside)
    for S in (sht.SHT(nside, lmax), sht.SHT(nside, lmax, fast=True)):
        assert _rel(S.synth(a), D.synth(a)) < 1e-12
        assert _rel(S.adjoint(x), D.adjoint(x)) < 1e-12


def test_pcg_matches_dense_cholesky_nside16():
    nside = 16
    wl = ci.workload_masked_t(nside)
    z, phi = healpix.pixel_coords(nside)
    P = cr.Problem(nside, wl.lmax, wl.cl(), wl.bl(), wl.ninv(z, phi))
    op = cr.CROperator(P, sht.SHT(nside, wl.lmax, fast=True))
    d = op.sht.synth(op.b * wl.signal()) + wl.noise(z, phi)
    b = op.rhs(d, wl.w0(), wl.w1())
    x, info = cr.pcg(op, b, 1e-13, 5000)
    assert info.converged
    xd = dense.DenseY(nside, wl.lmax, lmin=2).cr_solve(P.cl, P.bl, P.ninv, b)
    assert math.sqrt(op.dot(x - xd, x - xd) / op.dot(xd, xd)) < 1e-10
