"""Pins of the oracle's constrained-realization solve: dense Cholesky,
operator symmetry and definiteness, the exact Jacobi diagonal, the paper's
closed forms in the harmonic-diagonal model, and special cases."""
import math

import numpy as np
import pytest

import crinputs as ci
from oracle import cr, dense, healpix, sht


def _setup(nside, wl=None, lmax=None):
    wl = ci.workload_masked_t(nside, lmax) if wl is None else wl
    z, phi = healpix.pixel_coords(nside)
    ninv = wl.ninv(z, phi)
    P = cr.Problem(nside, wl.lmax, wl.cl(), wl.bl(), ninv)
    op = cr.CROperator(P)
    d = op.sht.synth(op.b * wl.signal()) + wl.noise(z, phi)
    return wl, P, op, d


@pytest.mark.parametrize("nside", [4, 8])
def test_pcg_matches_dense_cholesky(nside):
    wl, P, op, d = _setup(nside)
    b = op.rhs(d, wl.w0(), wl.w1())
    x, info = cr.pcg(op, b, 1e-13, 5000)
    assert info.converged
    D = dense.DenseY(nside, wl.lmax, lmin=2)
    xd = D.cr_solve(P.cl, P.bl, P.ninv, b)
    assert math.sqrt(op.dot(x - xd, x - xd) / op.dot(xd, xd)) < 1e-10


def test_operator_symmetric_positive_definite():
    wl, P, op, d = _setup(8)
    rng = np.random.default_rng(2)
    for _ in range(3):
        x = op.project(ci.white_alm(rng, wl.lmax))
        y = op.project(ci.white_alm(rng, wl.lmax))
        assert abs(op.dot(x, op.apply(y)) - op.dot(op.apply(x), y)) < 1e-12 * abs(op.dot(x, op.apply(y))) + 1e-12
        assert op.dot(x, op.apply(x)) > 0


@pytest.mark.parametrize("nside", [4, 8])
def test_jacobi_diagonal_equals_dense_diagonal(nside):
    wl, P, op, d = _setup(nside)
    D = dense.DenseY(nside, wl.lmax, lmin=2)
    M = D.cr_matrix(P.cl, P.bl, P.ninv)
    dd = np.diag(M) / D.W
    acc = {}
    for v, (i, k) in zip(dd, D.src):
        acc.setdefault(i, []).append(v)
    dg = op.diag()
    err = max(abs(np.mean(v) - dg[i]) / dg[i] for i, v in acc.items())
    assert err < 1e-13


def test_harmonic_model_closed_forms():
    # paper eqs. hat_s_approx / hat_f_approx: exact in the harmonic-diagonal model
    lmax = 200
    cl = ci.cl_powerlaw(lmax, 1e4)
    bl = ci.gaussian_beam(lmax, 30 * ci.ARCMIN)
    nl = 4 * math.pi * 30.0 ** 2 / (12 * 64 * 64)
    op = cr.HarmonicDiagonalOperator(lmax, cl, bl, nl)
    rng = np.random.default_rng(4)
    r_lm = op.project(ci.white_alm(rng, lmax) * 100)
    w0 = op.project(ci.white_alm(rng, lmax))
    w1 = op.project(ci.white_alm(rng, lmax))
    xm, _ = cr.pcg(op, op.rhs(r_lm=r_lm), 1e-14)
    xf, _ = cr.pcg(op, op.rhs(w0=w0, w1_lm=w1), 1e-14)
    cm, cf = op.closed_form_mean(r_lm), op.closed_form_fluct(w0, w1)
    assert np.max(np.abs(xm - cm)) < 1e-12 * np.max(np.abs(cm))
    assert np.max(np.abs(xf - cf)) < 1e-12 * np.max(np.abs(cf))


def test_full_sky_uniform_noise_close_to_closed_form_at_low_l():
    # On HEALPix the closed form holds only up to the pixel-quadrature error E
    # of (4 pi / Npix) Y^T Y = I + E; at Nside 16 and l <= 4 that error is a
    # few 1e-3, so the CG mean field agrees with eq. hat_s_approx to 1e-2 there.
    nside = 16
    wl = ci.workload_plain_t(nside)
    z, phi = healpix.pixel_coords(nside)
    ninv = wl.ninv(z, phi)
    P = cr.Problem(nside, wl.lmax, wl.cl(), wl.bl(), ninv)
    op = cr.CROperator(P)
    a = wl.signal()
    d = op.sht.synth(op.b * a) + wl.noise(z, phi)
    xm, info = cr.pcg(op, op.rhs(d=d), 1e-12)
    nl = 4 * math.pi * wl.sigma_uk ** 2 / P.ninv.size
    H = cr.HarmonicDiagonalOperator(wl.lmax, P.cl, P.bl, nl)
    r_lm = op.sht.analysis(d, n_iter=3)
    cm = H.closed_form_mean(r_lm)
    low = (op.ls >= 2) & (op.ls <= 4)
    assert np.max(np.abs(xm[low] - cm[low])) < 1e-2 * np.max(np.abs(cm[low]))


def test_fully_masked_gives_prior_draw():
    # paper Sect. 2.2.1, low signal-to-noise limit: N -> infinity gives
    # a^ -> 0 and f^ -> sqrt(C_l) w0 exactly.
    wl, P, op, d = _setup(8)
    P0 = cr.Problem(P.nside, P.lmax, P.cl, P.bl, np.zeros_like(P.ninv))
    op0 = cr.CROperator(P0)
    w0 = wl.w0()
    x, info = cr.pcg(op0, op0.rhs(d, w0, wl.w1()), 1e-14)
    assert np.max(np.abs(x - op0.project(op0.shalf * w0))) < 1e-12 * np.max(np.abs(x))


def test_linearity_in_rhs_terms():
    wl, P, op, d = _setup(8)
    w0, w1 = wl.w0(), wl.w1()
    full = op.rhs(d, w0, w1)
    parts = op.rhs(d=d) + op.rhs(w0=w0) + op.rhs(w1=w1)
    assert np.max(np.abs(full - parts)) < 1e-12 * np.max(np.abs(full))
    xf, _ = cr.pcg(op, full, 1e-13)
    xs = sum(cr.pcg(op, bb, 1e-13)[0] for bb in (op.rhs(d=d), op.rhs(w0=w0), op.rhs(w1=w1)))
    assert math.sqrt(op.dot(xf - xs, xf - xs) / op.dot(xf, xf)) < 1e-9


def test_constrained_realization_covariance_small():
    # The CR solution with random (w0, w1) has covariance A^-1 (eq. mapmakingeq):
    # with d = 0 the sample covariance of many draws approaches the dense inverse.
    nside, lmax = 2, 5
    wl = ci.workload_masked_t(nside, lmax)
    z, phi = healpix.pixel_coords(nside)
    P = cr.Problem(nside, lmax, wl.cl(), wl.bl(), wl.ninv(z, phi))
    D = dense.DenseY(nside, lmax, lmin=2)
    M = D.cr_matrix(P.cl, P.bl, P.ninv)
    # in orthonormal real coordinates v = sqrt(W) u the covariance is (W^-1/2 M W^-1/2)^-1
    sw = np.sqrt(D.W)
    cov_exact = np.linalg.inv(M / sw[:, None] / sw[None, :])
    op = cr.CROperator(P)
    rng = np.random.default_rng(11)
    n = 3000
    samples = []
    for _ in range(n):
        w0 = ci.white_alm(rng, lmax)
        w1 = ci.white_map(rng, P.ninv.size)
        s = D.cr_solve(P.cl, P.bl, P.ninv, op.rhs(None, w0, w1))
        samples.append(D.to_real(s) * sw)
    cov = np.cov(np.array(samples).T)
    dg = np.sqrt(np.diag(cov_exact))
    rel = (cov - cov_exact) / np.outer(dg, dg)
    assert np.max(np.abs(rel)) < 6.0 / math.sqrt(n) * 2
