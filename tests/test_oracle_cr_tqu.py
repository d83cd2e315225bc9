"""Pins of the T+Q+U constrained-realization oracle (oracle/cr_tqu.py): dense
Cholesky solve of the real-parametrised system, symmetry, the temperature
block against the pinned T-only operator when TE = 0, the fully masked sky,
and the 3x3 spectra blocks."""
import math

import numpy as np
import pytest

import crinputs as ci
from oracle import cr, cr_tqu, healpix
from oracle.sht import lm_arrays


def tqu_problem(nside, lmax=None, te=0.3, seed=1, fwhm_arcmin=None):
    lmax = 3 * nside - 1 if lmax is None else lmax
    fw = (60.0 * 64 / nside) if fwhm_arcmin is None else fwhm_arcmin
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=fw, cfg=2)
    z, phi = healpix.pixel_coords(nside)
    cl = ci.cl_tqu(lmax, wl.amp, te)
    nt = wl.ninv(z, phi)
    P = cr_tqu.ProblemTQU(nside, lmax, cl, wl.bl(), nt, nt / 2.0)
    return wl, P


def _real_basis(lmax):
    """Columns J such that the complex (3, nalm) vector of real dofs u is J u,
    orthonormal in the real-field inner product."""
    ls, ms = lm_arrays(lmax, lmax)
    cols = []
    for k in range(3):
        for i in np.flatnonzero(ls >= 2):
            e = np.zeros((3, ls.size), dtype=np.complex128)
            if ms[i] == 0:
                e[k, i] = 1.0
                cols.append(e)
            else:
                e[k, i] = 1.0 / math.sqrt(2.0)
                cols.append(e)
                e2 = np.zeros_like(e)
                e2[k, i] = 1j / math.sqrt(2.0)
                cols.append(e2)
    return cols


def test_pcg_matches_dense_cholesky():
    wl, P = tqu_problem(4, 11)
    op = cr_tqu.CROperatorTQU(P)
    rng = np.random.default_rng(3)
    d = rng.standard_normal((3, op.sht.npix)) * 50.0
    w0 = np.stack([ci.white_alm(rng, 11) for _ in range(3)])
    w1 = rng.standard_normal((3, op.sht.npix))
    b = op.rhs(d=d, w0=w0, w1=w1)
    J = _real_basis(11)
    AJ = [op.apply(ej) for ej in J]
    A = np.array([[op.dot(ei, aj) for aj in AJ] for ei in J])
    assert np.allclose(A, A.T, rtol=1e-10, atol=1e-10 * np.abs(A).max())
    L = np.linalg.cholesky(A)
    bu = np.array([op.dot(ei, b) for ei in J])
    u = np.linalg.solve(L.T, np.linalg.solve(L, bu))
    ref = sum(ui * ei for ui, ei in zip(u, J))
    x, info = cr.pcg(op, b, 1e-13, 5000)
    assert info.converged
    assert op.norm(x - ref) <= 1e-10 * op.norm(ref)


def test_temperature_block_equals_t_only_when_te_zero():
    wl, P = tqu_problem(8, 23, te=0.0)
    op = cr_tqu.CROperatorTQU(P)
    opT = cr.CROperator(cr.Problem(8, 23, P.cl[0], P.bl, P.ninv_t, 2))
    rng = np.random.default_rng(4)
    x = op.project(np.stack([ci.white_alm(rng, 23) for _ in range(3)]))
    y = op.apply(x)
    assert np.allclose(y[0], opT.apply(x[0]), rtol=0, atol=1e-12 * np.abs(y[0]).max())
    assert np.allclose(op.diag()[0], opT.diag(), rtol=1e-13)


def test_operator_symmetric_and_masked_sky_gives_prior_draw():
    wl, P = tqu_problem(4, 11)
    op = cr_tqu.CROperatorTQU(P)
    rng = np.random.default_rng(5)
    x = op.project(np.stack([ci.white_alm(rng, 11) for _ in range(3)]))
    y = op.project(np.stack([ci.white_alm(rng, 11) for _ in range(3)]))
    assert abs(op.dot(op.apply(x), y) - op.dot(x, op.apply(y))) <= 1e-11 * op.norm(x) * op.norm(op.apply(y))
    P0 = cr_tqu.ProblemTQU(4, 11, P.cl, P.bl, np.zeros_like(P.ninv_t), np.zeros_like(P.ninv_p))
    op0 = cr_tqu.CROperatorTQU(P0)
    w0 = op0.project(np.stack([ci.white_alm(rng, 11) for _ in range(3)]))
    s, info = cr.pcg(op0, op0.rhs(w0=w0), 1e-14)
    # s = S^{1/2} w0: S^-1/2 s = S^-1 ... i.e. S^-1/2 applied to s gives back w0
    back = op0._block(op0.sinvh_lm, s)
    assert op0.norm(back - w0) <= 1e-11 * op0.norm(w0)


def test_spectra_blocks():
    lmax = 40
    cl = ci.cl_tqu(lmax, ci.amplitude_for_rms(lmax), 0.3)
    sinv, sinvh = cr_tqu.spectra_blocks(cl, lmax)
    for l in (2, 10, 40):
        C = np.array([[cl[0][l], cl[3][l], 0], [cl[3][l], cl[1][l], 0], [0, 0, cl[2][l]]])
        assert np.allclose(sinv[l] @ C, np.eye(3), atol=1e-12)
        assert np.allclose(sinvh[l], sinvh[l].T)
        assert np.allclose(sinvh[l] @ sinvh[l], sinv[l], rtol=1e-12)
    assert np.all(sinv[:2] == 0)
