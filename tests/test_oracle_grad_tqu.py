"""Pins of the oracle's T+Q+U gradient of ln pi over C_l bins
(oracle/grad.py grad_lnpi_tqu): central finite differences of its own ln pi
with a step of 1e-4 relative on every bin, and the reduction to the pinned
temperature gradient when the polarisation carries no data (N_P^-1 = 0) and
TE = 0 (the E and B mean fields vanish and the adjoint solve has no E, B part,
so every bin derivative equals the temperature one). A planted mistake (the
S^-1/2 term dropped) fails the finite differences."""
import math

import numpy as np

import crinputs as ci
from oracle import cr, cr_tqu, grad, healpix


def _problem(nside=4, te=0.3, pol=True, seed=3):
    wl = ci.workload_masked_t(nside)
    z, phi = healpix.pixel_coords(nside)
    nt = wl.ninv(z, phi)
    cl = np.ascontiguousarray(ci.cl_tqu(wl.lmax, wl.amp, te))
    P = cr_tqu.ProblemTQU(nside, wl.lmax, cl, wl.bl(), nt, nt / 2.0 if pol else 0.0 * nt, 2)
    rng = np.random.default_rng(seed)
    npix = 12 * nside * nside
    op = cr_tqu.CROperatorTQU(P)
    a = np.stack([ci.signal_alm(rng, cl[0], wl.lmax) for _ in range(3)])
    d = op.synth(op.b * op.project(a)) + rng.standard_normal((3, npix)) * 10.0
    w0 = np.stack([ci.white_alm(rng, wl.lmax) for _ in range(3)])
    w1 = rng.standard_normal((3, npix))
    return wl, P, d, w0, w1


def test_tqu_gradient_matches_central_differences():
    wl, P, d, w0, w1 = _problem()
    edges = np.array([2, 4, 6, 9, wl.lmax + 1])
    g, L = grad.grad_lnpi_tqu(P, d, w0, w1, edges)
    h = 1e-4
    for k in range(edges.size - 1):
        e = np.zeros(edges.size - 1)
        e[k] = h
        fd = (grad.lnpi_at_tqu(P, d, w0, w1, edges, e) - grad.lnpi_at_tqu(P, d, w0, w1, edges, -e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])
    assert math.isfinite(L)


def test_tqu_gradient_reduces_to_temperature_without_polarisation_data():
    wl, P, d, w0, w1 = _problem(te=0.0, pol=False)
    edges = np.array([2, 5, 8, wl.lmax + 1])
    g3, _ = grad.grad_lnpi_tqu(P, d, w0, w1, edges)
    PT = cr.Problem(P.nside, P.lmax, P.cl[0], P.bl, P.ninv_t, 2)
    gT, _ = grad.grad_lnpi(PT, d[0], w0[0], w1[0], edges)
    assert np.allclose(g3, gT, rtol=1e-9, atol=1e-9 * np.max(np.abs(gT)))
    # with polarisation data the gradient differs (control)
    wl, P2, d2, w02, w12 = _problem(te=0.0, pol=True)
    g3p, _ = grad.grad_lnpi_tqu(P2, d, w0, w1, edges)
    assert not np.allclose(g3p, gT, rtol=1e-3)


def test_planted_dropped_term_fails_differences():
    wl, P, d, w0, w1 = _problem(seed=5)
    edges = np.array([2, 6, wl.lmax + 1])
    g, _ = grad.grad_lnpi_tqu(P, d, w0, w1, edges)
    # the S^-1/2 w0 term alone (what dropping it would remove)
    from oracle.cr_tqu import CROperatorTQU
    op = CROperatorTQU(P)
    fhat, _ = cr.pcg(op, op.rhs(w0=w0, w1=w1), 1e-12)
    lam, _ = cr.pcg(op, op.apply_data_term(fhat), 1e-12)
    masks = grad.bin_masks(op.ls, edges)
    t2 = np.array([0.5 * op.dot(lam, mk[None, :] * op._block(op.sinvh_lm, op.project(w0))) for mk in masks])
    h = 1e-4
    fd = np.array([(grad.lnpi_at_tqu(P, d, w0, w1, edges, h * np.eye(2)[k]) -
                    grad.lnpi_at_tqu(P, d, w0, w1, edges, -h * np.eye(2)[k])) / (2 * h) for k in range(2)])
    assert np.all(np.abs(fd - g) <= 1e-6 * np.maximum(1.0, np.abs(g)))
    assert np.any(np.abs(fd - (g - t2)) > 1e-4 * np.maximum(1.0, np.abs(g)))
