"""Pins of the gradient oracle (oracle/grad.py) against finite differences,
an exact complex-step derivative of the harmonic-diagonal model's closed-form
ln pi, and the symmetry of the adjoint solve."""
import math

import numpy as np
import pytest

import crinputs as ci
from oracle import cr, grad, healpix
from oracle.joint import lnpi
from oracle.sht import lm_arrays


def _masked(nside, lmax, seed=3):
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=60.0 * 64 / nside, cfg=1)
    z, phi = healpix.pixel_coords(nside)
    P = cr.Problem(nside, lmax, wl.cl(), wl.bl(), wl.ninv(z, phi), 2)
    op = cr.CROperator(P)
    rng = np.random.default_rng(seed)
    a_true = wl.signal()
    d = op.sht.synth(op.b * a_true) + wl.sigma_map(z, phi) * rng.standard_normal(op.sht.npix)
    return wl, P, op, d, rng


def _real_dofs(op, rng, n):
    ls, ms = op.ls, op.msel
    cand = np.flatnonzero(ls >= 2)
    idx = rng.choice(cand, size=n, replace=False)
    out = []
    for i in idx:
        imag = ms[i] > 0 and rng.random() < 0.5
        out.append((int(i), bool(imag)))
    return out


def test_grad_chi2_central_differences():
    wl, P, op, d, rng = _masked(4, 11)
    a = op.project(ci.white_alm(rng, 11) * 30.0)
    g = grad.grad_chi2(op, d, a)
    for i, imag in _real_dofs(op, rng, 32):
        e = np.zeros_like(a)
        e[i] = 1j if imag else 1.0
        h = 1e-4 * max(abs(a[i]), 1.0)
        fd = (grad.chi2(op, d, a + h * e) - grad.chi2(op, d, a - h * e)) / (2 * h)
        w = 1.0 if op.msel[i] == 0 else 2.0
        an = w * (g[i].imag if imag else g[i].real)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (i, imag, fd, an)


def _harmonic(lmax=63, seed=11):
    rng = np.random.default_rng(seed)
    amp = ci.amplitude_for_rms(lmax)
    cl = ci.cl_powerlaw(lmax, amp)
    bl = ci.gaussian_beam(lmax, 40.0 * ci.ARCMIN)
    nl = 4 * math.pi * 10.0 ** 2 / (12 * 32 * 32)
    H = cr.HarmonicDiagonalOperator(lmax, cl, bl, nl)
    r = H.project(ci.white_alm(rng, lmax) * 20.0)
    w0 = H.project(ci.white_alm(rng, lmax))
    w1 = H.project(ci.white_alm(rng, lmax))
    return H, r, w0, w1


def _harmonic_lnpi(H, r, w0, w1, Cvals):
    vals = grad.harmonic_lnpi_modes(Cvals, H.b, H.nl, r, w0, w1)
    wm = np.where(H.msel == 0, 1.0, 2.0) * H.keep
    return vals * wm


def test_grad_lnpi_harmonic_model_complex_step():
    H, r, w0, w1 = _harmonic()
    edges = grad.bin_edges(H.lmax)
    ahat = H.closed_form_mean(r)
    fhat = H.closed_form_fluct(w0, w1)
    g, _ = grad.grad_lnpi_op(H, ahat, fhat, w0, edges, tol=1e-15)
    # exact derivative: d/dtheta_k sum_modes w_m lnpi_mode(C e^theta) = sum_{bin k} w_m C dlnpi/dC
    hstep = 1e-30
    dC = _harmonic_lnpi(H, r, w0, w1, H.C + 1j * hstep * H.C).imag / hstep   # = C d/dC per mode
    for k in range(edges.size - 1):
        sel = (H.ls >= edges[k]) & (H.ls < edges[k + 1])
        ref = float(np.sum(dC[sel]))
        assert abs(g[k] - ref) <= 1e-9 * max(1.0, abs(ref)), (k, g[k], ref)


def test_planted_gradient_mistake_is_caught():
    H, r, w0, w1 = _harmonic()
    edges = grad.bin_edges(H.lmax)
    ahat, fhat = H.closed_form_mean(r), H.closed_form_fluct(w0, w1)
    _, lam = grad.grad_lnpi_op(H, ahat, fhat, w0, edges, tol=1e-15)
    dC = _harmonic_lnpi(H, r, w0, w1, H.C + 1j * 1e-30 * H.C).imag / 1e-30
    worst = 0.0
    for k, mk in enumerate(grad.bin_masks(H.ls, edges)):
        t1 = H.dot(ahat, mk * H.sinv * ahat)
        t2 = H.dot(lam, mk * H.sinvhalf * w0)
        t3 = H.dot(lam, mk * H.sinv * fhat)
        wrong = 0.5 * t1 - 0.5 * t2 - t3          # sign of the w0 term flipped
        ref = float(np.sum(dC[(H.ls >= edges[k]) & (H.ls < edges[k + 1])]))
        worst = max(worst, abs(wrong - ref) / max(1.0, abs(ref)))
    assert worst > 1e-3


def test_grad_lnpi_pixel_central_differences():
    nside, lmax = 8, 23
    wl, P, op, d, rng = _masked(nside, lmax)
    w0 = ci.white_alm(rng, lmax)
    w1 = rng.standard_normal(op.sht.npix)
    edges = grad.bin_edges(lmax)
    theta = 0.05 * rng.standard_normal(edges.size - 1)
    g, L = grad.grad_lnpi(P, d, w0, w1, edges, theta, tol=1e-13)
    assert abs(L - grad.lnpi_at(P, d, w0, w1, edges, theta, tol=1e-13)) <= 1e-10 * abs(L)
    h = 1e-4
    for k in (0, 3, 7, 12, 19):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (grad.lnpi_at(P, d, w0, w1, edges, tp, tol=1e-13)
              - grad.lnpi_at(P, d, w0, w1, edges, tm, tol=1e-13)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * max(1.0, abs(fd)), (k, fd, g[k])


def test_adjoint_solve_symmetric():
    wl, P, op, d, rng = _masked(4, 11)
    u = op.project(ci.white_alm(rng, 11))
    v = op.project(ci.white_alm(rng, 11))
    Au, _ = cr.pcg(op, u, 1e-14)
    Av, _ = cr.pcg(op, v, 1e-14)
    assert abs(op.dot(Au, v) - op.dot(u, Av)) <= 1e-10 * abs(op.dot(Au, v))


def test_bin_edges():
    e = grad.bin_edges(1535)
    assert e[0] == 2 and e[-1] == 1536 and e.size == 21
    assert np.all(np.diff(e) >= 1)
    # floor(2 x 768^(k/20)) = 2, 2, 3, 5, 7, 10, 14, 20, ...; lifted to strictly increasing from e_0 = 2
    assert [int(x) for x in e[:12]] == [2, 3, 4, 5, 7, 10, 14, 20, 28, 39, 55, 77]
    assert [int(x) for x in grad.bin_edges(23)] == list(range(2, 22)) + [24]
