"""Gradients of the constrained-realization problem (test infrastructure).

Two derivatives are needed around the joint sampler of the paper (Sect. 2.2):

* chi^2(a) = (d - Y B a)^T N^-1 (d - Y B a), the data term of the
  posterior (data model of Sect. 2.2): its gradient with respect to the sky
  amplitudes is g = -2 B Y^T N^-1 (d - Y B a). g is the gradient in the
  real-field inner product <a, c> = sum_l a_l0 c_l0 + 2 sum_{m>0} Re(a_lm c*_lm)
  (d chi^2 = <g, da>), on the modes kept by the problem (l >= lmin).

* L(theta) = ln pi(theta) (the pi(theta) expression after the acceptance
  rate, Eq. (25)-(26)) at fixed w0, w1, with the spectrum scaled per
  multipole bin, C_l(theta) = C_l^fid exp(theta_k) for l in bin k. With
  a^ the mean field, f^ the fluctuation and M = B Y^T N^-1 Y B:
  - the first two terms of ln pi are the maximum over a of a quadratic whose
    maximiser is a^ (completing the square), so only their explicit theta
    dependence counts: -1/2 a^T (dS^-1/dtheta_k) a^ = +1/2 a^T S^-1_k a^;
  - the last term -1/2 f^T M f^ depends on theta through f^ = A^-1 (S^-1/2 w0
    + B Y^T N^-1/2 w1): with one extra (adjoint) solve lambda = A^-1 M f^ its
    derivative is -lambda^T (dS^-1/2/dtheta_k w0 - dS^-1/dtheta_k f^)
    = +1/2 lambda^T S^-1/2_k w0 - lambda^T S^-1_k f^,
  where X_k is X restricted to the modes of bin k.

Bin edges (20 bins, logarithmic): e_0 = 2, e_k = max(e_{k-1} + 1,
floor(2 ((lmax + 1)/2)^(k/20))), e_20 = lmax + 1; bin k holds e_k <= l < e_{k+1}.

Pins (tests/test_oracle_grad.py): central finite differences of chi^2 and of
ln pi, an exact complex-step derivative of the closed-form ln pi of the
harmonic-diagonal model (Eqs. (19)-(20)), and the symmetry of the adjoint
solve.
"""
from __future__ import annotations

import math

import numpy as np

from .cr import CROperator, Problem, pcg
from .joint import lnpi


def bin_edges(lmax: int, nbins: int = 20, lmin: int = 2) -> np.ndarray:
    e = [lmin]
    for k in range(1, nbins):
        e.append(max(e[-1] + 1, int(math.floor(2.0 * ((lmax + 1) / 2.0) ** (k / nbins)))))
    e.append(lmax + 1)
    e = np.array(e, dtype=np.int64)
    if np.any(np.diff(e) <= 0):
        raise ValueError("lmax too small for %d bins" % nbins)
    return e


def bin_masks(ls: np.ndarray, edges: np.ndarray) -> list:
    return [((ls >= edges[k]) & (ls < edges[k + 1])).astype(np.float64) for k in range(edges.size - 1)]


def chi2(op: CROperator, d: np.ndarray, a: np.ndarray) -> float:
    res = d - op.sht.synth(op.b * op.project(a))
    return float(np.sum(op.p.ninv * res * res))


def grad_chi2(op: CROperator, d: np.ndarray, a: np.ndarray) -> np.ndarray:
    res = d - op.sht.synth(op.b * op.project(a))
    return op.project(-2.0 * op.b * op.sht.adjoint(op.p.ninv * res))


def scaled_problem(fid: Problem, edges: np.ndarray, theta: np.ndarray) -> Problem:
    cl = fid.cl.copy()
    for k in range(edges.size - 1):
        cl[edges[k]:edges[k + 1]] *= math.exp(theta[k])
    return Problem(fid.nside, fid.lmax, cl, fid.bl, fid.ninv, fid.lmin)


def grad_lnpi_op(op, ahat, fhat, w0, edges: np.ndarray, tol: float, maxiter: int = 20000):
    """dL/dtheta_k at theta (the spectrum of op) from the mean field, the
    fluctuation and one adjoint solve; returns (grad, lambda)."""
    lam, _ = pcg(op, op.apply_data_term(fhat), tol, maxiter)
    masks = bin_masks(op.ls, edges)
    w0p = op.project(w0)
    g = np.empty(len(masks))
    for k, mk in enumerate(masks):
        t1 = op.dot(ahat, mk * op.sinv * ahat)
        t2 = op.dot(lam, mk * op.sinvhalf * w0p)
        t3 = op.dot(lam, mk * op.sinv * fhat)
        g[k] = 0.5 * t1 + 0.5 * t2 - t3
    return g, lam


def grad_lnpi(fid: Problem, d, w0, w1, edges: np.ndarray, theta=None, tol: float = 1e-12,
              maxiter: int = 20000):
    """(dL/dtheta, L) at theta (default 0) for the pixel-space problem."""
    theta = np.zeros(edges.size - 1) if theta is None else np.asarray(theta, dtype=np.float64)
    op = CROperator(scaled_problem(fid, edges, theta))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    fhat, _ = pcg(op, op.rhs(w0=w0, w1=w1), tol, maxiter)
    g, _ = grad_lnpi_op(op, ahat, fhat, w0, edges, tol, maxiter)
    return g, lnpi(op, d, ahat, fhat)


def lnpi_at(fid: Problem, d, w0, w1, edges: np.ndarray, theta, tol: float = 1e-12, maxiter: int = 20000) -> float:
    op = CROperator(scaled_problem(fid, edges, np.asarray(theta, dtype=np.float64)))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    fhat, _ = pcg(op, op.rhs(w0=w0, w1=w1), tol, maxiter)
    return lnpi(op, d, ahat, fhat)


# --------------------------------------------------- harmonic-diagonal model
def harmonic_lnpi_modes(C, b, nl, r, w0, w1):
    """ln pi of the harmonic-diagonal model per stored mode (before the
    real-field weights), from the closed forms of the mean field and the
    fluctuation (Eqs. (19)-(20)); C may be complex (complex-step
    differentiation: the expression is written analytically in C)."""
    D = nl + b * b * C
    sq = np.sqrt(C)
    # chi^2 + prior of the mean field = |r|^2 / D
    mean = (r.real ** 2 + r.imag ** 2) / D
    # b^2 |f^|^2 / N with f^ = (w0 N sqrt C + w1 sqrt N b C) / D, expanded in C
    c0 = (w0.real ** 2 + w0.imag ** 2) * nl * nl * C
    c1 = 2.0 * (w0.real * w1.real + w0.imag * w1.imag) * nl * math.sqrt(nl) * b * C * sq
    c2 = (w1.real ** 2 + w1.imag ** 2) * nl * b * b * C * C
    fl = b * b * (c0 + c1 + c2) / (nl * D * D)
    return -0.5 * (mean + fl)


# ------------------------------------------------------------------- T+Q+U
# The same derivative for a sky (a_T, a_E, a_B) with the 3x3 spectrum blocks
# of Sect. 2.2.2 (oracle/cr_tqu.py), each block scaled as a whole per bin:
# C_l(theta) = C_l^fid exp(theta_k) for l in bin k, so S^-1 and S^-1/2 of the
# bin scale by exp(-theta_k) and exp(-theta_k / 2) and the three terms keep
# their form with the blocks: dL/dtheta_k = 1/2 a^T S^-1_k a + 1/2 lambda^T
# S^-1/2_k w0 - lambda^T S^-1_k f, lambda = A^-1 M f (one adjoint solve).
def scaled_problem_tqu(fid, edges: np.ndarray, theta: np.ndarray):
    from .cr_tqu import ProblemTQU
    cl = np.array(fid.cl, dtype=np.float64, copy=True)
    for k in range(edges.size - 1):
        cl[:, edges[k]:edges[k + 1]] *= math.exp(theta[k])
    return ProblemTQU(fid.nside, fid.lmax, cl, fid.bl, fid.ninv_t, fid.ninv_p, fid.lmin)


def grad_lnpi_tqu(fid, d, w0, w1, edges: np.ndarray, theta=None, tol: float = 1e-12, maxiter: int = 20000):
    """(dL/dtheta, L) at theta (default 0) for a T+Q+U problem (ProblemTQU);
    d, w1 maps [3][npix], w0 [3][nalm]."""
    from .cr_tqu import CROperatorTQU
    from .joint import lnpi_tqu
    theta = np.zeros(edges.size - 1) if theta is None else np.asarray(theta, dtype=np.float64)
    op = CROperatorTQU(scaled_problem_tqu(fid, edges, theta))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    fhat, _ = pcg(op, op.rhs(w0=w0, w1=w1), tol, maxiter)
    lam, _ = pcg(op, op.apply_data_term(fhat), tol, maxiter)
    w0p = op.project(w0)
    masks = bin_masks(op.ls, edges)
    g = np.empty(len(masks))
    for k, mk in enumerate(masks):
        t1 = op.dot(ahat, mk[None, :] * op._block(op.sinv_lm, ahat))
        t2 = op.dot(lam, mk[None, :] * op._block(op.sinvh_lm, w0p))
        t3 = op.dot(lam, mk[None, :] * op._block(op.sinv_lm, fhat))
        g[k] = 0.5 * t1 + 0.5 * t2 - t3
    return g, lnpi_tqu(op, d, ahat, fhat)


def lnpi_at_tqu(fid, d, w0, w1, edges: np.ndarray, theta, tol: float = 1e-12, maxiter: int = 20000) -> float:
    from .cr_tqu import CROperatorTQU
    from .joint import lnpi_tqu
    op = CROperatorTQU(scaled_problem_tqu(fid, edges, np.asarray(theta, dtype=np.float64)))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    fhat, _ = pcg(op, op.rhs(w0=w0, w1=w1), tol, maxiter)
    return lnpi_tqu(op, d, ahat, fhat)
