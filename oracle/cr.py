"""Constrained-realization operator, right-hand side and PCG.

Paper, Sect. 2.2.1: completing the square in the joint posterior gives the
precision S^-1 + B^T N^-1 B of the sky amplitudes; the mean field
(eq. mean-field-map), the constrained realization (eq. mapmakingeq) and the
fluctuation map (eq. fluc-map) all solve systems with that matrix, by
conjugate gradients (Shewchuk 1994) with a diagonal preconditioner (Sect. 4).

Readings used here:
* the paper's B (beam + projection to pixels) is Y diag(b_l);
* S = diag(C_l); modes with l < lmin (C_l = 0) are fixed to zero, i.e. the
  system is solved on the l >= lmin subspace; Im a_l0 is identically zero;
* the Jacobi diagonal is D_lm = 1/C_l + b_l^2 sum_r lambda_lm(z_r)^2 W_r with
  W_r the ring sum of N^-1: the mean of the Re and Im diagonal entries of
  B Y^T N^-1 Y B;
* PCG starts from x0 = 0 and stops when the relative residual
  ||r|| / ||b|| (real-field norm) is at most tol; the recursively updated
  residual is replaced by the true residual b - A x every 50 iterations
  (the search direction is kept), and confirmed against it before stopping
  (if it fails, the iteration restarts from the true residual).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .sht import SHT, lm_arrays, dot


@dataclass
class Problem:
    nside: int
    lmax: int
    cl: np.ndarray       # C_l, length lmax+1
    bl: np.ndarray       # b_l, length lmax+1
    ninv: np.ndarray     # N^-1 per pixel, 0 = masked
    lmin: int = 2


class CROperator:
    def __init__(self, prob: Problem, sht: SHT | None = None):
        self.p = prob
        self.sht = sht if sht is not None else SHT(prob.nside, prob.lmax)
        ls, ms = lm_arrays(prob.lmax, self.sht.mmax)
        self.ls, self.msel = ls, ms
        self.keep = (ls >= prob.lmin).astype(np.float64)
        cl = np.where(ls >= prob.lmin, prob.cl[ls], 1.0)
        self.sinv = self.keep / cl
        self.sinvhalf = self.keep / np.sqrt(cl)
        self.shalf = self.keep * np.sqrt(cl)
        self.b = prob.bl[ls]

    def project(self, a: np.ndarray) -> np.ndarray:
        out = a * self.keep
        m0 = self.msel == 0
        out[m0] = out[m0].real
        return out

    def dot(self, a, c) -> float:
        return dot(a, c, self.p.lmax, self.sht.mmax)

    def norm(self, a) -> float:
        return math.sqrt(max(self.dot(a, a), 0.0))

    # A x = S^-1 x + B Y^T N^-1 Y B x
    def apply(self, x: np.ndarray) -> np.ndarray:
        x = self.project(x)
        m = self.sht.synth(self.b * x)
        y = self.b * self.sht.adjoint(self.p.ninv * m)
        return self.project(self.sinv * x + y)

    def apply_data_term(self, x: np.ndarray) -> np.ndarray:
        """M x = B Y^T N^-1 Y B x."""
        x = self.project(x)
        return self.project(self.b * self.sht.adjoint(self.p.ninv * self.sht.synth(self.b * x)))

    def rhs(self, d=None, w0=None, w1=None) -> np.ndarray:
        """B Y^T N^-1 d + S^-1/2 w0 + B Y^T N^-1/2 w1 (terms with None omitted)."""
        u = np.zeros(self.sht.npix)
        if d is not None:
            u = u + self.p.ninv * d
        if w1 is not None:
            u = u + np.sqrt(self.p.ninv) * w1
        out = np.zeros(self.sht.nalm, dtype=np.complex128)
        if d is not None or w1 is not None:
            out = self.b * self.sht.adjoint(u)
        if w0 is not None:
            out = out + self.sinvhalf * w0
        return self.project(out)

    def diag(self) -> np.ndarray:
        W = self.sht.ring_weights(self.p.ninv)
        G = np.broadcast_to(W[None, :], (self.sht.mmax + 1, W.size)).astype(np.complex128)
        lam2 = self.sht.legendre_adjoint(G, square=True).real
        return np.where(self.keep > 0, self.sinv + self.b ** 2 * lam2, 1.0)


@dataclass
class PCGInfo:
    iters: int
    rel_resid_true: float
    converged: bool
    history: list


def pcg(op, b: np.ndarray, tol: float, maxiter: int = 10000, precond=None,
        x0: np.ndarray | None = None, replace_every: int = 50) -> tuple[np.ndarray, PCGInfo]:
    """Preconditioned conjugate gradients in the real-field inner product.
    precond: None (Jacobi diagonal of op), an array D (z = r / D) or a
    callable r -> z (symmetric positive definite). Every replace_every
    iterations r is replaced by the true residual b - A x."""
    if callable(precond):
        apply_pc = precond
    else:
        D = op.diag() if precond is None else precond
        apply_pc = lambda r: r / D
    bnorm = op.norm(b)
    x = np.zeros_like(b) if x0 is None else op.project(np.array(x0, dtype=np.complex128))
    if bnorm == 0.0:
        return np.zeros_like(b), PCGInfo(0, 0.0, True, [])
    r = b - op.apply(x) if x0 is not None else b.copy()
    z = op.project(apply_pc(r))
    p = z.copy()
    rz = op.dot(r, z)
    hist = []
    it = 0
    while it < maxiter:
        q = op.apply(p)
        alpha = rz / op.dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        if replace_every and it % replace_every == 0:
            r = b - op.apply(x)
        rel = op.norm(r) / bnorm
        hist.append(rel)
        if rel <= tol:
            rt = b - op.apply(x)
            if op.norm(rt) / bnorm <= tol:
                break
            r = rt
            z = op.project(apply_pc(r))
            p = z.copy()
            rz = op.dot(r, z)
            continue
        z = op.project(apply_pc(r))
        rz_new = op.dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    rel_true = op.norm(b - op.apply(x)) / bnorm
    return x, PCGInfo(it, rel_true, rel_true <= tol, hist)


class HarmonicDiagonalOperator:
    """The full-sky uniform-noise model of the paper (eqs. exact_harm,
    hat_s_approx, hat_f_approx): Y^T N^-1 Y replaced by N_l^-1 I with
    N_l = 4 pi sigma^2 / Npix (App. A, full-sky limit)."""

    def __init__(self, lmax: int, cl: np.ndarray, bl: np.ndarray, nl: float, lmin: int = 2):
        self.lmax, self.mmax = lmax, lmax
        ls, ms = lm_arrays(lmax, lmax)
        self.ls, self.msel = ls, ms
        self.keep = (ls >= lmin).astype(np.float64)
        c = np.where(ls >= lmin, cl[ls], 1.0)
        self.C, self.b, self.nl = c, bl[ls], nl
        self.sinv = self.keep / c
        self.sinvhalf = self.keep / np.sqrt(c)

    def project(self, a):
        out = a * self.keep
        m0 = self.msel == 0
        out[m0] = out[m0].real
        return out

    def dot(self, a, c):
        return dot(a, c, self.lmax, self.mmax)

    def norm(self, a):
        return math.sqrt(self.dot(a, a))

    def apply(self, x):
        return self.project((1.0 / self.C + self.b ** 2 / self.nl) * x)

    def apply_data_term(self, x):
        """M x with M = B^T N^-1 B = b_l^2 / N_l."""
        return self.project(self.b ** 2 / self.nl * x)

    def diag(self):
        return np.where(self.keep > 0, 1.0 / self.C + self.b ** 2 / self.nl, 1.0)

    def rhs(self, r_lm=None, w0=None, w1_lm=None):
        out = np.zeros(self.ls.size, dtype=np.complex128)
        if r_lm is not None:
            out += self.b * r_lm / self.nl
        if w0 is not None:
            out += w0 / np.sqrt(self.C)
        if w1_lm is not None:
            out += self.b * w1_lm / np.sqrt(self.nl)
        return self.project(out)

    def closed_form_mean(self, r_lm):
        """eq. hat_s_approx."""
        return self.project(r_lm * self.b * self.C / (self.nl + self.b ** 2 * self.C))

    def closed_form_fluct(self, w0, w1_lm):
        """eq. hat_f_approx."""
        den = self.nl + self.b ** 2 * self.C
        return self.project(w0 * self.nl * np.sqrt(self.C) / den
                            + w1_lm * math.sqrt(self.nl) * self.b * self.C / den)
