"""Temperature + polarisation constrained-realization operator (test
infrastructure).

The same system as oracle/cr.py (Sect. 2.2.1) for the sky vector
a = (a_T, a_E, a_B) with maps (T, Q, U):

    A = S^-1 + B Y^T N^-1 Y B,   b = B Y^T N^-1 d + S^-1/2 w0 + B Y^T N^-1/2 w1

where Y maps (a_T) to T by the scalar synthesis and (a_E, a_B) to (Q, U) by
the spin-2 synthesis of oracle/spin2.py; N^-1 is diagonal per pixel and
component (N_T^-1 for T, N_P^-1 for Q and U); B = diag(b_l) for all three;
S is block diagonal in l with the 3x3 blocks of the paper's C_l^i matrix
(Sect. 2.2.2: TT, TE, EE coupled, BB apart, EB = TB = 0). S^-1/2 is the
symmetric principal root of S^-1. Modes with l < lmin (= 2) are fixed to 0 in
all three components.

The Jacobi diagonal used with this operator: D_T = (S^-1)_TT + b_l^2
sum_r lambda_lm(z_r)^2 W_T,r and D_E = (S^-1)_EE + b_l^2 sum_r lambda_lm^2
W_P,r, D_B likewise with (S^-1)_BB, W_X,r the ring sums of N_X^-1 (the spin-0
functions stand in for the spin-2 ones in the polarisation entries: a
preconditioner only needs to be symmetric positive definite).

Vectors are complex arrays of shape (3, nalm); the inner product is the sum of
the three real-field products.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .sht import SHT, dot, lm_arrays
from .spin2 import PolSHT


@dataclass
class ProblemTQU:
    nside: int
    lmax: int
    cl: np.ndarray       # [4][lmax+1]: TT, EE, BB, TE
    bl: np.ndarray       # [lmax+1]
    ninv_t: np.ndarray   # [npix]
    ninv_p: np.ndarray   # [npix] (Q and U)
    lmin: int = 2


def spectra_blocks(cl: np.ndarray, lmax: int, lmin: int = 2):
    """Per-l S^-1 and S^-1/2 as arrays [lmax+1][3][3] (zero below lmin)."""
    sinv = np.zeros((lmax + 1, 3, 3))
    sinvh = np.zeros((lmax + 1, 3, 3))
    for l in range(lmin, lmax + 1):
        C = np.array([[cl[0][l], cl[3][l]], [cl[3][l], cl[1][l]]])
        ev, V = np.linalg.eigh(C)
        if np.any(ev <= 0) or cl[2][l] <= 0:
            raise ValueError("spectrum not positive definite at l = %d" % l)
        sinv[l, :2, :2] = (V / ev) @ V.T
        sinvh[l, :2, :2] = (V / np.sqrt(ev)) @ V.T
        sinv[l, 2, 2] = 1.0 / cl[2][l]
        sinvh[l, 2, 2] = 1.0 / math.sqrt(cl[2][l])
    return sinv, sinvh


class CROperatorTQU:
    def __init__(self, prob: ProblemTQU):
        self.p = prob
        self.sht = SHT(prob.nside, prob.lmax)
        self.pol = PolSHT(prob.nside, prob.lmax)
        ls, ms = lm_arrays(prob.lmax, self.sht.mmax)
        self.ls, self.msel = ls, ms
        self.keep = (ls >= prob.lmin).astype(np.float64)
        sinv, sinvh = spectra_blocks(prob.cl, prob.lmax, prob.lmin)
        self.sinv_lm = sinv[ls]        # [nalm][3][3]
        self.sinvh_lm = sinvh[ls]
        self.b = prob.bl[ls]

    def project(self, a: np.ndarray) -> np.ndarray:
        out = np.array(a, dtype=np.complex128) * self.keep[None, :]
        m0 = self.msel == 0
        out[:, m0] = out[:, m0].real
        return out

    def dot(self, a, c) -> float:
        return sum(dot(a[k], c[k], self.p.lmax, self.sht.mmax) for k in range(3))

    def norm(self, a) -> float:
        return math.sqrt(max(self.dot(a, a), 0.0))

    def _block(self, M, x):
        return np.einsum("nij,jn->in", M, x)

    def synth(self, x):
        T = self.sht.synth(x[0])
        Q, U = self.pol.synth(x[1], x[2])
        return np.stack([T, Q, U])

    def adjoint(self, m):
        aT = self.sht.adjoint(m[0])
        aE, aB = self.pol.adjoint(m[1], m[2])
        return np.stack([aT, aE, aB])

    def _ninv(self):
        return np.stack([self.p.ninv_t, self.p.ninv_p, self.p.ninv_p])

    def apply_data_term(self, x):
        x = self.project(x)
        return self.project(self.b * self.adjoint(self._ninv() * self.synth(self.b * x)))

    def apply(self, x):
        x = self.project(x)
        return self.project(self._block(self.sinv_lm, x)) + self.apply_data_term(x)

    def rhs(self, d=None, w0=None, w1=None):
        n = self._ninv()
        u = np.zeros((3, self.sht.npix))
        if d is not None:
            u = u + n * d
        if w1 is not None:
            u = u + np.sqrt(n) * w1
        out = np.zeros((3, self.sht.nalm), dtype=np.complex128)
        if d is not None or w1 is not None:
            out = self.b * self.adjoint(u)
        if w0 is not None:
            out = out + self._block(self.sinvh_lm, self.project(w0))
        return self.project(out)

    def diag(self):
        R = self.sht.rings
        out = np.ones((3, self.sht.nalm))
        for k, ninv in ((0, self.p.ninv_t), (1, self.p.ninv_p), (2, self.p.ninv_p)):
            W = self.sht.ring_weights(ninv)
            G = np.broadcast_to(W[None, :], (self.sht.mmax + 1, W.size)).astype(np.complex128)
            lam2 = self.sht.legendre_adjoint(G, square=True).real
            out[k] = np.where(self.keep > 0, self.sinv_lm[:, k, k] + self.b ** 2 * lam2, 1.0)
        return out
