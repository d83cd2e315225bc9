"""Dense brute force: Y as an explicit matrix from SciPy's ``sph_harm_y``.

This is an implementation of Y independent of ``legendre``/``sht`` (SciPy
evaluates Y_lm itself), used to pin the ring-factored oracle and to solve the
constrained-realization system by Cholesky for small Nside.

Real coordinates. A real field with m >= 0 storage has the real degrees of
freedom u = (a_l0 ; Re a_lm, Im a_lm for m > 0). In them
(Y a)_p = sum u_l0 Y_l0(p) + sum [2 Re Y_lm(p) Re a_lm - 2 Im Y_lm(p) Im a_lm],
so Y is the matrix Yd with those columns. The harmonic inner product is
u^T W u with W = diag(1 for m = 0, 2 for m > 0), and the transpose of the
library's definition (Y^T x)_lm = sum_p x_p Y*_lm(p) is W^-1 Yd^T.

Constrained-realization system (paper eq. mapmakingeq, with the reading
S = diag(C_l), B = diag(b_l) and the paper's "B" = Y B):
(S^-1 + B Y^T N^-1 Y B) s = rhs  <=>  (W S^-1 + B Yd^T N^-1 Yd B) u_s = W u_rhs,
a symmetric positive definite system solved by Cholesky.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
from scipy.special import sph_harm_y

from . import healpix
from .sht import lm_arrays


class DenseY:
    def __init__(self, nside: int, lmax: int, lmin: int = 0):
        self.nside, self.lmax, self.lmin = nside, lmax, lmin
        z, phi = healpix.pixel_coords(nside)
        theta = np.arccos(np.clip(z, -1.0, 1.0))
        ls, ms = lm_arrays(lmax, lmax)
        self.ls, self.ms = ls, ms
        cols, wts, src = [], [], []   # src: (alm index, 0=re / 1=im)
        for i, (l, m) in enumerate(zip(ls, ms)):
            if l < lmin:
                continue
            y = sph_harm_y(int(l), int(m), theta, phi)
            if m == 0:
                cols.append(y.real); wts.append(1.0); src.append((i, 0))
            else:
                cols.append(2.0 * y.real); wts.append(2.0); src.append((i, 0))
                cols.append(-2.0 * y.imag); wts.append(2.0); src.append((i, 1))
        self.Y = np.stack(cols, axis=1)          # (npix, ndof)
        self.W = np.array(wts)
        self.src = src
        self.nalm = ls.size

    @property
    def ndof(self) -> int:
        return self.Y.shape[1]

    def to_real(self, alm: np.ndarray) -> np.ndarray:
        return np.array([alm[i].real if k == 0 else alm[i].imag for i, k in self.src])

    def from_real(self, u: np.ndarray) -> np.ndarray:
        out = np.zeros(self.nalm, dtype=np.complex128)
        for val, (i, k) in zip(u, self.src):
            if k == 0:
                out[i] += val
            else:
                out[i] += 1j * val
        return out

    def synth(self, alm: np.ndarray) -> np.ndarray:
        return self.Y @ self.to_real(alm)

    def adjoint(self, x: np.ndarray) -> np.ndarray:
        return self.from_real((self.Y.T @ x) / self.W)

    def _per_dof(self, per_l: np.ndarray) -> np.ndarray:
        return np.array([per_l[self.ls[i]] for i, _ in self.src])

    def cr_matrix(self, cl: np.ndarray, bl: np.ndarray, ninv: np.ndarray) -> np.ndarray:
        """W S^-1 + B Yd^T N^-1 Yd B (symmetric)."""
        bd = self._per_dof(bl)
        YB = self.Y * bd[None, :]
        M = YB.T @ (ninv[:, None] * YB)
        M[np.diag_indices_from(M)] += self.W / self._per_dof(cl)
        return M

    def cr_solve(self, cl, bl, ninv, rhs_alm: np.ndarray) -> np.ndarray:
        M = self.cr_matrix(cl, bl, ninv)
        u = scipy.linalg.cho_solve(scipy.linalg.cho_factor(M), self.W * self.to_real(rhs_alm))
        return self.from_real(u)
