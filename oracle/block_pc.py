"""Per-m block preconditioner of the constrained-realization system (test
infrastructure).

Appendix A of the paper: for a noise model that depends on latitude only
(a constant-latitude mask with ring-wise noise), N^-1 in harmonic space is
diagonal in m, so S^-1 + B Y^T N^-1 Y B splits into one dense (l, l') matrix
per m that can be inverted directly. For any other noise model the same
matrices, built from the azimuthal mean of N^-1 on each ring, are the
preconditioner named in Sect. 4 as the main lever on the cost of the solve:

    M_m[l, l'] = delta_ll' / C_l + b_l b_l' sum_r lambda_lm(z_r) lambda_l'm(z_r) W_r,

with W_r = ring sum of N^-1, averaged over each ring and its mirror ring
(z -> -z) so that, as for the paper's mask, the blocks couple only l - l'
even; for a noise model symmetric under z -> -z this is exactly the m-block
of the operator (the azimuthal sum of e^{i(m - m)phi} is the ring length).
Rows l < lmin are the identity. The preconditioner is z_m = M_m^-1 r_m,
applied to the real and imaginary parts alike (a real symmetric matrix per
m), so it is symmetric positive definite in the real-field inner product.

Pins (tests/test_oracle_block_pc.py): each block equals the (l m, l' m)
block of the dense operator built from SciPy's spherical harmonics for a
z-symmetric noise model with azimuthal structure; the block diagonal equals
the Jacobi diagonal for any noise; for a noise model constant on each ring
and z-symmetric, PCG with this preconditioner converges in a handful of
iterations (only aliasing between m and m + n_phi on the polar rings is
left out); the preconditioner is symmetric in the real-field inner product.
"""
from __future__ import annotations

import numpy as np

from .legendre import lambda_rows
from .sht import lm_arrays


class BlockPreconditioner:
    def __init__(self, op):
        sht = op.sht
        R = sht.rings
        W = sht.ring_weights(op.p.ninv)
        mirror = R.nrings - 1 - np.arange(R.nrings)
        Wbar = 0.5 * (W + W[mirror])
        lmax, mmax = op.p.lmax, sht.mmax
        self.lmax, self.mmax = lmax, mmax
        ls, ms = lm_arrays(lmax, mmax)
        self.idx = [np.flatnonzero(ms == m) for m in range(mmax + 1)]   # l = m .. lmax
        lam = [np.zeros((lmax - m + 1, R.nrings)) for m in range(mmax + 1)]
        for l, row in lambda_rows(lmax, mmax, R.z, R.sin_theta):
            for m in range(row.shape[0]):
                lam[m][l - m] = row[m]
        self.blocks = []
        self.inv = []
        for m in range(mmax + 1):
            ii = self.idx[m]
            L = lam[m] * op.b[ii][:, None]
            M = (L * Wbar[None, :]) @ L.T
            keep = op.keep[ii] > 0
            M[~keep, :] = 0.0
            M[:, ~keep] = 0.0
            M[np.diag_indices_from(M)] += np.where(keep, op.sinv[ii], 1.0)
            self.blocks.append(M)
            self.inv.append(np.linalg.inv(M))

    def __call__(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros_like(r)
        for m, ii in enumerate(self.idx):
            z[ii] = self.inv[m] @ r[ii]
        return z
