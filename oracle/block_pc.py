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
T+Q+U blocks: the T-T, E-E and B-B (l m, l' m) entries of the T+Q+U operator
for ring-constant z-symmetric noise on equatorial rings (no aliasing there);
symmetry, positivity and a several-fold cut in PCG iterations on a masked sky.
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
        if getattr(sht, "fast", False):
            # the same lambda_lm from the plain-C recurrence, one m at a time
            from .clegendre import lambda_m
            lam = [lambda_m(lmax, m, R.z, R.sin_theta) for m in range(mmax + 1)]
        else:
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


class BlockPreconditionerTQU:
    """Per-m blocks for T+Q+U systems (oracle/cr_tqu.py), one set per
    component: T as in BlockPreconditioner with N_T^-1; E and B with the
    spin-2 functions of oracle/spin2.py and N_P^-1,

        M_m^E[l, l'] = (S^-1)_EE,l delta_ll' + b_l b_l' sum_r (W_lm W_l'm + X_lm X_l'm)(z_r) Wp_r,

    (B likewise with (S^-1)_BB), Wp_r the ring sums of N_P^-1 averaged over
    mirror rings. For a noise model that depends on latitude only these are
    the E-E and B-B m-blocks of the operator; the couplings left out are T-E
    through the prior and E-B through the mask (terms W_l X_l', l - l' odd),
    so the preconditioner is block diagonal in (T, E, B) and SPD."""

    def __init__(self, op):
        from .spin2 import wx_rows
        sht = op.sht
        R = sht.rings
        mirror = R.nrings - 1 - np.arange(R.nrings)
        def sym(w):
            return 0.5 * (w + w[mirror])
        Wt = sym(sht.ring_weights(op.p.ninv_t))
        Wp = sym(sht.ring_weights(op.p.ninv_p))
        lmax, mmax = op.p.lmax, sht.mmax
        ls, ms = lm_arrays(lmax, mmax)
        self.idx = [np.flatnonzero(ms == m) for m in range(mmax + 1)]
        lam = [np.zeros((lmax - m + 1, R.nrings)) for m in range(mmax + 1)]
        Wf = [np.zeros((lmax - m + 1, R.nrings)) for m in range(mmax + 1)]
        Xf = [np.zeros((lmax - m + 1, R.nrings)) for m in range(mmax + 1)]
        for l, row in lambda_rows(lmax, mmax, R.z, R.sin_theta):
            for m in range(row.shape[0]):
                lam[m][l - m] = row[m]
        for l, W, X in wx_rows(lmax, mmax, R.z, R.sin_theta):
            for m in range(W.shape[0]):
                Wf[m][l - m] = W[m]
                Xf[m][l - m] = X[m]
        keep = op.keep
        self.inv = []
        for m in range(mmax + 1):
            ii = self.idx[m]
            b = op.b[ii][:, None]
            kp = keep[ii] > 0
            Lt = lam[m] * b
            Mt = (Lt * Wt[None, :]) @ Lt.T
            Lw, Lx = Wf[m] * b, Xf[m] * b
            Mp = (Lw * Wp[None, :]) @ Lw.T + (Lx * Wp[None, :]) @ Lx.T
            blocks = []
            for k, M in ((0, Mt), (1, Mp.copy()), (2, Mp.copy())):
                M[~kp, :] = 0.0
                M[:, ~kp] = 0.0
                M[np.diag_indices_from(M)] += np.where(kp, op.sinv_lm[ii, k, k], 1.0)
                blocks.append(np.linalg.inv(M))
            self.inv.append(blocks)

    def __call__(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros_like(r)
        for m, ii in enumerate(self.idx):
            for k in range(3):
                z[k, ii] = self.inv[m][k] @ r[k, ii]
        return z
