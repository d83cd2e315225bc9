"""Pins of the per-m block preconditioner of the oracle (oracle/block_pc.py):
its blocks against the dense operator built from SciPy's spherical harmonics,
its diagonal against the Jacobi diagonal, symmetry in the real-field inner
product, and its effect on PCG."""
import math

import numpy as np
import pytest

import crinputs as ci
from oracle import cr, dense, healpix
from oracle.block_pc import BlockPreconditioner
from oracle.sht import lm_arrays


def _problem(nside, ninv_fn, lmax=None):
    lmax = 3 * nside - 1 if lmax is None else lmax
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=60.0 * 64 / nside, cfg=1)
    z, phi = healpix.pixel_coords(nside)
    P = cr.Problem(nside, lmax, wl.cl(), wl.bl(), ninv_fn(z, phi))
    return wl, P, cr.CROperator(P)


def _sym_noise(z, phi):
    # symmetric under z -> -z, with azimuthal structure and a band mask
    return (np.abs(z) > 0.2) * (1.0 + 0.6 * np.cos(phi) + 0.3 * np.sin(3 * phi) + z * z) / 50.0


def test_blocks_equal_dense_operator_m_blocks():
    nside, lmax = 8, 23
    wl, P, op = _problem(nside, _sym_noise, lmax)
    pc = BlockPreconditioner(op)
    D = dense.DenseY(nside, lmax, lmin=0)
    cl = np.where(np.arange(lmax + 1) >= 2, P.cl, 1.0)      # dense S^-1 on all l; compare l >= 2 rows
    Md = D.cr_matrix(cl, P.bl, P.ninv)
    pos = {key: k for k, key in enumerate(D.src)}
    ls, ms = lm_arrays(lmax, lmax)
    for m in (0, 1, 2, 5, 11, 23):
        ii = pc.idx[m]
        keep = ls[ii] >= 2
        sub = np.ix_(keep, keep)
        re = [pos[(i, 0)] for i in ii[keep]]
        blk = Md[np.ix_(re, re)]
        if m > 0:
            im = [pos[(i, 1)] for i in ii[keep]]
            blk = 0.5 * (blk + Md[np.ix_(im, im)]) / 2.0
        assert np.allclose(pc.blocks[m][sub], blk, rtol=1e-10, atol=1e-12 * np.abs(blk).max()), m


def test_block_diagonal_is_the_jacobi_diagonal():
    # any noise (not z-symmetric): the diagonal only sees lambda^2
    wl, P, op = _problem(8, lambda z, phi: (1.0 + 0.5 * z + 0.4 * np.cos(2 * phi)) / 30.0)
    pc = BlockPreconditioner(op)
    D = op.diag()
    for m, ii in enumerate(pc.idx):
        assert np.allclose(np.diag(pc.blocks[m]), D[ii], rtol=1e-12)


def test_symmetric_in_real_field_product():
    wl, P, op = _problem(8, _sym_noise)
    pc = BlockPreconditioner(op)
    rng = np.random.default_rng(3)
    x = op.project(ci.white_alm(rng, P.lmax))
    y = op.project(ci.white_alm(rng, P.lmax))
    a, b = op.dot(pc(x), y), op.dot(x, pc(y))
    assert abs(a - b) <= 1e-12 * abs(a)
    assert op.dot(pc(x), x) > 0


def test_pcg_with_block_preconditioner():
    nside = 16
    wl, P, op = _problem(nside, lambda z, phi: wl_ninv(z, phi, nside))
    pc = BlockPreconditioner(op)
    z, phi = healpix.pixel_coords(nside)
    d = op.sht.synth(op.b * wl.signal()) + wl.noise(z, phi)
    b = op.rhs(d, wl.w0(), wl.w1())
    xj, ij = cr.pcg(op, b, 1e-10, 5000)
    xb, ib = cr.pcg(op, b, 1e-10, 5000, precond=pc)
    assert ij.converged and ib.converged
    assert ib.iters < 30 < ij.iters
    assert op.norm(xb - xj) <= 1e-7 * op.norm(xj)


def wl_ninv(z, phi, nside):
    wl = ci.workload_masked_t(nside, 3 * nside - 1, cfg=1)
    return wl.ninv(z, phi)


def test_tqu_blocks_equal_operator_entries():
    # noise constant on rings, symmetric under z -> -z and zero on the polar
    # cap rings (equatorial rings hold 4 nside pixels, so no m <= lmax aliases
    # there): the T-T, E-E and B-B (l m, l' m) entries of the T+Q+U operator
    # are exactly the blocks
    from oracle import cr_tqu
    from oracle.block_pc import BlockPreconditionerTQU
    nside, lmax = 8, 23
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=480.0, cfg=2)
    z, phi = healpix.pixel_coords(nside)
    nt = (np.abs(z) < 0.6) * (1.0 + z * z) / 40.0
    P = cr_tqu.ProblemTQU(nside, lmax, ci.cl_tqu(lmax, wl.amp, 0.3), wl.bl(), nt, 0.5 * nt)
    op = cr_tqu.CROperatorTQU(P)
    pc = BlockPreconditionerTQU(op)
    ls, ms = lm_arrays(lmax, lmax)
    for m in (0, 1, 3, 8):
        ii = pc.idx[m]
        blocks = [np.linalg.inv(pc.inv[m][k]) for k in range(3)]
        for jl in (2, 5, 11):
            col = jl - m
            if col < 0 or ls[ii[col]] < 2:
                continue
            for k in range(3):
                x = np.zeros((3, ls.size), dtype=np.complex128)
                x[k, ii[col]] = 1.0
                y = op.apply(x)
                got = y[k, ii].real
                ref = blocks[k][:, col]
                keep = ls[ii] >= 2
                assert np.allclose(got[keep], ref[keep], rtol=1e-10, atol=1e-12 * np.abs(ref).max()), (m, jl, k)


def test_tqu_block_pc_symmetric_and_cuts_iterations():
    from oracle import cr_tqu
    from oracle.block_pc import BlockPreconditionerTQU
    nside = 8
    lmax = 3 * nside - 1
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=480.0, cfg=2)
    z, phi = healpix.pixel_coords(nside)
    nt = wl.ninv(z, phi)
    P = cr_tqu.ProblemTQU(nside, lmax, ci.cl_tqu(lmax, wl.amp, 0.3), wl.bl(), nt, 0.5 * nt)
    op = cr_tqu.CROperatorTQU(P)
    pc = BlockPreconditionerTQU(op)
    rng = np.random.default_rng(4)
    x = op.project(np.stack([ci.white_alm(rng, lmax) for _ in range(3)]))
    y = op.project(np.stack([ci.white_alm(rng, lmax) for _ in range(3)]))
    a, c = op.dot(pc(x), y), op.dot(x, pc(y))
    assert abs(a - c) <= 1e-10 * abs(a)
    assert op.dot(pc(x), x) > 0
    d = 30.0 * rng.standard_normal((3, op.sht.npix))
    w0 = np.stack([ci.white_alm(rng, lmax) for _ in range(3)])
    b = op.rhs(d, w0, rng.standard_normal((3, op.sht.npix)))
    xj, sj = cr.pcg(op, b, 1e-8, 5000)
    xb, sb = cr.pcg(op, b, 1e-8, 5000, precond=pc)
    assert sb.converged and sj.converged
    assert sb.iters * 4 < sj.iters, (sb.iters, sj.iters)
    assert op.norm(xb - xj) <= 1e-6 * op.norm(xj)
