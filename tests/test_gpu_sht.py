"""GPU parity of the HIP transforms (through the C ABI) against the oracle:
synthesis Y, its transpose Y^T and analysis, FP64 to 1e-10 (relative 2-norm)."""
import math

import numpy as np
import pytest
import torch

import crinputs as ci
from oracle import sht as osht
from tests.gpu_helpers import rel, tc

pytestmark = pytest.mark.gpu
TOL = 1e-10

def _mod():
    from paper_2306_15511_amd import crsht as m
    return m


CASES = [
    (1, 2, None), (1, 0, None), (2, 5, None), (4, 11, None), (4, 20, None),   # lmax > 3 nside - 1: aliasing
    (8, 23, None), (8, 23, 10), (16, 47, None), (32, 95, None), (32, 60, 33), (64, 191, None), (128, 383, None),
    (3, 8, None), (6, 17, None),                                               # nside not a power of two
]


@pytest.mark.parametrize("nside,lmax,mmax", CASES)
def test_synth_and_adjoint_match_oracle(nside, lmax, mmax):
    m = _mod()
    print("case", nside, lmax, mmax, flush=True)
    plan = m.Plan(nside, lmax, -1 if mmax is None else mmax, nrhs_max=2)
    S = osht.SHT(nside, lmax, mmax)
    rng = np.random.default_rng(nside * 1000 + lmax)
    a = ci.white_alm(rng, lmax, mmax)
    x = rng.standard_normal(S.npix)
    ref_map = S.synth(a)
    ref_alm = S.adjoint(x)
    got_map = m.synth(plan, tc(a)).cpu().numpy()
    got_alm = m.adjoint(plan, tc(x)).cpu().numpy()
    assert rel(got_map, ref_map) < TOL
    assert rel(got_alm, ref_alm) < TOL
    plan.close()


def test_batched_columns_match_single():
    m = _mod()
    nside, lmax = 16, 47
    plan = m.Plan(nside, lmax, nrhs_max=11)
    S = osht.SHT(nside, lmax)
    rng = np.random.default_rng(7)
    A = np.stack([ci.white_alm(rng, lmax) for _ in range(11)])   # 11 = 8 + 2 + 1 column passes
    X = rng.standard_normal((11, S.npix))
    gm = m.synth(plan, tc(A)).cpu().numpy()
    ga = m.adjoint(plan, tc(X)).cpu().numpy()
    for c in range(11):
        assert rel(gm[c], S.synth(A[c])) < TOL
        assert rel(ga[c], S.adjoint(X[c])) < TOL


def test_imaginary_part_of_m0_is_ignored():
    m = _mod()
    plan = m.Plan(8, 23)
    S = osht.SHT(8, 23)
    a = ci.white_alm(np.random.default_rng(1), 23)
    b = a.copy()
    b[:24] += 1j * 3.0
    assert rel(m.synth(plan, tc(b)).cpu().numpy(), S.synth(a)) < TOL
    out = m.adjoint(plan, tc(np.random.default_rng(2).standard_normal(S.npix))).cpu().numpy()
    assert np.all(out[:24].imag == 0.0)


@pytest.mark.parametrize("nside,lmax", [(16, 47), (64, 191)])
def test_analysis_matches_oracle(nside, lmax):
    m = _mod()
    plan = m.Plan(nside, lmax)
    S = osht.SHT(nside, lmax)
    x = np.random.default_rng(3).standard_normal(S.npix)
    for n_iter in (0, 2):
        got = m.analysis(plan, tc(x), n_iter).cpu().numpy()
        assert rel(got, S.analysis(x, n_iter)) < TOL


def test_nside256_full_parity():
    m = _mod()
    nside, lmax = 256, 767
    print("case nside256", flush=True)
    plan = m.Plan(nside, lmax)
    S = osht.SHT(nside, lmax)
    rng = np.random.default_rng(256)
    a = ci.white_alm(rng, lmax)
    x = rng.standard_normal(S.npix)
    assert rel(m.synth(plan, tc(a)).cpu().numpy(), S.synth(a)) < TOL
    assert rel(m.adjoint(plan, tc(x)).cpu().numpy(), S.adjoint(x)) < TOL


def test_nside512_sampled_rings_and_adjointness():
    # the benchmarked size: sampled rings against the oracle, adjointness exactly
    m = _mod()
    nside, lmax = 512, 1535
    print("case nside512", flush=True)
    plan = m.Plan(nside, lmax)
    S = osht.SHT(nside, lmax)
    rng = np.random.default_rng(512)
    a = ci.white_alm(rng, lmax)
    got = m.synth(plan, tc(a)).cpu().numpy()
    rings = [0, 1, 2, 37, 300, 510, 511, 512, 900, 1023, 1500, 2045, 2046]
    ref = osht.synth_rings(S, a, rings)
    R = S.rings
    for k in rings:
        f, n = int(R.first[k]), int(R.nphi[k])
        assert rel(got[f:f + n], ref[k]) < TOL, k
    y = rng.standard_normal(S.npix)
    ya = m.adjoint(plan, tc(y)).cpu().numpy()
    lhs = float(np.dot(got, y))
    rhs = osht.dot(a, ya, lmax, lmax)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(got) * np.linalg.norm(y)


def test_invalid_arguments():
    m = _mod()
    plan = m.Plan(4, 11, nrhs_max=1)
    a = torch.zeros(2 * plan.nalm, dtype=torch.complex128, device="cuda")
    with pytest.raises(m.CrshtError):
        m.synth(plan, a)                       # 2 columns > nrhs_max
    with pytest.raises(m.CrshtError):
        m.synth(plan, a[:plan.nalm], prec=7)   # unknown precision
    _ = math


def test_nside1024_adjoint_matrix_cores_two_pair_launches():
    # Nside 1024 has 2048 ring pairs: the FP64 matrix-core adjoint (two or
    # more columns) covers them in two launches, the second adding to the
    # first. Against the single-column vector kernel, column by column, and
    # adjointness with the synthesis of the same columns
    m = _mod()
    nside, lmax, n = 1024, 2047, 3
    print("case nside1024 adjoint, 3 columns", flush=True)
    plan = m.Plan(nside, lmax, nrhs_max=n)
    rng = np.random.default_rng(1025)
    npix = 12 * nside * nside
    y = torch.from_numpy(rng.standard_normal((n, npix))).to("cuda:0")
    got = m.adjoint(plan, y)
    for c in range(n):
        one = m.adjoint(plan, y[c:c + 1].contiguous())
        e = float(torch.linalg.vector_norm(got[c] - one[0]) / torch.linalg.vector_norm(one[0]))
        print("column", c, "matrix cores vs vector kernel", e, flush=True)
        assert e < 1e-12
    a = np.stack([ci.white_alm(rng, lmax) for _ in range(n)])
    ls, ms = ci.alm_lm_arrays(lmax)
    w = torch.from_numpy(np.where(ms == 0, 1.0, 2.0)).to("cuda:0")
    da = tc(a)
    sx = m.synth(plan, da)
    for c in range(n):
        lhs = float(torch.sum(sx[c] * y[c]))
        rhs = float(torch.sum(w * (da[c].real * got[c].real + da[c].imag * got[c].imag)))
        assert abs(lhs - rhs) <= 1e-12 * float(torch.linalg.vector_norm(sx[c])) * float(torch.linalg.vector_norm(y[c]))
