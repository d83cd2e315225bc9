"""GPU checks of the gradients: the synthesis gradient (autograd backward),
grad chi^2 with respect to a_lm and d ln pi / d theta for binned C_l by the
adjoint solve, against the oracle (oracle/grad.py) and central finite
differences, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import crinputs as ci
from oracle import grad as ograd, sht as osht
from tests.gpu_helpers import masked_problem, real_rel, rel, tc

pytestmark = pytest.mark.gpu


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


def _gp(m, P):
    return m.Problem(P.cl, P.bl, tc(P.ninv), P.lmin)


def test_synth_grad_matches_oracle():
    m = _m()
    nside, lmax = 8, 23
    print("case synth_grad", nside, lmax, flush=True)
    plan = m.Plan(nside, lmax, nrhs_max=2)
    S = osht.SHT(nside, lmax)
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((2, S.npix))
    got = m.synth_grad(plan, tc(Y)).cpu().numpy()
    ms = osht.lm_arrays(lmax, lmax)[1]
    for c in range(2):
        ref = S.adjoint(Y[c]) * np.where(ms == 0, 1.0, 2.0)
        ref[ms == 0] = ref[ms == 0].real
        assert rel(got[c], ref) < 1e-10


def test_synth_autograd_gradcheck():
    m = _m()
    nside, lmax = 2, 5
    print("case gradcheck", flush=True)
    plan = m.Plan(nside, lmax)
    rng = np.random.default_rng(7)
    a = tc(ci.white_alm(rng, lmax)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: m.synth_ad(plan, x), (a,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_synth_autograd_loss_gradient():
    """d/da of L = sum_p w_p map_p^2 through the autograd wrapper equals the
    oracle's w_m Y^T (2 w map) (dot-product form of the adjoint)."""
    m = _m()
    nside, lmax = 16, 47
    plan = m.Plan(nside, lmax)
    S = osht.SHT(nside, lmax)
    rng = np.random.default_rng(9)
    a0 = ci.white_alm(rng, lmax)
    wpix = rng.uniform(0.5, 2.0, S.npix)
    a = tc(a0).requires_grad_(True)
    L = (tc(wpix) * m.synth_ad(plan, a) ** 2).sum()
    L.backward()
    ms = osht.lm_arrays(lmax, lmax)[1]
    ref = S.adjoint(2.0 * wpix * S.synth(a0)) * np.where(ms == 0, 1.0, 2.0)
    ref[ms == 0] = ref[ms == 0].real
    assert rel(a.grad.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("nside", [8, 16])
def test_grad_chi2_matches_oracle(nside):
    m = _m()
    print("case grad_chi2", nside, flush=True)
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax, nrhs_max=2)
    rng = np.random.default_rng(nside)
    A = np.stack([op.project(30.0 * ci.white_alm(rng, wl.lmax)) for _ in range(2)])
    D = np.stack([d, d + rng.standard_normal(d.size)])
    g, chi2 = m.grad_chi2(plan, _gp(m, P), tc(D), tc(A))
    g = g.cpu().numpy()
    for c in range(2):
        assert real_rel(op, g[c], ograd.grad_chi2(op, D[c], A[c])) < 1e-10
        assert abs(chi2[c] - ograd.chi2(op, D[c], A[c])) <= 1e-11 * ograd.chi2(op, D[c], A[c])


def _lnpi_inputs(nside, seed=4):
    wl, P, op, d = masked_problem(nside, fwhm_arcmin=60.0 * 64 / nside)
    rng = np.random.default_rng(seed)
    w0 = ci.white_alm(rng, wl.lmax)
    w1 = rng.standard_normal(op.sht.npix)
    return wl, P, op, d, w0, w1


def test_grad_lnpi_matches_oracle():
    m = _m()
    nside = 8
    print("case grad_lnpi oracle", nside, flush=True)
    wl, P, op, d, w0, w1 = _lnpi_inputs(nside)
    edges = ograd.bin_edges(wl.lmax)
    plan = m.Plan(nside, wl.lmax)
    g, L, st = m.grad_lnpi(plan, _gp(m, P), tc(d), tc(w0), tc(w1), edges, tol=1e-13)
    assert all(s.status == 0 for s in st)
    gr, Lr = ograd.grad_lnpi(P, d, w0, w1, edges, tol=1e-13)
    print("max |g - g_oracle| / max|g| = %.3e" % (np.max(np.abs(g - gr)) / np.max(np.abs(gr))), flush=True)
    assert np.all(np.abs(g - gr) <= 1e-7 * np.maximum(1.0, np.abs(gr)))
    assert abs(L - Lr) <= 1e-10 * abs(Lr)


def test_grad_lnpi_central_differences_nside32():
    m = _m()
    nside = 32
    print("case grad_lnpi fd", nside, flush=True)
    wl, P, op, d, w0, w1 = _lnpi_inputs(nside)
    edges = ograd.bin_edges(wl.lmax)
    plan = m.Plan(nside, wl.lmax)
    dd, ww0, ww1 = tc(d), tc(w0), tc(w1)
    g, L, _ = m.grad_lnpi(plan, _gp(m, P), dd, ww0, ww1, edges, tol=1e-13)
    h = 1e-4
    for k in (0, 6, 13, 19):
        vals = []
        for sgn in (1, -1):
            cl = P.cl.copy()
            cl[edges[k]:edges[k + 1]] *= math.exp(sgn * h)
            _, Lk, _ = m.grad_lnpi(plan, m.Problem(cl, P.bl, tc(P.ninv), P.lmin), dd, ww0, ww1, edges, tol=1e-13)
            vals.append(Lk)
        fd = (vals[0] - vals[1]) / (2 * h)
        print("bin %d: fd %.8e adjoint %.8e" % (k, fd, g[k]), flush=True)
        assert abs(fd - g[k]) <= 2e-5 * max(1.0, abs(fd))


def test_grad_lnpi_mixed_precision_error_stated():
    """The mixed-precision solves (bf16x3 operator, FP64 refinement to 1e-10)
    give the gradient to within the stated bound of the FP64 one."""
    m = _m()
    nside = 32
    wl, P, op, d, w0, w1 = _lnpi_inputs(nside, seed=8)
    edges = ograd.bin_edges(wl.lmax)
    plan = m.Plan(nside, wl.lmax)
    args = (plan, _gp(m, P), tc(d), tc(w0), tc(w1), edges)
    g64, L64, _ = m.grad_lnpi(*args, tol=1e-10)
    gmx, Lmx, st = m.grad_lnpi(*args, tol=1e-10, prec=m.CR_MIXED)
    err = np.max(np.abs(gmx - g64) / np.maximum(1.0, np.abs(g64)))
    print("mixed vs FP64 gradient: max rel err %.3e, ln pi rel err %.3e" % (err, abs(Lmx - L64) / abs(L64)),
          flush=True)
    assert all(s.status == 0 for s in st)
    assert err < 1e-6
    assert abs(Lmx - L64) <= 1e-8 * abs(L64)


def test_gradient_invalid_arguments():
    m = _m()
    wl, P, op, d = masked_problem(4)
    plan = m.Plan(4, wl.lmax)
    gp = _gp(m, P)
    with pytest.raises(m.CrshtError):
        m.grad_lnpi(plan, gp, tc(d), None, None, [5, 3, 8])          # not increasing
    with pytest.raises(m.CrshtError):
        m.grad_lnpi(plan, gp, tc(d), None, None, [2, wl.lmax + 5])   # past lmax + 1
