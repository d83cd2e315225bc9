"""GPU checks of the batched driver cr_solve_batched: independent problems of
different Nside, amplitude, white-noise level and band mask (the recipe of
the 64-problem batched workload, at sizes the oracle solves quickly) against
single device-driven solves of the same problems (cr_solve_async: identical
results and iteration counts), against cr_solve in mixed precision (the same
refinement decisions, taken on the host there), and against the oracle."""
import math

import numpy as np
import pytest
import torch

import crinputs as ci
from oracle import cr, healpix
from tests.gpu_helpers import real_rel, tc

pytestmark = pytest.mark.gpu


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


def _problem(j, nside):
    """Problem j of the batched recipe at a small Nside: amplitude U[0.5, 2] A,
    white sigma U[5, 50] uK, band mask of sky fraction f ~ U[0, 0.3]."""
    lmax = 3 * nside - 1
    r = ci.rng_for(3, j, ci.STREAM_PARAMS)
    qa, sig, f = r.uniform(0.5, 2.0), r.uniform(5.0, 50.0), r.uniform(0.0, 0.3)
    wl = ci.Workload("small_batched_%02d" % j, nside, lmax, cfg=3, prob=j, amp=qa * ci.amplitude_for_rms(lmax),
                     fwhm_rad=30.0 * ci.ARCMIN * 256.0 / nside, sigma_uk=sig, mask_sin_b=f, tol=1e-6)
    z, phi = healpix.pixel_coords(nside)
    P = cr.Problem(nside, lmax, wl.cl(), wl.bl(), wl.ninv(z, phi))
    op = cr.CROperator(P)
    d = op.sht.synth(op.b * wl.signal()) + wl.noise(z, phi)
    return wl, P, op, d, wl.w0(), wl.w1()


NSIDES = [4, 8, 16, 32, 4, 8, 16, 32, 6]


def test_batched_matches_single_and_oracle():
    m = _m()
    print("case batched fp64", flush=True)
    cases = [_problem(j, ns) for j, ns in enumerate(NSIDES)]
    plans = [m.Plan(ns, 3 * ns - 1) for ns in NSIDES]
    probs = [m.Problem(P.cl, P.bl, tc(P.ninv), 2) for (_, P, _, _, _, _) in cases]
    D = [tc(c[3]) for c in cases]
    W0 = [tc(c[4]) for c in cases]
    W1 = [tc(c[5]) for c in cases]
    out, st = m.solve_batched(plans, probs, D, W0, W1, tol=1e-10)
    for j, (wl, P, op, d, w0, w1) in enumerate(cases):
        assert st[j].status == 0 and st[j].rel_resid_true <= 1e-10, (j, st[j])
        single, sd = m.solve_async(plans[j], probs[j], D[j], W0[j], W1[j], tol=1e-10, maxiter=20000,
                                   check_every=16)
        torch.cuda.synchronize()
        st1 = m.decode_stats(sd, 1)
        assert np.array_equal(out[j].cpu().numpy(), single.cpu().numpy()[0]), j
        assert st1[0].iters == st[j].iters
        ref, _ = cr.pcg(op, op.rhs(d=d, w0=w0, w1=w1), 1e-12)
        assert real_rel(op, out[j].cpu().numpy(), ref) < 1e-7, j
        b = op.rhs(d=d, w0=w0, w1=w1)
        assert op.norm(b - op.apply(out[j].cpu().numpy())) / op.norm(b) <= 1.5e-10, j


def test_batched_mixed_precision_and_missing_terms():
    m = _m()
    print("case batched mixed", flush=True)
    ns = [8, 16, 32, 64]
    cases = [_problem(20 + j, n) for j, n in enumerate(ns)]
    plans = [m.Plan(n, 3 * n - 1) for n in ns]
    probs = [m.Problem(P.cl, P.bl, tc(P.ninv), 2) for (_, P, _, _, _, _) in cases]
    D = [tc(c[3]) for c in cases]
    # mean field only (w0, w1 omitted)
    out, st = m.solve_batched(plans, probs, D, None, None, tol=1e-6, prec=m.CR_MIXED)
    for j, (wl, P, op, d, w0, w1) in enumerate(cases):
        assert st[j].status == 0, (j, st[j])
        x = out[j].cpu().numpy()
        b = op.rhs(d=d)
        res = op.norm(b - op.apply(x)) / op.norm(b)
        print("problem %d nside %d: iters %d replacements %d oracle residual %.2e" % (
            j, ns[j], st[j].iters, st[j].refinements, res), flush=True)
        assert res <= 1.5e-6
        # the host-driven mixed solve takes the same decisions from the same scalars
        single, st1 = m.solve(plans[j], probs[j], D[j], None, None, tol=1e-6, prec=m.CR_MIXED, check_every=16)
        e = real_rel(op, x, single.cpu().numpy()[0])
        print("   vs cr_solve: iters %d / %d, rel diff %.2e" % (st[j].iters, st1[0].iters, e), flush=True)
        assert st1[0].iters == st[j].iters and st1[0].refinements == st[j].refinements
        assert e <= 1e-12


def test_batched_rejects_shared_plan():
    m = _m()
    wl, P, op, d, w0, w1 = _problem(0, 4)
    plan = m.Plan(4, 11)
    pr = m.Problem(P.cl, P.bl, tc(P.ninv), 2)
    with pytest.raises(m.CrshtError):
        m.solve_batched([plan, plan], [pr, pr], [tc(d), tc(d)])
