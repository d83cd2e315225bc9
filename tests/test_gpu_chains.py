"""GPU parity of the standard Gibbs amplitude move (gibbs_cl_step) against the
oracle (same draws), the warm-started mean-field solve of the joint move, and
the chain driver (paper_2306_15511_amd/chains.py) replayed move by move by
the oracle's joint and Gibbs moves with the same random numbers."""
import math

import numpy as np
import pytest
import torch

import crinputs as ci
from oracle import cr, joint
from tests.gpu_helpers import masked_problem, real_rel, tc

pytestmark = pytest.mark.gpu


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


def _setup(nside, tol):
    m = _m()
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), 2)
    st = joint.init_state(P, d, 1.0, wl.w0(), wl.w1(), tol)
    return m, wl, P, d, plan, gp, st


def _chain(m, st):
    return m.Chain(st.q, st.lnpi, tc(st.ahat), tc(st.fhat))


@pytest.mark.parametrize("gscale", [1.0, 0.8, 1.3])
def test_gibbs_step_matches_oracle(gscale):
    tol = 1e-12
    m, wl, P, d, plan, gp, st = _setup(8, tol)
    print("case gibbs step", gscale, flush=True)
    alpha = joint.gibbs_shape(P)
    assert abs(m.gibbs_shape(P.lmax, 2) - alpha) < 1e-12
    g = gscale * alpha
    rng = ci.rng_for(1, 1, ci.STREAM_MH)
    w0n, w1n = ci.white_alm(rng, wl.lmax), rng.standard_normal(P.ninv.size)
    ch = _chain(m, st)
    res = m.gibbs_step(plan, gp, tc(d), ch, g, tc(w0n), tc(w1n), tol=tol)
    new, r = joint.gibbs_step(P, d, st, g, w0n, w1n, tol)
    print("t gpu %.15e oracle %.15e q %.6f" % (res.t, r.t, r.q_new), flush=True)
    assert abs(res.t - r.t) <= 1e-12 * r.t
    assert abs(res.q_new - r.q_new) <= 1e-12 * r.q_new and abs(ch.q - new.q) <= 1e-12 * new.q
    assert abs(ch.lnpi - new.lnpi) <= 1e-9 * abs(new.lnpi)
    opn = cr.CROperator(joint.scaled_problem(P, new.q))
    assert real_rel(opn, ch.ahat.cpu().numpy(), new.ahat) < 1e-8
    assert real_rel(opn, ch.fhat.cpu().numpy(), new.fhat) < 1e-8
    assert res.mean_stats.status == 0 and res.fluct_stats.status == 0


def test_joint_mean_field_warm_start():
    # the warm-started mean-field solve of the move reaches the same tolerance
    # as a cold solve at the proposal, in fewer iterations
    m = _m()
    nside = 32
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), 2)
    tol = 1e-8
    ch0, _ = m.solve(plan, gp, tc(d), tol=tol)
    fl0, _ = m.solve(plan, gp, None, tc(wl.w0()), tc(wl.w1()), tol=tol)
    ch = m.Chain(1.0, m.lnpi(plan, gp, 1.0, tc(d), ch0[0], fl0[0]), ch0[0].clone(), fl0[0].clone())
    xi = 0.5
    res = m.joint_step(plan, gp, tc(d), ch, xi, 1e-300, tc(wl.w0()), tc(wl.w1()), sigma_lnq=0.02, tol=tol)
    qn = res.q_new
    cold, stc = m.solve(plan, m.Problem(P.cl * qn, P.bl, tc(P.ninv), 2), tc(d), tol=tol)
    print("warm iters %d cold iters %d" % (res.mean_stats.iters, stc[0].iters), flush=True)
    assert res.accepted and res.mean_stats.status == 0
    assert res.mean_stats.rel_resid_true <= tol
    assert res.mean_stats.iters < stc[0].iters
    opn = cr.CROperator(joint.scaled_problem(P, qn))
    assert real_rel(opn, ch.ahat.cpu().numpy(), cold[0].cpu().numpy()) < 1e-5


@pytest.mark.parametrize("kind", ["joint", "gibbs"])
def test_chain_driver_replays_oracle(kind):
    from paper_2306_15511_amd import chains
    tol = 1e-12
    m, wl, P, d, plan, gp, st = _setup(8, tol)
    print("case chains", kind, flush=True)
    nchain, nsteps = 2, 4
    alpha = joint.gibbs_shape(P)
    draws = {}

    def draw(c, s):
        if (c, s) not in draws:
            rng = np.random.default_rng([77, c, s])
            r = {"xi": float(rng.standard_normal()), "u": float(rng.uniform())} if kind == "joint" else \
                {"g": float(rng.gamma(alpha))}
            r["w0"] = ci.white_alm(rng, wl.lmax)
            r["w1"] = rng.standard_normal(P.ninv.size)
            draws[(c, s)] = r
        return draws[(c, s)]

    gch = [_chain(m, st) for _ in range(nchain)]
    run = chains.run_chains(plan, gp, tc(d), gch, nsteps, kind=kind, sigma_lnq=0.05, draw=draw, tol=tol)
    for c in range(nchain):
        ost = st
        for s in range(nsteps):
            r = draw(c, s)
            if kind == "joint":
                ost, res = joint.joint_step(P, d, ost, r["xi"], r["u"], r["w0"], r["w1"], 0.05, tol)
                assert bool(run.accepted[c, s]) == res.accepted
            else:
                ost, res = joint.gibbs_step(P, d, ost, r["g"], r["w0"], r["w1"], tol)
            assert abs(run.q[c, s + 1] - ost.q) <= 1e-10 * ost.q, (c, s)
        assert abs(gch[c].lnpi - ost.lnpi) <= 1e-8 * abs(ost.lnpi)
    summ = run.summary()
    print(summ, flush=True)
    assert summ["steps"] == nsteps and 0.0 <= summ["acceptance"] <= 1.0 and summ["iat_lnq"] >= 1.0
    _ = math, torch
