"""GPU parity of ln pi and of the joint amplitude move against the oracle
(same draws): ln A in FP64, the accept decision, and the updated chain."""
import math

import numpy as np
import pytest

import crinputs as ci
from oracle import cr, joint
from tests.gpu_helpers import masked_problem, real_rel, tc

pytestmark = pytest.mark.gpu


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


def test_lnpi_matches_oracle():
    m = _m()
    nside = 8
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), 2)
    rng = np.random.default_rng(3)
    a = op.project(ci.white_alm(rng, wl.lmax) * 50)
    f = op.project(ci.white_alm(rng, wl.lmax) * 50)
    for q in (1.0, 0.7):
        ref = joint.lnpi(cr.CROperator(joint.scaled_problem(P, q)), d, a, f)
        got = m.lnpi(plan, gp, q, tc(d), tc(a), tc(f))
        assert abs(got - ref) <= 1e-11 * abs(ref)


@pytest.mark.parametrize("xi,u", [(0.3, 0.5), (-1.2, 1e-9), (2.0, 0.999999)])
def test_joint_step_matches_oracle(xi, u):
    m = _m()
    nside = 8
    tol = 1e-12
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), 2)
    st = joint.init_state(P, d, 1.0, wl.w0(), wl.w1(), tol)
    rng = ci.rng_for(1, 0, ci.STREAM_MH)
    w0n, w1n = ci.white_alm(rng, wl.lmax), rng.standard_normal(P.ninv.size)
    ch = m.Chain(st.q, st.lnpi, tc(st.ahat), tc(st.fhat))
    res = m.joint_step(plan, gp, tc(d), ch, xi, u, tc(w0n), tc(w1n), sigma_lnq=0.02, tol=tol)
    new, r = joint.joint_step(P, d, st, xi, u, w0n, w1n, 0.02, tol)
    print("lnA gpu", res.lnA, "oracle", r.lnA, flush=True)
    assert abs(res.q_new - r.q_new) <= 1e-15 * r.q_new
    assert abs(res.lnA - r.lnA) <= 1e-8 + 1e-13 * abs(r.lnpi_new)   # absolute: ln A decides the move
    assert res.accepted == r.accepted
    assert abs(ch.q - new.q) <= 1e-15 * new.q
    assert abs(ch.lnpi - new.lnpi) <= 1e-7 * abs(new.lnpi)
    opn = cr.CROperator(joint.scaled_problem(P, new.q))
    assert real_rel(opn, ch.ahat.cpu().numpy(), new.ahat) < 1e-8
    assert real_rel(opn, ch.fhat.cpu().numpy(), new.fhat) < 1e-8
    _ = math
