"""Pins of the oracle's joint (C_l amplitude, sky) Metropolis move."""
import math

import numpy as np

import crinputs as ci
from oracle import cr, dense, healpix, joint


def _problem(nside=4):
    wl = ci.workload_masked_t(nside)
    z, phi = healpix.pixel_coords(nside)
    P = cr.Problem(nside, wl.lmax, wl.cl(), wl.bl(), wl.ninv(z, phi))
    op = cr.CROperator(P)
    d = op.sht.synth(op.b * wl.signal()) + wl.noise(z, phi)
    return wl, P, op, d


def _ln_joint(P, D, d, s, q):
    """ln P(s, q | d) of eq. joint-posterior (uniform prior in q), up to a
    constant: -1/2 chi^2 - 1/2 s^T S^-1 s - 1/2 ln |S|."""
    op = cr.CROperator(joint.scaled_problem(P, q))
    res = d - op.sht.synth(op.b * s)
    chi2 = float(np.sum(P.ninv * res * res))
    prior = op.dot(s, op.sinv * s)
    logdet = sum(math.log(q * P.cl[D.ls[i]]) for i, _ in D.src)
    return -0.5 * (chi2 + prior + logdet)


def test_acceptance_identity_against_joint_posterior():
    # With s = a^ + f^ and s' = a^' + sqrt(q'/q) f^, the paper's pi gives
    # ln pi(q') - ln pi(q) = ln P(s', q'|d) - ln P(s, q|d) + ln|J|, where
    # |J| = (q'/q)^{ndof/2} is the Jacobian of the deterministic rescaling.
    # A dropped or misread term of pi (e.g. the middle term) breaks it.
    wl, P, op, d = _problem(4)
    D = dense.DenseY(4, wl.lmax, lmin=2)
    q, qn = 1.0, 1.37
    st = joint.init_state(P, d, q, wl.w0(), wl.w1(), 1e-14)
    opn = cr.CROperator(joint.scaled_problem(P, qn))
    ahat_n, _ = cr.pcg(opn, opn.rhs(d=d), 1e-14)
    fs = math.sqrt(qn / q) * st.fhat
    lhs = joint.lnpi(opn, d, ahat_n, fs) - st.lnpi
    ndof = D.ndof
    rhs = (_ln_joint(P, D, d, ahat_n + fs, qn) - _ln_joint(P, D, d, st.ahat + st.fhat, q)
           + 0.5 * ndof * math.log(qn / q))
    assert abs(lhs - rhs) < 1e-7 * max(1.0, abs(lhs))


def test_misread_middle_term_breaks_identity():
    # Planted mistake: reading the middle term as s^T S^-1 a^ (the garbled
    # text) with s = a^ + f^ instead of a^T S^-1 a^ changes ln pi differences.
    wl, P, op, d = _problem(4)
    q, qn = 1.0, 1.37
    st = joint.init_state(P, d, q, wl.w0(), wl.w1(), 1e-14)
    opn = cr.CROperator(joint.scaled_problem(P, qn))
    ahat_n, _ = cr.pcg(opn, opn.rhs(d=d), 1e-14)
    fs = math.sqrt(qn / q) * st.fhat
    good = joint.lnpi(opn, d, ahat_n, fs) - st.lnpi
    bad_new = joint.lnpi(opn, d, ahat_n, fs) - 0.5 * opn.dot(fs, opn.sinv * ahat_n)
    bad_old = st.lnpi - 0.5 * op.dot(st.fhat, op.sinv * st.ahat)
    assert abs((bad_new - bad_old) - good) > 1e-6 * abs(good)


def test_joint_step_accept_and_reject_paths():
    wl, P, op, d = _problem(4)
    st = joint.init_state(P, d, 1.0, wl.w0(), wl.w1(), 1e-12)
    rng = ci.rng_for(1, 0, ci.STREAM_MH)
    w0n, w1n = wl.w0() * 0.5, wl.w1() * 0.5
    # u -> 1 with xi chosen so the proposal is unlikely to be accepted
    s_rej, r = joint.joint_step(P, d, st, xi=40.0, u=1.0 - 1e-15, w0_new=w0n, w1_new=w1n,
                                sigma_lnq=0.02, tol=1e-12)
    if not r.accepted:
        assert s_rej is st
    # u -> 0 accepts unless ln A is hugely negative
    s_acc, r2 = joint.joint_step(P, d, st, xi=0.1, u=1e-300, w0_new=w0n, w1_new=w1n,
                                 sigma_lnq=0.02, tol=1e-12)
    assert r2.accepted and abs(s_acc.q - math.exp(0.002)) < 1e-15
    assert np.isclose(r2.q_new, s_acc.q)
    # accepted state re-evaluates ln pi with the freshly solved fluctuation
    opn = cr.CROperator(joint.scaled_problem(P, s_acc.q))
    assert abs(s_acc.lnpi - joint.lnpi(opn, d, s_acc.ahat, s_acc.fhat)) < 1e-9 * abs(s_acc.lnpi)
    _ = rng
