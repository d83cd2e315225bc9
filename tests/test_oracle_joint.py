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


def _tiny(nside=2, lmax=4):
    wl = ci.workload_masked_t(nside, lmax)
    z, phi = healpix.pixel_coords(nside)
    ninv = wl.ninv(z, phi)
    P = cr.Problem(nside, lmax, wl.cl(), wl.bl(), ninv)
    op = cr.CROperator(P)
    d = op.sht.synth(op.b * wl.signal()) + wl.noise(z, phi)
    return wl, P, op, d


def test_gibbs_conditional_parameters_against_numeric_density():
    # q | s for a uniform prior in q: the density is p(s | q) of the real
    # degrees of freedom (variance q C_l / W per coordinate, W = 1 for m = 0,
    # 2 for m > 0), integrated numerically on a grid of q; the step's
    # inverse-gamma (shape gibbs_shape, scale t/2) must have its moments
    wl, P, op, d = _tiny(2, 3)
    rng = np.random.default_rng(3)
    st = joint.init_state(P, d, 1.0, ci.white_alm(rng, P.lmax), rng.standard_normal(d.size), 1e-12)
    D = dense.DenseY(P.nside, P.lmax, lmin=2)
    u = D.to_real(st.ahat + st.fhat)
    var1 = D._per_dof(P.cl) / D.W
    qs = np.exp(np.linspace(np.log(1e-3), np.log(1e3), 200001))
    lp = np.array([-0.5 * np.sum(u * u / (q * var1)) - 0.5 * np.sum(np.log(q * var1)) for q in qs[::100]])
    qg = qs[::100]
    w = np.exp(lp - lp.max()) * qg                      # uniform prior in q on a log grid
    mean = float(np.sum(w * qg) / np.sum(w))
    var = float(np.sum(w * (qg - mean) ** 2) / np.sum(w))
    _, r = joint.gibbs_step(P, d, st, 1.0, ci.white_alm(rng, P.lmax), rng.standard_normal(d.size), 1e-10)
    a, b = joint.gibbs_shape(P), 0.5 * r.t
    assert abs(b / (a - 1.0) - mean) < 2e-3 * mean
    assert abs(b * b / ((a - 1.0) ** 2 * (a - 2.0)) - var) < 1e-2 * var
    assert abs(r.q_new - b / 1.0) < 1e-12 * r.q_new      # g = 1


def _iat(x, c=5.0):
    """Integrated autocorrelation time (Sokal's automatic window)."""
    x = np.asarray(x) - np.mean(x)
    n = x.size
    f = np.fft.rfft(x, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    acf /= acf[0]
    tau = 1.0
    for m in range(1, n):
        tau = 1.0 + 2.0 * np.sum(acf[1:m + 1])
        if m >= c * tau:
            break
    return max(tau, 1.0)


def test_joint_and_gibbs_chains_sample_exact_marginal_posterior():
    # brute force on a tiny masked problem: p(q | d) from the Gaussian
    # likelihood of the observed pixels, d ~ N(0, Y B S(q) B Y^T + N), on a
    # grid of q; both samplers' chains must reproduce its mean within four
    # standard errors (from the chains' own autocorrelation times)
    wl, P, op, d = _tiny(2, 4)
    D = dense.DenseY(P.nside, P.lmax, lmin=2)
    obs = P.ninv > 0
    Yo = D.Y[obs] * D._per_dof(P.bl)[None, :]
    var1 = D._per_dof(P.cl) / D.W
    def lnL(q):
        C = (Yo * (q * var1)[None, :]) @ Yo.T + np.diag(1.0 / P.ninv[obs])
        L = np.linalg.cholesky(C)
        y = np.linalg.solve(L, d[obs])
        return -0.5 * float(y @ y) - float(np.log(np.diag(L)).sum())
    qs = np.exp(np.linspace(np.log(0.02), np.log(50.0), 3000))
    lp = np.array([lnL(q) for q in qs])
    w = np.exp(lp - lp.max()) * qs
    exact = float(np.sum(w * qs) / np.sum(w))
    rng = np.random.default_rng(5)
    st0 = joint.init_state(P, d, 1.0, ci.white_alm(rng, P.lmax), rng.standard_normal(d.size), 1e-10)
    alpha = joint.gibbs_shape(P)
    for kind in ("joint", "gibbs"):
        st, trace, acc = st0, [], 0
        for _ in range(800):
            w0n, w1n = ci.white_alm(rng, P.lmax), rng.standard_normal(d.size)
            if kind == "joint":
                st, r = joint.joint_step(P, d, st, rng.standard_normal(), rng.uniform(), w0n, w1n, 0.3, 1e-8)
                acc += r.accepted
            else:
                st, r = joint.gibbs_step(P, d, st, rng.gamma(alpha), w0n, w1n, 1e-8)
            trace.append(st.q)
        x = np.array(trace[100:])
        se = x.std() * math.sqrt(_iat(x) / x.size)
        print(kind, "mean %.3f exact %.3f se %.3f accept %.2f" % (x.mean(), exact, se, acc / 800))
        assert abs(x.mean() - exact) < 4.0 * se, (kind, x.mean(), exact, se)
        if kind == "joint":
            assert 0.2 < acc / 800 < 0.95


# ------------------------------------------------ HMC over bin log-amplitudes
def test_fixed_fluctuation_gradient_against_central_differences():
    # d ln pi / d theta_k at a fixed whitened fluctuation (f carried as
    # exp((theta - theta0)/2) f0) against central differences of ln pi itself,
    # on three bins; both terms of the gradient are far above the tolerance,
    # so dropping either (or a wrong factor on the fluctuation term) fails
    wl, P, op, d = _problem(4)
    edges = [2, 4, 8, P.lmax + 1]
    rng = np.random.default_rng(11)
    th0 = np.array([0.1, -0.2, 0.05])
    st = joint.init_bin_state(P, d, edges, th0, ci.white_alm(rng, P.lmax), rng.standard_normal(d.size), 1e-13)
    th = th0 + np.array([0.3, -0.15, 0.2])
    lp, g, ahat = joint.lnpi_grad_fixed(P, d, edges, th0, th, st.fhat, 1e-13)
    h = 1e-4
    fd = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        lpp = joint.lnpi_grad_fixed(P, d, edges, th0, th + e, st.fhat, 1e-13)[0]
        lpm = joint.lnpi_grad_fixed(P, d, edges, th0, th - e, st.fhat, 1e-13)[0]
        fd[k] = (lpp - lpm) / (2 * h)
    assert np.all(np.abs(g - fd) < 1e-6 * np.maximum(1.0, np.abs(fd))), (g, fd)
    opb = cr.CROperator(joint.bin_problem(P, edges, th))
    f = st.fhat * joint.bin_factors(P.lmax, edges, th - th0, 0.5)[opb.ls]
    Mf = opb.apply_data_term(f)
    for k in range(3):
        sel = (opb.ls >= edges[k]) & (opb.ls < edges[k + 1])
        assert 0.5 * opb.dot(ahat * sel, opb.sinv * ahat * sel) > 1e-3
        assert 0.5 * opb.dot(f * sel, Mf) > 1e-3
    # at theta = theta0 the carried fluctuation is f0 itself
    assert abs(joint.lnpi_grad_fixed(P, d, edges, th0, th0, st.fhat, 1e-13)[0] - st.lnpi) < 1e-9 * abs(st.lnpi)


def test_leapfrog_energy_error_falls_as_step_squared():
    # fixed trajectory length, step halved: |dH| of the same trajectory falls
    # by about four (second-order integrator); a wrong half step at either end
    # or a gradient of the wrong sign makes it first order or divergent
    wl, P, op, d = _tiny(2, 4)
    edges = [2, 3, 5]
    rng = np.random.default_rng(7)
    st = joint.init_bin_state(P, d, edges, np.array([1.0, 0.6]), ci.white_alm(rng, P.lmax),
                              rng.standard_normal(d.size), 1e-12)
    p0 = np.array([0.7, -0.4])
    w0n, w1n = ci.white_alm(rng, P.lmax), rng.standard_normal(d.size)
    dh = [joint.hmc_step(P, d, edges, st, p0, 0.5, w0n, w1n, 0.4 / n, n, 1e-12)[1].dH for n in (4, 8, 16)]
    assert abs(dh[0]) > 1e-4
    for a, b in zip(dh, dh[1:]):
        assert 3.0 < a / b < 5.0, dh


def _two_bin_exact(P, d, edges):
    """Exact posterior means of (theta_0, theta_1) of two bins on the tiny
    masked problem: Gaussian likelihood of the observed pixels with C_l
    exp(theta_b) on bin b, uniform priors in the amplitudes exp(theta_b),
    on a grid."""
    D = dense.DenseY(P.nside, P.lmax, lmin=2)
    obs = P.ninv > 0
    Yo = D.Y[obs] * D._per_dof(P.bl)[None, :]
    var1 = D._per_dof(P.cl) / D.W
    lsd = D._per_dof(np.arange(P.lmax + 1, dtype=np.float64))
    t0, t1 = np.linspace(-4.0, 10.0, 141), np.linspace(-3.0, 4.0, 71)
    lp = np.zeros((t0.size, t1.size))
    for i, a0 in enumerate(t0):
        for j, a1 in enumerate(t1):
            C = (Yo * (var1 * np.where(lsd < edges[1], math.exp(a0), math.exp(a1)))[None, :]) @ Yo.T
            L = np.linalg.cholesky(C + np.diag(1.0 / P.ninv[obs]))
            y = np.linalg.solve(L, d[obs])
            lp[i, j] = -0.5 * float(y @ y) - float(np.log(np.diag(L)).sum()) + a0 + a1
    w = np.exp(lp - lp.max())
    assert w[-1].sum() < 1e-5 * w.sum() and w[:, -1].sum() < 1e-5 * w.sum()
    return [float((w.sum(1) * t0).sum() / w.sum()), float((w.sum(0) * t1).sum() / w.sum())]


def test_hmc_chain_samples_exact_marginal_posterior():
    # two bins (l = 2; l = 3..4) of the tiny masked problem: the exact
    # posterior of (theta_0, theta_1) from the Gaussian likelihood of the
    # observed pixels with a uniform prior in the amplitudes exp(theta_k), on
    # a grid; the HMC chain's means within four standard errors
    wl, P, op, d = _tiny(2, 4)
    edges = [2, 3, 5]
    exact = _two_bin_exact(P, d, edges)
    rng = np.random.default_rng(5)
    st = joint.init_bin_state(P, d, edges, np.zeros(2), ci.white_alm(rng, P.lmax), rng.standard_normal(d.size), 1e-10)
    trace, acc = [], 0
    for _ in range(300):
        st, r = joint.hmc_step(P, d, edges, st, rng.standard_normal(2), rng.uniform(), ci.white_alm(rng, P.lmax),
                               rng.standard_normal(d.size), 0.2, 3, 1e-8)
        acc += r.accepted
        trace.append(st.theta.copy())
    x = np.array(trace[50:])
    for k in range(2):
        se = x[:, k].std() * math.sqrt(_iat(x[:, k]) / x.shape[0])
        print(k, "mean %.3f exact %.3f se %.3f" % (x[:, k].mean(), exact[k], se))
        assert abs(x[:, k].mean() - exact[k]) < 4.0 * se, (k, x[:, k].mean(), exact[k], se)
    assert 0.5 < acc / 300 <= 1.0


# ------------------------------------------------ standard Gibbs over bins
def test_bin_gibbs_conditional_parameters():
    # per-bin t_b from the dense real coordinates of the sky (variance C_l / W
    # per coordinate) against the step's, the shapes from the bins' real
    # degrees of freedom, and A_b = (t_b / 2) / g_b
    wl, P, op, d = _tiny(2, 4)
    edges = [2, 3, 5]
    rng = np.random.default_rng(13)
    st = joint.init_bin_state(P, d, edges, np.array([0.2, -0.1]), ci.white_alm(rng, P.lmax),
                              rng.standard_normal(d.size), 1e-12)
    D = dense.DenseY(P.nside, P.lmax, lmin=2)
    u = D.to_real(st.ahat + st.fhat)
    var1 = D._per_dof(P.cl) / D.W
    lsd = D._per_dof(np.arange(P.lmax + 1, dtype=np.float64))
    tb = [float(np.sum((u * u / var1)[(lsd >= edges[k]) & (lsd < edges[k + 1])])) for k in range(2)]
    kb = [int(np.sum((lsd >= edges[k]) & (lsd < edges[k + 1]))) for k in range(2)]
    assert np.allclose(joint.gibbs_bins_shape(P, edges), 0.5 * np.array(kb) - 1.0)
    g = np.array([1.7, 6.2])
    new, t = joint.gibbs_bins_step(P, d, edges, st, g, ci.white_alm(rng, P.lmax), rng.standard_normal(d.size), 1e-10)
    assert np.allclose(t, tb, rtol=1e-12)
    assert np.allclose(np.exp(new.theta), 0.5 * np.array(tb) / g, rtol=1e-12)


def test_bin_gibbs_chain_samples_exact_marginal_posterior():
    wl, P, op, d = _tiny(2, 4)
    edges = [2, 3, 5]
    exact = _two_bin_exact(P, d, edges)
    alpha = joint.gibbs_bins_shape(P, edges)
    rng = np.random.default_rng(9)
    st = joint.init_bin_state(P, d, edges, np.zeros(2), ci.white_alm(rng, P.lmax), rng.standard_normal(d.size), 1e-10)
    trace = []
    for _ in range(400):
        st, _ = joint.gibbs_bins_step(P, d, edges, st, rng.gamma(alpha), ci.white_alm(rng, P.lmax),
                                      rng.standard_normal(d.size), 1e-8)
        trace.append(st.theta.copy())
    x = np.array(trace[50:])
    for k in range(2):
        se = x[:, k].std() * math.sqrt(_iat(x[:, k]) / x.shape[0])
        print(k, "mean %.3f exact %.3f se %.3f" % (x[:, k].mean(), exact[k], se))
        assert abs(x[:, k].mean() - exact[k]) < 4.0 * se, (k, x[:, k].mean(), exact[k], se)


def test_tqu_lnpi_reduces_to_temperature_without_polarisation_data():
    # with N_P^-1 = 0 and C^TE = 0 the E and B mean fields vanish and their
    # fluctuations never reach the data term, so ln pi of T+Q+U equals the
    # temperature ln pi of the same T problem; with polarisation data the
    # extra terms are present (the reduction is not trivially met)
    from oracle import cr_tqu
    nside, lmax = 4, 11
    wl = ci.workload_masked_t(nside, lmax)
    z, phi = healpix.pixel_coords(nside)
    nt = wl.ninv(z, phi)
    cl = ci.cl_tqu(lmax, wl.amp, 0.0)
    P3 = cr_tqu.ProblemTQU(nside, lmax, cl, wl.bl(), nt, np.zeros_like(nt))
    op3 = cr_tqu.CROperatorTQU(P3)
    P1 = cr.Problem(nside, lmax, cl[0], wl.bl(), nt)
    op1 = cr.CROperator(P1)
    rng = np.random.default_rng(4)
    d3 = np.stack([op1.sht.synth(op1.b * wl.signal()) + wl.noise(z, phi), rng.standard_normal(nt.size),
                   rng.standard_normal(nt.size)])
    w0 = np.stack([ci.white_alm(rng, lmax) for _ in range(3)])
    w1 = rng.standard_normal((3, nt.size))
    a3, _ = cr.pcg(op3, op3.rhs(d=d3), 1e-13)
    f3, _ = cr.pcg(op3, op3.rhs(w0=w0, w1=w1), 1e-13)
    a1, _ = cr.pcg(op1, op1.rhs(d=d3[0]), 1e-13)
    f1, _ = cr.pcg(op1, op1.rhs(w0=w0[0], w1=w1[0]), 1e-13)
    assert np.max(np.abs(a3[1:])) < 1e-12 * np.max(np.abs(a3[0]))
    # the fluctuation's E, B parts are prior draws: their prior term stays, so
    # compare the terms: chi^2 and the data term of f equal, the prior of a equal
    t3 = joint.lnpi_terms_tqu(op3, d3, a3, f3)
    t1 = joint.lnpi_terms(op1, d3[0], a1, f1)
    for x, y in zip(t3, t1):
        assert abs(x - y) <= 1e-9 * max(1.0, abs(y)), (t3, t1)
    P3p = cr_tqu.ProblemTQU(nside, lmax, cl, wl.bl(), nt, nt / 2.0)
    op3p = cr_tqu.CROperatorTQU(P3p)
    a3p, _ = cr.pcg(op3p, op3p.rhs(d=d3), 1e-13)
    assert abs(joint.lnpi_terms_tqu(op3p, d3, a3p, f3)[0] - t1[0]) > 1e-3 * abs(t1[0])
