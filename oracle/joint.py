"""Joint sky-signal and C_l-amplitude Metropolis move (paper Sect. 2.2.2,
after Racine et al. 2016), reduced to one parameter: C_l(q) = q C_l^fid.

Steps of the move (the paper's enumerated algorithm, steps 2-4):
1. propose q' = q exp(sigma xi) (Gaussian transition in ln q);
2. solve the mean field a^(q') (eq. mean-field-map);
3. rescale the fluctuation f^_s = C(q')^{1/2} C(q)^{-1/2} f^ = sqrt(q'/q) f^;
4. evaluate ln pi(q') with f^_s (eq. acceptance-rate and the pi(theta)
   definition after it) and ln A = ln pi(q') - ln pi(q) + ln(q'/q);
5. accept iff ln u < ln A; only when accepted solve a fresh fluctuation
   f^(q') with new w0, w1 (eq. fluc-map) and re-evaluate ln pi with it.

Readings: the garbled middle term of pi is read as a^T S^-1 a^ (completing
the square makes it exact); the prior is uniform in q, so the lognormal
proposal contributes the Jacobian factor q'/q; ties ln u = ln A reject.

The standard two-block Gibbs move (Sect. 2.2.1; the baseline the joint move
is compared with) for the same one-parameter family is gibbs_step: q given
the current sky from its inverse-gamma conditional, then the sky given q.

gibbs_bins_step is the standard Gibbs move for per-bin amplitudes (one
inverse-gamma draw per bin given the sky). hmc_step is the derivative-based
sampler Sect. 4 points to, on per-bin
log-amplitudes: the joint move's target (ln pi at a fixed whitened
fluctuation) explored by Hamiltonian trajectories, with the gradient of
lnpi_grad_fixed.

Pins (tests/test_oracle_joint.py): the acceptance identity against the joint
posterior of the dense model, the misread middle term breaking it, accept and
reject paths; the Gibbs conditional's draws against a numerical integral of
q^(-k/2) exp(-t/(2q)); both samplers' chains against the exact marginal
posterior p(q | d) of a tiny masked problem (Gaussian likelihood of the
observed pixels, brute force on a grid of q); the fixed-fluctuation gradient
against central differences of ln pi; the leapfrog energy error falling as
eps^2; an HMC chain against the same exact posterior.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .cr import CROperator, Problem, pcg


def scaled_problem(fid: Problem, q: float) -> Problem:
    return Problem(fid.nside, fid.lmax, q * fid.cl, fid.bl, fid.ninv, fid.lmin)


def lnpi_terms(op: CROperator, d: np.ndarray, ahat: np.ndarray, fhat: np.ndarray):
    """(chi^2 of the mean field, a^T S^-1 a^, f^T B^T N^-1 B f^)."""
    res = d - op.sht.synth(op.b * op.project(ahat))
    chi2 = float(np.sum(op.p.ninv * res * res))
    prior = op.dot(ahat, op.sinv * ahat)
    ff = op.sht.synth(op.b * op.project(fhat))
    fluct = float(np.sum(op.p.ninv * ff * ff))
    return chi2, prior, fluct


def lnpi(op: CROperator, d, ahat, fhat) -> float:
    return -0.5 * sum(lnpi_terms(op, d, ahat, fhat))


@dataclass
class ChainState:
    q: float
    ahat: np.ndarray
    fhat: np.ndarray
    lnpi: float


def init_state(fid: Problem, d, q: float, w0, w1, tol: float, maxiter: int = 20000, sht=None,
               precond=None) -> ChainState:
    """Algorithm step 1 with a fixed amplitude q instead of a Boltzmann code.
    sht: the transforms to use (default: a new numpy SHT); precond: as for
    pcg (None = the Jacobi diagonal)."""
    op = CROperator(scaled_problem(fid, q), sht)
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter, precond=precond)
    fhat, _ = pcg(op, op.rhs(w0=w0, w1=w1), tol, maxiter, precond=precond)
    return ChainState(q, ahat, fhat, lnpi(op, d, ahat, fhat))


@dataclass
class StepResult:
    accepted: bool
    lnA: float
    q_new: float
    lnpi_new: float


def joint_step(fid: Problem, d, state: ChainState, xi: float, u: float, w0_new, w1_new,
               sigma_lnq: float, tol: float, maxiter: int = 20000, sht=None, precond=None):
    q_new = state.q * math.exp(sigma_lnq * xi)
    op = CROperator(scaled_problem(fid, q_new), sht)
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter, precond=precond)
    f_scaled = math.sqrt(q_new / state.q) * state.fhat
    lp_new = lnpi(op, d, ahat, f_scaled)
    lnA = lp_new - state.lnpi + math.log(q_new / state.q)
    accepted = math.log(u) < lnA
    if not accepted:
        return state, StepResult(False, lnA, q_new, lp_new)
    fhat, _ = pcg(op, op.rhs(w0=w0_new, w1=w1_new), tol, maxiter, precond=precond)
    new = ChainState(q_new, ahat, fhat, lnpi(op, d, ahat, fhat))
    return new, StepResult(True, lnA, q_new, lp_new)


# ------------------------------------------------------------ standard Gibbs
def n_dof(lmax: int, lmin: int) -> int:
    """Real degrees of freedom of a real field with lmin <= l <= lmax."""
    return sum(2 * l + 1 for l in range(lmin, lmax + 1))


def gibbs_shape(fid: Problem) -> float:
    """Shape of the inverse-gamma conditional q | s under a uniform prior in q:
    p(q | s) is proportional to q^(-k/2) exp(-t / (2 q)), i.e. shape k/2 - 1."""
    return 0.5 * n_dof(fid.lmax, fid.lmin) - 1.0


@dataclass
class GibbsResult:
    q_new: float
    t: float


def gibbs_step(fid: Problem, d, state: ChainState, g: float, w0_new, w1_new, tol: float, maxiter: int = 20000):
    """One move of the standard two-block Gibbs sampler (Sect. 2.2.1) for
    C_l(q) = q C_l^fid: q | s with s = a^ + f^ the current sky, t = s^T
    S_fid^-1 s, q' = (t / 2) / g for g ~ Gamma(gibbs_shape, 1) supplied by the
    caller; then s | q': the mean field and a fresh fluctuation at q'."""
    op_fid = CROperator(fid)
    s = state.ahat + state.fhat
    t = op_fid.dot(s, op_fid.sinv * s)
    q_new = 0.5 * t / g
    op = CROperator(scaled_problem(fid, q_new))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    fhat, _ = pcg(op, op.rhs(w0=w0_new, w1=w1_new), tol, maxiter)
    return ChainState(q_new, ahat, fhat, lnpi(op, d, ahat, fhat)), GibbsResult(q_new, t)


# ------------------------------------------------ HMC over bin log-amplitudes
def bin_factors(lmax: int, edges, x, c: float = 1.0) -> np.ndarray:
    """Per-l factor exp(c x_k) on [edges[k], edges[k+1]), 1 elsewhere."""
    f = np.ones(lmax + 1)
    for k in range(len(edges) - 1):
        f[edges[k]:edges[k + 1]] = math.exp(c * x[k])
    return f


def bin_problem(fid: Problem, edges, theta) -> Problem:
    return Problem(fid.nside, fid.lmax, fid.cl * bin_factors(fid.lmax, edges, theta), fid.bl, fid.ninv, fid.lmin)


def lnpi_grad_fixed(fid: Problem, d, edges, theta0, theta, f0, tol: float, maxiter: int = 20000):
    """ln pi at the log-amplitudes theta with the fluctuation f0 (given at
    theta0) carried along as exp((theta - theta0)/2) f0 per bin, and its
    gradient: d ln pi/d theta_k = 1/2 a_k^T S^-1 a_k - 1/2 f_k^T M f, with
    M = B Y^T N^-1 Y B (the mean field a is the minimiser of chi^2 + a^T S^-1 a,
    so only the explicit S^-1 is differentiated). Returns (ln pi, grad, a)."""
    op = CROperator(bin_problem(fid, edges, theta))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    ls = op.ls
    f = f0 * bin_factors(fid.lmax, edges, np.asarray(theta) - np.asarray(theta0), 0.5)[ls]
    lp = lnpi(op, d, ahat, f)
    Mf = op.apply_data_term(f)
    grad = np.zeros(len(edges) - 1)
    for k in range(len(edges) - 1):
        sel = (ls >= edges[k]) & (ls < edges[k + 1])
        ak, fk = ahat * sel, f * sel
        grad[k] = 0.5 * op.dot(ak, op.sinv * ak) - 0.5 * op.dot(fk, Mf)
    return lp, grad, ahat


@dataclass
class BinState:
    theta: np.ndarray
    ahat: np.ndarray
    fhat: np.ndarray
    lnpi: float


def init_bin_state(fid: Problem, d, edges, theta, w0, w1, tol: float, maxiter: int = 20000) -> BinState:
    op = CROperator(bin_problem(fid, edges, theta))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    fhat, _ = pcg(op, op.rhs(w0=w0, w1=w1), tol, maxiter)
    return BinState(np.array(theta, dtype=np.float64), ahat, fhat, lnpi(op, d, ahat, fhat))


@dataclass
class HmcResult:
    accepted: bool
    dH: float
    lnpi_new: float


def hmc_step(fid: Problem, d, edges, state: BinState, p0, u: float, w0_new, w1_new, eps: float, nleap: int,
             tol: float, maxiter: int = 20000):
    """Hamiltonian Monte Carlo move of the bin log-amplitudes at a fixed
    whitened fluctuation: potential U = -ln pi - sum theta (uniform prior in
    the amplitudes exp(theta_k)), unit masses, nleap leapfrog steps of size
    eps from momentum p0; accept iff ln u < -(H_end - H_start); then, accepted
    or not, a fresh fluctuation at the amplitudes the move ends on (a draw of
    the whitened fluctuation given the amplitudes, which leaves the joint
    target invariant by itself)."""
    th0 = np.array(state.theta, dtype=np.float64)
    p = np.array(p0, dtype=np.float64)
    lp, g, ahat = lnpi_grad_fixed(fid, d, edges, th0, th0, state.fhat, tol, maxiter)
    H0 = -lp - th0.sum() + 0.5 * float(p @ p)
    p = p + 0.5 * eps * (g + 1.0)
    th = th0.copy()
    for i in range(nleap):
        th = th + eps * p
        lp, g, ahat = lnpi_grad_fixed(fid, d, edges, th0, th, state.fhat, tol, maxiter)
        p = p + (1.0 if i + 1 < nleap else 0.5) * eps * (g + 1.0)
    H1 = -lp - th.sum() + 0.5 * float(p @ p)
    dH = H1 - H0
    accepted = bool(np.isfinite(dH) and math.log(u) < -dH)
    th_end, a_end = (th, ahat) if accepted else (th0, state.ahat)
    op = CROperator(bin_problem(fid, edges, th_end))
    fhat, _ = pcg(op, op.rhs(w0=w0_new, w1=w1_new), tol, maxiter)
    return BinState(th_end, a_end, fhat, lnpi(op, d, a_end, fhat)), HmcResult(accepted, dH, lp)


# ------------------------------------------------ standard Gibbs over bins
def bin_dof(lmin: int, edges) -> np.ndarray:
    """Real degrees of freedom of each bin (l >= lmin)."""
    return np.array([sum(2 * l + 1 for l in range(max(edges[k], lmin), edges[k + 1])) for k in range(len(edges) - 1)],
                    dtype=np.float64)


def gibbs_bins_shape(fid: Problem, edges) -> np.ndarray:
    """Per-bin inverse-gamma shapes k_b/2 - 1 of A_b | s under uniform priors in
    the amplitudes A_b = exp(theta_b)."""
    return 0.5 * bin_dof(fid.lmin, edges) - 1.0


def gibbs_bins_step(fid: Problem, d, edges, state: BinState, g, w0_new, w1_new, tol: float, maxiter: int = 20000):
    """Standard two-block Gibbs move (Sect. 2.2.1) for per-bin amplitudes:
    with s = a^ + f^ and t_b = sum over the bin of s^T S_fid^-1 s, each
    A_b | s is inverse gamma (shape gibbs_bins_shape, scale t_b/2): A_b =
    (t_b/2)/g_b for g_b ~ Gamma(shape_b, 1) from the caller; theta_b = ln A_b;
    then the mean field and a fresh fluctuation at the new spectrum. Returns
    (new state, t)."""
    op_fid = CROperator(fid)
    s = state.ahat + state.fhat
    t = np.array([op_fid.dot(s * ((op_fid.ls >= edges[k]) & (op_fid.ls < edges[k + 1])), op_fid.sinv * s)
                  for k in range(len(edges) - 1)])
    theta = np.log(0.5 * t / np.asarray(g, dtype=np.float64))
    op = CROperator(bin_problem(fid, edges, theta))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    fhat, _ = pcg(op, op.rhs(w0=w0_new, w1=w1_new), tol, maxiter)
    return BinState(theta, ahat, fhat, lnpi(op, d, ahat, fhat)), t


# ------------------------------------------------ T+Q+U ln pi and joint move
def lnpi_terms_tqu(op, d, ahat, fhat):
    """(chi^2, a^T S^-1 a, f^T B^T N^-1 B f) of a T+Q+U problem
    (oracle.cr_tqu.CROperatorTQU; maps [3][npix], alm [3][nalm])."""
    n = op._ninv()
    res = d - op.synth(op.b * op.project(ahat))
    chi2 = float(np.sum(n * res * res))
    a = op.project(ahat)
    prior = op.dot(a, op._block(op.sinv_lm, a))
    ff = op.synth(op.b * op.project(fhat))
    return chi2, prior, float(np.sum(n * ff * ff))


def lnpi_tqu(op, d, ahat, fhat) -> float:
    return -0.5 * sum(lnpi_terms_tqu(op, d, ahat, fhat))


def joint_step_tqu(fid, d, state: ChainState, xi: float, u: float, w0_new, w1_new, sigma_lnq: float, tol: float,
                   maxiter: int = 20000):
    """joint_step for a T+Q+U problem (all four spectra scaled by q)."""
    from .cr_tqu import CROperatorTQU, ProblemTQU

    def op_at(q):
        return CROperatorTQU(ProblemTQU(fid.nside, fid.lmax, fid.cl * q, fid.bl, fid.ninv_t, fid.ninv_p, fid.lmin))

    q_new = state.q * math.exp(sigma_lnq * xi)
    op = op_at(q_new)
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    f_scaled = math.sqrt(q_new / state.q) * state.fhat
    lp_new = lnpi_tqu(op, d, ahat, f_scaled)
    lnA = lp_new - state.lnpi + math.log(q_new / state.q)
    accepted = math.log(u) < lnA
    if not accepted:
        return state, StepResult(False, lnA, q_new, lp_new)
    fhat, _ = pcg(op, op.rhs(w0=w0_new, w1=w1_new), tol, maxiter)
    return ChainState(q_new, ahat, fhat, lnpi_tqu(op, d, ahat, fhat)), StepResult(True, lnA, q_new, lp_new)
