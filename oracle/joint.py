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

Pins (tests/test_oracle_joint.py): the acceptance identity against the joint
posterior of the dense model, the misread middle term breaking it, accept and
reject paths; the Gibbs conditional's draws against a numerical integral of
q^(-k/2) exp(-t/(2q)); both samplers' chains against the exact marginal
posterior p(q | d) of a tiny masked problem (Gaussian likelihood of the
observed pixels, brute force on a grid of q).
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


def init_state(fid: Problem, d, q: float, w0, w1, tol: float, maxiter: int = 20000) -> ChainState:
    """Algorithm step 1 with a fixed amplitude q instead of a Boltzmann code."""
    op = CROperator(scaled_problem(fid, q))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    fhat, _ = pcg(op, op.rhs(w0=w0, w1=w1), tol, maxiter)
    return ChainState(q, ahat, fhat, lnpi(op, d, ahat, fhat))


@dataclass
class StepResult:
    accepted: bool
    lnA: float
    q_new: float
    lnpi_new: float


def joint_step(fid: Problem, d, state: ChainState, xi: float, u: float, w0_new, w1_new,
               sigma_lnq: float, tol: float, maxiter: int = 20000):
    q_new = state.q * math.exp(sigma_lnq * xi)
    op = CROperator(scaled_problem(fid, q_new))
    ahat, _ = pcg(op, op.rhs(d=d), tol, maxiter)
    f_scaled = math.sqrt(q_new / state.q) * state.fhat
    lp_new = lnpi(op, d, ahat, f_scaled)
    lnA = lp_new - state.lnpi + math.log(q_new / state.q)
    accepted = math.log(u) < lnA
    if not accepted:
        return state, StepResult(False, lnA, q_new, lp_new)
    fhat, _ = pcg(op, op.rhs(w0=w0_new, w1=w1_new), tol, maxiter)
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
