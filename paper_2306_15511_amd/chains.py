"""Chains of the joint amplitude / sky sampler and of the standard Gibbs
sampler on one GPU (paper Sect. 2.2.1 and 2.2.2, for the one-parameter family
C_l(q) = q C_l^fid with a uniform prior in q), and of the Hamiltonian sampler
of per-bin log-amplitudes (C_l = C_l^fid exp(theta_k) on bins in l, uniform
prior in the amplitudes; the derivative-based sampler of Sect. 4).

Every move is one library call (joint_cl_step, gibbs_cl_step or hmc_cl_step): the solves,
ln pi and the accept test run on the GPU; this module only orders the moves
of many chains, draws their random numbers on the host (numpy, so a run is
reproducible from its seed) and reduces the traces to the diagnostics of the
paper's comparison: the acceptance rate of the joint move and the integrated
autocorrelation time of ln q. The mean-field solve of each move starts from
the chain's previous mean field (warm start inside the library), and ln pi
of the current state is carried in the chain (cached, never recomputed).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np
import torch

from . import crsht


def white_alm(rng: np.random.Generator, lmax: int) -> np.ndarray:
    """Unit-variance draw of a real field's m >= 0 coefficients (m-major):
    Re, Im ~ N(0, 1/2) for m > 0, real N(0, 1) for m = 0."""
    ms = np.concatenate([np.full(lmax - m + 1, m) for m in range(lmax + 1)])
    g = rng.standard_normal((2, ms.size))
    out = (g[0] + 1j * g[1]) / math.sqrt(2.0)
    out[ms == 0] = g[0][ms == 0]
    return out


def integrated_autocorr_time(x, c: float = 5.0) -> float:
    """Integrated autocorrelation time 1 + 2 sum_k rho_k with Sokal's
    automatic window (the smallest M with M >= c tau(M))."""
    x = np.asarray(x, dtype=np.float64)
    x = x - x.mean()
    n = x.size
    if n < 2 or not np.any(x):
        return 1.0
    f = np.fft.rfft(x, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    acf /= acf[0]
    tau = 1.0
    for m in range(1, n):
        tau = 1.0 + 2.0 * float(np.sum(acf[1:m + 1]))
        if m >= c * tau:
            break
    return max(tau, 1.0)


def autocorrelation(x) -> np.ndarray:
    """zeta(Delta) for Delta = 0 .. n-1 (Sect. 5, Markov chain correlation
    length): the mean over the n - Delta available pairs (i, i + Delta) of the
    product of the chain values standardised by the chain's own mean and
    standard deviation."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    sd = x.std()
    if n < 2 or sd == 0.0:
        return np.ones(max(n, 1))
    y = (x - x.mean()) / sd
    f = np.fft.rfft(y, 2 * n)
    sums = np.fft.irfft(f * np.conj(f), 2 * n)[:n]
    return sums / np.arange(n, 0, -1)


def correlation_length(x, threshold: float = 0.1) -> int:
    """The paper's overall correlation length: the first lag Delta with
    zeta(Delta) < threshold (0.1); the chain length if there is none."""
    z = autocorrelation(x)
    below = np.nonzero(z < threshold)[0]
    return int(below[0]) if below.size else int(z.size)


def scaled(fid: crsht.Problem, q: float) -> crsht.Problem:
    return crsht.Problem(np.asarray(fid.cl) * q, fid.bl, fid.ninv, fid.lmin)


def init_chain(plan: crsht.Plan, fid: crsht.Problem, d: torch.Tensor, q: float, w0: torch.Tensor,
               w1: torch.Tensor, **solve_kw) -> crsht.Chain:
    """State at amplitude q: mean field, fluctuation from (w0, w1), ln pi."""
    p = scaled(fid, q)
    ahat, _ = crsht.solve(plan, p, d, **solve_kw)
    fhat, _ = crsht.solve(plan, p, None, w0, w1, **solve_kw)
    ahat, fhat = ahat[0].clone(), fhat[0].clone()
    return crsht.Chain(q, crsht.lnpi(plan, fid, q, d, ahat, fhat), ahat, fhat)


@dataclass
class ChainRun:
    kind: str
    q: np.ndarray            # [nchains, nsteps + 1] amplitude after each move (start first)
    accepted: np.ndarray     # [nchains, nsteps] joint: accept flags; gibbs: all True
    mean_iters: np.ndarray   # [nchains, nsteps] iterations of the mean-field solve
    fluct_iters: np.ndarray  # [nchains, nsteps] iterations of the fluctuation solve (0 if rejected)
    acceptance: np.ndarray   # [nchains]
    iat: np.ndarray          # [nchains] integrated autocorrelation time of ln q (after burn-in)
    corr_len: np.ndarray     # [nchains] first lag with zeta(lag) < 0.1 of ln q (after burn-in)

    def summary(self) -> dict:
        return {"kind": self.kind, "chains": int(self.q.shape[0]), "steps": int(self.q.shape[1] - 1),
                "acceptance": float(self.acceptance.mean()), "iat_lnq": float(self.iat.mean()),
                "corr_len_lnq": float(self.corr_len.mean()),
                "mean_iters": float(self.mean_iters.mean()), "q_mean": float(self.q[:, 1:].mean())}


def default_draws(kind: str, lmax: int, npix: int, alpha: float, sigma_lnq: float, seed: int):
    """Random numbers of each move in a fixed order (numpy Generator seeded
    per chain): joint: xi, u, w0, w1; gibbs: g ~ Gamma(alpha, 1), w0, w1."""
    rngs = {}

    def draw(chain: int, step: int) -> dict:
        rng = rngs.setdefault(chain, np.random.default_rng([seed, chain]))
        out = {}
        if kind == "joint":
            out["xi"] = float(rng.standard_normal())
            out["u"] = float(rng.uniform())
        else:
            out["g"] = float(rng.gamma(alpha))
        out["w0"] = white_alm(rng, lmax)
        out["w1"] = rng.standard_normal(npix)
        return out

    return draw


def device_draws(plan: crsht.Plan, kind: str, alpha: Optional[float] = None, seed: int = 0, nbins: int = 1):
    """Like default_draws, with w0 and w1 drawn on the device (crsht.white:
    Philox4x32-10 keyed by seed and chain, counter = step); the scalars (xi,
    u; g; p0, u for kind "hmc") from a numpy Generator per chain."""
    rngs = {}

    def draw(chain: int, step: int) -> dict:
        rng = rngs.setdefault(chain, np.random.default_rng([seed, chain, 2]))
        out = {}
        if kind == "joint":
            out["xi"] = float(rng.standard_normal())
            out["u"] = float(rng.uniform())
        elif kind == "gibbs":
            out["g"] = float(rng.gamma(alpha))
        else:
            out["p0"] = rng.standard_normal(nbins)
            out["u"] = float(rng.uniform())
        w0, w1 = crsht.white(plan, 1, (seed << 24) + chain, step)
        out["w0"], out["w1"] = w0[0], w1[0]
        return out

    return draw


def _on(x, dev) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(dev)
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _stack(xs, dev) -> torch.Tensor:
    if isinstance(xs[0], torch.Tensor):
        return torch.stack([x.to(dev) for x in xs]).contiguous()
    return torch.from_numpy(np.ascontiguousarray(np.stack(xs))).to(dev)


def run_chains(plan: crsht.Plan, fid: crsht.Problem, d: torch.Tensor, chains: list, nsteps: int,
               kind: str = "joint", sigma_lnq: float = 0.02, seed: int = 0, burn: int = 0,
               draw: Optional[Callable[[int, int], dict]] = None, batched: bool = False, **solve_kw) -> ChainRun:
    """Advance every chain (crsht.Chain, updated in place) by nsteps moves of
    the joint sampler (kind "joint", Gaussian proposal of width sigma_lnq in
    ln q) or of the standard Gibbs sampler (kind "gibbs"). draw(chain, step)
    returns that move's random numbers (default: default_draws). batched:
    every step moves all chains in one joint_cl_step_batch or
    gibbs_cl_step_batch call (the chains' solves as the columns of one
    solve; len(chains) columns, 2 len(chains) for Gibbs moves, at most the
    plan's nrhs_max)."""
    if kind not in ("joint", "gibbs"):
        raise ValueError("kind must be 'joint' or 'gibbs'")

    n = len(chains)
    alpha = crsht.gibbs_shape(plan.lmax, fid.lmin)
    if draw is None:
        draw = default_draws(kind, plan.lmax, plan.npix, alpha, sigma_lnq, seed)
    dev = d.device
    q = np.zeros((n, nsteps + 1))
    acc = np.zeros((n, nsteps), dtype=bool)
    mi = np.zeros((n, nsteps), dtype=np.int64)
    fi = np.zeros((n, nsteps), dtype=np.int64)
    for c, ch in enumerate(chains):
        q[c, 0] = ch.q
    for s in range(nsteps):
        if batched:
            rs = [draw(c, s) for c in range(n)]
            w0 = _stack([r["w0"] for r in rs], dev)
            w1 = _stack([r["w1"] for r in rs], dev)
            if kind == "joint":
                res = crsht.joint_step_batch(plan, fid, d, chains, [r["xi"] for r in rs], [r["u"] for r in rs], w0,
                                             w1, sigma_lnq=sigma_lnq, **solve_kw)
            else:
                res = crsht.gibbs_step_batch(plan, fid, d, chains, [r["g"] for r in rs], w0, w1, **solve_kw)
            for c, ch in enumerate(chains):
                acc[c, s] = res[c].accepted if kind == "joint" else True
                mi[c, s] = res[c].mean_stats.iters
                fi[c, s] = res[c].fluct_stats.iters
                q[c, s + 1] = ch.q
            continue
        for c, ch in enumerate(chains):
            r = draw(c, s)
            w0 = _on(r["w0"], dev)
            w1 = _on(r["w1"], dev)
            if kind == "joint":
                res = crsht.joint_step(plan, fid, d, ch, r["xi"], r["u"], w0, w1, sigma_lnq=sigma_lnq, **solve_kw)
                acc[c, s] = res.accepted
            else:
                res = crsht.gibbs_step(plan, fid, d, ch, r["g"], w0, w1, **solve_kw)
                acc[c, s] = True
            mi[c, s] = res.mean_stats.iters
            fi[c, s] = res.fluct_stats.iters
            q[c, s + 1] = ch.q
    lnq = np.log(q[:, 1 + burn:])
    iat = np.array([integrated_autocorr_time(x) for x in lnq])
    cl = np.array([correlation_length(x) for x in lnq])
    return ChainRun(kind, q, acc, mi, fi, acc.mean(axis=1), iat, cl)


def bin_scaled(fid: crsht.Problem, edges, theta) -> crsht.Problem:
    """fid with C_l exp(theta_k) on [edges[k], edges[k+1])."""
    f = np.ones(len(fid.cl))
    for k in range(len(edges) - 1):
        f[edges[k]:edges[k + 1]] = math.exp(theta[k])
    return crsht.Problem(np.asarray(fid.cl) * f, fid.bl, fid.ninv, fid.lmin)


def init_bin_chain(plan: crsht.Plan, fid: crsht.Problem, d: torch.Tensor, edges, theta, w0: torch.Tensor,
                   w1: torch.Tensor, **solve_kw) -> crsht.BinChain:
    """State at the log-amplitudes theta: mean field, fluctuation, ln pi."""
    p = bin_scaled(fid, edges, theta)
    ahat, _ = crsht.solve(plan, p, d, **solve_kw)
    fhat, _ = crsht.solve(plan, p, None, w0, w1, **solve_kw)
    ahat, fhat = ahat[0].clone(), fhat[0].clone()
    return crsht.BinChain(np.asarray(edges, dtype=np.int32), np.asarray(theta, dtype=np.float64).copy(),
                          crsht.lnpi(plan, p, 1.0, d, ahat, fhat), ahat, fhat)


def curvature_scale(plan: crsht.Plan, fid: crsht.Problem, d: torch.Tensor, chain: crsht.BinChain, h: float = 1e-3,
                    **solve_kw) -> np.ndarray:
    """Width of the HMC target along each bin, 1/sqrt(-d^2 ln pi/d theta_k^2),
    from a forward difference of the fixed-fluctuation gradient at the chain's
    state (nbins + 1 mean-field solves); a guide for the leapfrog step."""
    th = np.asarray(chain.theta, dtype=np.float64)
    g0 = crsht.lnpi_grad_fixed(plan, fid, d, chain.edges, th, th, chain.fhat, a0=chain.ahat, **solve_kw)[0]
    out = np.zeros(th.size)
    for k in range(th.size):
        t1 = th.copy()
        t1[k] += h
        g1 = crsht.lnpi_grad_fixed(plan, fid, d, chain.edges, th, t1, chain.fhat, a0=chain.ahat, **solve_kw)[0]
        c = -(g1[k] - g0[k]) / h
        out[k] = 1.0 / math.sqrt(c) if c > 0 else float("inf")
    return out


@dataclass
class HmcRun:
    theta: np.ndarray        # [nchains, nsteps + 1, nbins] after each move (start first)
    accepted: np.ndarray     # [nchains, nsteps]
    dH: np.ndarray           # [nchains, nsteps] energy error of each trajectory
    solves: np.ndarray       # [nchains, nsteps] mean-field solves of each trajectory
    iters: np.ndarray        # [nchains, nsteps] their iterations, summed
    fluct_iters: np.ndarray  # [nchains, nsteps]
    acceptance: np.ndarray   # [nchains]
    iat: np.ndarray          # [nchains, nbins] integrated autocorrelation time of theta_k (after burn-in)
    corr_len: np.ndarray     # [nchains, nbins] first lag with zeta(lag) < 0.1 of theta_k (after burn-in)

    def summary(self) -> dict:
        return {"kind": "hmc", "chains": int(self.theta.shape[0]), "steps": int(self.theta.shape[1] - 1),
                "bins": int(self.theta.shape[2]), "acceptance": float(self.acceptance.mean()),
                "iat_theta": float(self.iat.mean()), "corr_len_theta": float(self.corr_len.mean()),
                "mean_iters_per_solve":
                float(self.iters.sum() / max(self.solves.sum(), 1)), "abs_dH": float(np.abs(self.dH).mean())}


def default_hmc_draws(nbins: int, lmax: int, npix: int, seed: int):
    """Random numbers of each HMC move in a fixed order (numpy Generator
    seeded per chain): momentum p0 [nbins], u, w0, w1."""
    rngs = {}

    def draw(chain: int, step: int) -> dict:
        rng = rngs.setdefault(chain, np.random.default_rng([seed, chain, 1]))
        return {"p0": rng.standard_normal(nbins), "u": float(rng.uniform()), "w0": white_alm(rng, lmax),
                "w1": rng.standard_normal(npix)}

    return draw


def run_hmc(plan: crsht.Plan, fid: crsht.Problem, d: torch.Tensor, chains: list, nsteps: int, eps: float,
            nleap: int, seed: int = 0, burn: int = 0, draw: Optional[Callable[[int, int], dict]] = None,
            **solve_kw) -> HmcRun:
    """Advance every chain (crsht.BinChain, updated in place) by nsteps HMC
    moves of nleap leapfrog steps of size eps."""
    n = len(chains)
    nb = len(chains[0].edges) - 1
    if draw is None:
        draw = default_hmc_draws(nb, plan.lmax, plan.npix, seed)
    dev = d.device
    th = np.zeros((n, nsteps + 1, nb))
    acc = np.zeros((n, nsteps), dtype=bool)
    dh = np.zeros((n, nsteps))
    sv = np.zeros((n, nsteps), dtype=np.int64)
    it = np.zeros((n, nsteps), dtype=np.int64)
    fi = np.zeros((n, nsteps), dtype=np.int64)
    for c, ch in enumerate(chains):
        th[c, 0] = ch.theta
    for s in range(nsteps):
        for c, ch in enumerate(chains):
            r = draw(c, s)
            w0 = _on(r["w0"], dev)
            w1 = _on(r["w1"], dev)
            res = crsht.hmc_step(plan, fid, d, ch, r["p0"], r["u"], w0, w1, eps, nleap, **solve_kw)
            acc[c, s], dh[c, s], sv[c, s], it[c, s] = res.accepted, res.dH, res.solves, res.iters
            fi[c, s] = res.fluct_stats.iters
            th[c, s + 1] = ch.theta
    iat = np.array([[integrated_autocorr_time(th[c, 1 + burn:, k]) for k in range(nb)] for c in range(n)])
    cl = np.array([[correlation_length(th[c, 1 + burn:, k]) for k in range(nb)] for c in range(n)])
    return HmcRun(th, acc, dh, sv, it, fi, acc.mean(axis=1), iat, cl)


__all__ = ["white_alm", "integrated_autocorr_time", "autocorrelation", "correlation_length", "scaled", "init_chain",
           "ChainRun", "default_draws", "run_chains", "device_draws", "bin_scaled", "init_bin_chain", "curvature_scale", "HmcRun", "default_hmc_draws", "run_hmc"]
