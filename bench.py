#!/usr/bin/env python3
"""Benchmark: constrained-realization PCG solves/s and SHT pairs/s on one MI355X.

Workload (temperature, HEALPix Nside 512, lmax 1535): C_l = A/(l(l+1)) with a
100 uK pixel rms, Gaussian beam FWHM 10 arcmin, anisotropic white noise
sigma_p = 30 uK / sqrt(h_p) with h_p = 1 + 4 sin^2(ecliptic-like latitude),
N^-1 = 0 in the band |b| < 20 deg, data d = Y B a_true + n, fresh w0/w1 per
column. One step = one full constrained-realization solve (right-hand side
and all PCG iterations, per-m block preconditioner built once per noise model
before the timed steps) to a true relative residual of 1e-6 for `--nrhs`
independent columns at once. The default is the batched mixed-precision form
(16 columns, bf16x3 MFMA Legendre steps inside PCG with FP64 vectors, scalars
and residual replacement); `--prec f64` runs the plain FP64 form. Inputs are
resident on the GPU before timing starts; the timed steps replay each block of
check_every PCG iterations as a captured HIP graph; the per-kernel launch
times come from one extra solve with HIP events around every launch of the
tracked kernels.

Beside `value` the line carries, unless switched off: `forms` (the same solve
as plain FP64 PCG at the same 16 columns, as mixed PCG at 1 column and as
FP64 at 1 column, all to the same 1e-6 residual), `tqu_line` (T+Q+U, 2
columns) and `cpu_baseline` (the oracle on the host cores).

Other workloads: tqu, batched64 (64 uneven problems), chains (joint, Gibbs
and HMC moves), and the counter-run probes probe-operator, probe-precond and
copy. Prints one JSON line. --gpus N with N > 1 is refused: the benchmark
runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
FP64_VECTOR_PEAK_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP64_MATRIX_PEAK_TFLOPS = 78.6     # dense FP64 MFMA (MI355X datasheet)
BF16_MFMA_PEAK_TFLOPS = 2500.0     # dense
HBM_PEAK_GBS = 8000.0

# HBM traffic of a kernel per timed unit from rocprofv3 --pmc FETCH_SIZE /
# WRITE_SIZE runs of this script's probe workload probe-operator (--nrhs 16
# --prec mixed / f64) and, for k_pc_apply, of the headline solve itself (its
# FP32-z form), at Nside 512, scaled by the same counters on a 1 GiB copy
# (FETCH x 2.0, WRITE x 1.0); valid only for the 16-column temperature
# workload and while the kernel's source file hashes to `src`. (k_adj_mfma
# has none: the probe runs its plain form, the solve its PCG form, which
# also reads p and writes q.)
TRAFFIC = {
    "k_synth_mfma": {"bytes": 696603776, "src": "cf97a06e5dd06004"},
    "k_ring<float2, RING_FUSED>": {"bytes": 626375360, "src": "e3e614dbe0919562"},   # one pass (4 class launches)
    "k_legendre_synth_mfma": {"bytes": 2 * 679587920, "src": "4759d7b6f7f34de0"},  # one transform (2 launches)
    "k_legendre_adj_mfma": {"bytes": 4 * 464820008, "src": "4759d7b6f7f34de0"},  # one transform (2 x 2 launches)
    "k_pc_apply": {"bytes": 2389456395, "src": "648961bc9f2460e7"},   # solve form: FP32 z, <r, z> partials
}


def legendre_triples(nside: int, lmax: int, mmax: int) -> int:
    """(l, m, ring pair) points of one Legendre pass."""
    return sum(lmax - m + 1 for m in range(mmax + 1)) * (2 * nside)


def pick_nr(n: int) -> int:
    return 8 if n >= 8 else 4 if n >= 4 else 2 if n >= 2 else 1


def src_hash(rel: str) -> str:
    with open(os.path.join(ROOT, "paper_2306_15511_amd", "csrc", rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _oracle_threads() -> int:
    cores = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    return min(cores, int(env)) if env and env.isdigit() and int(env) > 0 else cores


def cpu_baseline(wl, iters: int, iters_src: str, tqu: bool = False):
    """The oracle on the host cores: one full SHT pair (synthesis + adjoint of
    one field) at the benchmark's Nside and lmax, with the oracle's plain-C
    Legendre sums and numpy FFTs; solves/s = 1/(s per pair x iterations).
    With tqu the pair also carries the spin-2 part on a bounded sample (the
    W, X rows of the numpy oracle on every 16th ring, scaled to all rings).
    Beside it, one whole oracle solve (right-hand side, block preconditioner
    set-up, PCG to 1e-6) of the same sky at Nside 128, lmax 383."""
    from oracle import sht as osht
    import crinputs as ci
    S = osht.SHT(wl.nside, wl.lmax, fast=True)
    a = ci.white_alm(np.random.default_rng(1), wl.lmax)
    x = np.random.default_rng(20).standard_normal(S.npix)
    t0 = time.perf_counter()
    S.synth(a)
    S.adjoint(x)
    t_pair = time.perf_counter() - t0
    sample = ("oracle SHT pair (plain-C Legendre sums + numpy FFT) at Nside %d, lmax %d, all %d rings: %.2f s"
              % (wl.nside, wl.lmax, S.rings.nrings, t_pair))
    if tqu:
        t_pair = t_pair + _spin2_sample_time(wl)
        sample += ("; T+Q+U: the T pair + the spin-2 rows of E, B (numpy oracle on every 16th ring, scaled) and "
                   "the Q, U FFTs: %.2f s" % t_pair)
    sample += "; solves/s = 1/(s per pair x %d iterations, %s)" % (iters, iters_src)
    out = {"value": 1.0 / (t_pair * max(iters, 1)), "unit": "solves/s", "cores": _oracle_threads(), "kind": "oracle",
           "sample": sample, "sht_pairs_per_s": 1.0 / t_pair}
    if not tqu:
        out["full_solve"] = _oracle_full_solve()
    return out


def _spin2_sample_time(wl) -> float:
    """Seconds of the spin-2 part of one T+Q+U SHT pair in the oracle: the
    (a_E, a_B) -> (Q, U) spectra of the numpy oracle on every 16th ring,
    scaled to all rings, twice (synthesis and transpose use the same W, X
    rows), plus the azimuthal FFTs of Q and U at full size."""
    from oracle import spin2
    import crinputs as ci
    pol = spin2.PolSHT(wl.nside, wl.lmax)
    R = pol.s.rings
    sel = np.arange(0, R.nrings, 16)
    aE, aB = (ci.white_alm(np.random.default_rng(2 + k), wl.lmax) for k in range(2))
    t0 = time.perf_counter()
    GQ, GU = pol.spectra(aE, aB, sel)
    t_rows = (time.perf_counter() - t0) * R.nrings / sel.size
    F = np.zeros((pol.mmax + 1, R.nrings), dtype=np.complex128)
    x = np.random.default_rng(21).standard_normal(pol.npix)
    t0 = time.perf_counter()
    pol.s.phi_synth(F)
    pol.s.phi_adjoint(x)
    t_fft = time.perf_counter() - t0
    return 2.0 * t_rows + 2.0 * t_fft


def _oracle_full_solve(nside: int = 128) -> dict:
    """One complete oracle constrained-realization solve (d, w0, w1 terms,
    right-hand side, per-m block preconditioner, PCG to 1e-6) of the
    benchmark's sky at a smaller Nside."""
    from oracle import cr, healpix
    from oracle import sht as osht
    from oracle.block_pc import BlockPreconditioner
    import crinputs as ci
    wl = ci.workload_masked_t(nside, 3 * nside - 1, fwhm_arcmin=10.0 * 512 / nside, cfg=2)
    z, phi = healpix.pixel_coords(nside)
    t0 = time.perf_counter()
    S = osht.SHT(nside, wl.lmax, fast=True)
    P = cr.Problem(nside, wl.lmax, wl.cl(), wl.bl(), wl.ninv(z, phi))
    op = cr.CROperator(P, S)
    d = S.synth(op.b * wl.signal()) + wl.noise(z, phi)
    t1 = time.perf_counter()
    b = op.rhs(d, wl.w0(), wl.w1())
    pc = BlockPreconditioner(op)
    x, info = cr.pcg(op, b, 1e-6, 2000, precond=pc)
    t2 = time.perf_counter()
    return {"nside": nside, "lmax": wl.lmax, "s": t2 - t1, "solves_per_s": 1.0 / (t2 - t1), "iters": info.iters,
            "rel_resid_true": info.rel_resid_true, "inputs_s": t1 - t0, "cores": _oracle_threads(),
            "what": "oracle CR solve of the benchmark sky (hit pattern, |b|<20deg, FWHM 10' x 512/Nside): "
                    "right-hand side + block preconditioner set-up + PCG to 1e-6, timed whole"}


def bench_batched(args):
    """64 independent T-only problems (16 each at Nside 64, 128, 256, 512,
    lmax = 3 Nside - 1; amplitude, white-noise level and band mask drawn per
    problem) in one cr_solve_batched call; one JSON line (solves/s)."""
    import torch
    from paper_2306_15511_amd import crsht
    import crinputs as ci
    dev = torch.device("cuda:0")
    plans, probs, D, W0, W1 = [], [], [], [], []
    for j in range(64):
        wl = ci.workload_batched(j)
        pl = crsht.Plan(wl.nside, wl.lmax)
        z, phi = pl.pixel_coords()
        ls, _ = ci.alm_lm_arrays(wl.lmax)
        cl, bl = wl.cl(), wl.bl()
        a = torch.from_numpy(bl[ls] * wl.signal()).to(dev)
        d = crsht.synth(pl, a) + torch.from_numpy(wl.noise(z, phi)).to(dev)
        plans.append(pl)
        probs.append(crsht.Problem(cl, bl, torch.from_numpy(wl.ninv(z, phi)).to(dev), 2))
        D.append(d)
        W0.append(torch.from_numpy(wl.w0()).to(dev))
        W1.append(torch.from_numpy(wl.w1()).to(dev))
    prec = crsht.CR_MIXED if args.prec == "mixed" else crsht.CR_F64
    use_block = (args.precond or "block") == "block"
    pc_setup_s = None
    if use_block:
        # per-m block preconditioner of every problem (each has its own noise
        # model), built once before the timed steps like the headline's
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pl, pr in zip(plans, probs):
            crsht.block_precond_build(pl, pr)
        torch.cuda.synchronize()
        pc_setup_s = time.perf_counter() - t0
    ce = args.check_every or (6 if use_block else 16)
    torch.cuda.synchronize()

    def step():
        return crsht.solve_batched(plans, probs, D, W0, W1, tol=args.tol, prec=prec, check_every=ce,
                                   inner_tol=args.inner_tol,
                                   precond=crsht.CR_PC_BLOCK if use_block else crsht.CR_PC_JACOBI)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        _, st = step()
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = 64 * args.steps
    res = {
        "metric": "batched constrained-realization solves/s (64 uneven problems, Nside 64-512)",
        "value": n / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3+f64" if prec == crsht.CR_MIXED else "f64", "data": "synthetic",
        "config": {"workload": "64 independent T-only CR solves, 16 each at Nside 64/128/256/512, lmax 3 Nside - 1, "
                               "amplitude U[0.5,2] A, white sigma U[5,50] uK, band mask f U[0,0.3], true residual %g"
                               % args.tol, "nprob": 64, "tol": args.tol,
                   "preconditioner": "per-m blocks (built once per noise model)" if use_block else "Jacobi"},
        "iters_per_solve": sum(x.iters for st in stats for x in st) / n,
        "rel_resid_true_max": max(x.rel_resid_true for st in stats for x in st),
        "all_converged": all(x.status == 0 for st in stats for x in st),
    }
    if pc_setup_s is not None:
        res["precond_setup_s"] = pc_setup_s
    print(json.dumps(res))


def bench_chains(args):
    """Joint (C_l amplitude, sky) moves against standard Gibbs moves and HMC
    moves of ln q on the headline sky (Nside 512, lmax 1535, hit-pattern
    noise, band mask, FWHM 10'): --chains chains advanced --steps moves each
    by the three samplers (mixed precision, per-m block preconditioner built
    once, warm-started mean fields); one JSON line with moves/s of the joint
    sampler as `value` and every sampler's acceptance, ln q autocorrelation
    time, moves per autocorrelation time per second and iterations."""
    import torch
    from paper_2306_15511_amd import chains, crsht
    import crinputs as ci
    nside = args.nside
    lmax = 3 * nside - 1 if args.lmax is None else args.lmax
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=10.0, cfg=2)
    dev = torch.device("cuda:0")
    plan = crsht.Plan(nside, lmax, nrhs_max=max(1, 2 * args.chains))
    z, phi = plan.pixel_coords()
    cl, bl = wl.cl(), wl.bl()
    ls, _ = ci.alm_lm_arrays(lmax)
    a = torch.from_numpy(bl[ls] * ci.signal_alm(ci.rng_for(2, 0, ci.STREAM_SIGNAL), cl, lmax)).to(dev)
    ns = args.noise_scale   # noise level relative to the headline sky (N -> ns^2 N)
    d = crsht.synth(plan, a) + torch.from_numpy(ns * wl.sigma_map(z, phi) *
                                                ci.white_map(ci.rng_for(2, 0, ci.STREAM_NOISE), wl.npix)).to(dev)
    fid = crsht.Problem(cl, bl, torch.from_numpy(wl.ninv(z, phi) / (ns * ns)).to(dev), 2)
    crsht.block_precond_build(plan, fid)
    kw = dict(tol=args.tol, prec=crsht.CR_MIXED if args.prec == "mixed" else crsht.CR_F64,
              inner_tol=args.inner_tol, precond=crsht.CR_PC_BLOCK)
    out = {}
    for name, kind, batched in (("joint", "joint", False), ("joint_batched", "joint", True),
                                ("gibbs", "gibbs", False), ("gibbs_batched", "gibbs", True)):
        rng = np.random.default_rng([11, 0])
        ch = [chains.init_chain(plan, fid, d, 1.0, torch.from_numpy(chains.white_alm(rng, lmax)).to(dev),
                                torch.from_numpy(rng.standard_normal(plan.npix)).to(dev), **kw)
              for _ in range(args.chains)]
        alpha = crsht.gibbs_shape(lmax, 2)
        chains.run_chains(plan, fid, d, ch, args.warmup, kind=kind, batched=batched,
                          draw=chains.device_draws(plan, kind, alpha, seed=1), **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run = chains.run_chains(plan, fid, d, ch, args.steps, kind=kind, batched=batched,
                                draw=chains.device_draws(plan, kind, alpha, seed=2), **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = dict(run.summary(), moves_per_s=args.chains * args.steps / dt, s=dt,
                         fluct_iters=float(run.fluct_iters.mean()))
        print("%s: %.1f moves/s, acceptance %.3f, iat ln q %.2f, correlation length %.1f"
              % (name, out[name]["moves_per_s"], out[name]["acceptance"], out[name]["iat_lnq"],
                 out[name]["corr_len_lnq"]), file=sys.stderr, flush=True)
    # HMC on theta = ln q (one bin over every kept l): step from the target's
    # curvature at the start (half its width), trajectories of three steps
    edges = [2, lmax + 1]
    rng = np.random.default_rng([11, 0])
    ch = [chains.init_bin_chain(plan, fid, d, edges, [0.0], torch.from_numpy(chains.white_alm(rng, lmax)).to(dev),
                                torch.from_numpy(rng.standard_normal(plan.npix)).to(dev), **kw)
          for _ in range(args.chains)]
    sig = float(chains.curvature_scale(plan, fid, d, ch[0], **kw)[0])
    eps, nleap = 0.5 * sig, 3
    chains.run_hmc(plan, fid, d, ch, args.warmup, eps, nleap, draw=chains.device_draws(plan, "hmc", seed=1), **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run = chains.run_hmc(plan, fid, d, ch, args.steps, eps, nleap, draw=chains.device_draws(plan, "hmc", seed=2),
                         **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["hmc"] = dict(run.summary(), moves_per_s=args.chains * args.steps / dt, s=dt, eps=eps, nleap=nleap,
                      width_lnq=sig, fluct_iters=float(run.fluct_iters.mean()))
    for kind in out:
        it = out[kind]["iat_theta"] if kind == "hmc" else out[kind]["iat_lnq"]
        out[kind]["eff_moves_per_s"] = out[kind]["moves_per_s"] / it
    res = {
        "metric": "joint C_l-amplitude / sky moves/s (Nside 512, lmax 1535)",
        "value": out["joint_batched"]["moves_per_s"], "unit": "moves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": out["joint_batched"]["s"] / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3+f64" if args.prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "%d chains, joint moves (sigma ln q 0.02; value: all chains moved in one batched "
                               "call per step, also one chain after another), standard Gibbs moves and HMC moves of "
                               "ln q (Gibbs moves also batched), T-only, Nside %d, "
                               "lmax %d, hit-pattern noise, |b|<20deg mask, FWHM 10', true residual %g, per-m block "
                               "preconditioner, warm-started mean fields, w0 and w1 drawn on the device (Philox4x32-10), "
                               "noise x %g" % (args.chains, nside, lmax, args.tol, args.noise_scale),
                   "chains": args.chains},
        "joint": out["joint"], "joint_batched": out["joint_batched"], "gibbs": out["gibbs"],
        "gibbs_batched": out["gibbs_batched"], "hmc": out["hmc"],
    }
    print(json.dumps(res))


def probe(args):
    """Short fixed workloads for hardware-counter runs (rocprofv3 --pmc):
    probe-operator applies the CR operator --reps times on the benchmark sky
    (FP64 or mixed, --nrhs columns, --ncomp 1 or 3); probe-precond builds the
    per-m block preconditioner and applies it --reps times; copy copies a
    float64 buffer of --mib MiB --reps times (calibration of FETCH_SIZE /
    WRITE_SIZE against exact bytes)."""
    import torch
    dev = torch.device("cuda:0")
    if args.workload == "copy":
        n = args.mib * 1024 * 1024 // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.reps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied %d bytes x %d" % (n * 8, args.reps))
        return
    import crinputs as ci
    from paper_2306_15511_amd import crsht
    nside = args.nside
    lmax = 3 * nside - 1 if args.lmax is None else args.lmax
    ncomp = args.ncomp
    nrhs = args.nrhs or 16
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=10.0, cfg=2)
    plan = crsht.Plan(nside, lmax, nrhs_max=nrhs, ncomp=ncomp)
    z, phi = plan.pixel_coords()
    nt = wl.ninv(z, phi)
    if ncomp == 3:
        cl = np.ascontiguousarray(ci.cl_tqu(lmax, wl.amp, 0.3))
        prob = crsht.Problem(cl, wl.bl(), torch.from_numpy(np.stack([nt, nt / 2.0, nt / 2.0])).to(dev), 2)
    else:
        prob = crsht.Problem(wl.cl(), wl.bl(), torch.from_numpy(nt).to(dev), 2)
    rng = np.random.default_rng(0)
    x = np.stack([ci.white_alm(rng, lmax) for _ in range(nrhs * ncomp)])
    x = torch.from_numpy(x.reshape(plan.alm_shape(nrhs))).to(dev)
    if args.workload == "probe-precond":
        crsht.block_precond_build(plan, prob)
        for _ in range(args.reps):
            crsht.block_precond_apply(plan, x)
        torch.cuda.synchronize()
        print("applied block preconditioner x %d at nside %d, %d columns" % (args.reps, nside, nrhs))
    else:
        prec = crsht.CR_MIXED if args.prec == "mixed" else crsht.CR_F64
        for _ in range(args.reps):
            crsht.apply(plan, prob, x, prec=prec)
        torch.cuda.synchronize()
        print("applied operator x %d at nside %d, %d columns, %s" % (args.reps, nside, nrhs, args.prec))
    plan.close()


def solve_line(args, tqu: bool, R: int, steps: int, warmup: int, compare: bool, kernels: bool = True):
    """One solve workload on the benchmark sky (T only, or T+Q+U with C^EE =
    0.05 C^TT, C^BB = 0.005 C^TT, TE correlation 0.3, sigma_QU = sqrt(2)
    sigma_T): inputs resident in HBM, `warmup` untimed and `steps` timed
    solves of R columns. Returns the result dict (value = solves/s)."""
    import torch
    from paper_2306_15511_amd import crsht
    import crinputs as ci

    nside = args.nside
    lmax = 3 * nside - 1 if args.lmax is None else args.lmax
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=10.0, cfg=2)
    wl.tol = args.tol
    inner_tol = args.inner_tol if args.inner_tol is not None else (1e-2 if tqu else 1e-3)
    nc = 3 if tqu else 1
    mixed = args.prec == "mixed"
    dev = torch.device("cuda:0")
    plan = crsht.Plan(nside, lmax, nrhs_max=R, ncomp=nc)
    z, phi = plan.pixel_coords()
    bl = wl.bl()
    ls, _ = ci.alm_lm_arrays(lmax)
    sig = wl.sigma_map(z, phi)
    if tqu:
        cl = ci.cl_tqu(lmax, wl.amp, 0.3)
        nt = wl.ninv(z, phi)
        ninv = torch.from_numpy(np.stack([nt, nt / 2.0, nt / 2.0])).to(dev)
        A = np.stack([bl[ls] * ci.signal_alm_tqu(ci.rng_for(2, c, ci.STREAM_SIGNAL), cl, lmax) for c in range(R)])
        noise = np.stack([np.stack([f * sig * ci.white_map(ci.rng_for(2, c, ci.STREAM_NOISE + 10 * k), wl.npix)
                                    for k, f in enumerate((1.0, 2 ** 0.5, 2 ** 0.5))]) for c in range(R)])
        w0 = np.stack([np.stack([ci.white_alm(ci.rng_for(2, c, ci.STREAM_W0 + 10 * k), lmax) for k in range(3)])
                       for c in range(R)])
        w1 = np.stack([np.stack([ci.white_map(ci.rng_for(2, c, ci.STREAM_W1 + 10 * k), wl.npix) for k in range(3)])
                       for c in range(R)])
    else:
        cl = wl.cl()
        ninv = torch.from_numpy(wl.ninv(z, phi)).to(dev)
        A = np.stack([bl[ls] * ci.signal_alm(ci.rng_for(2, c, ci.STREAM_SIGNAL), cl, lmax) for c in range(R)])
        noise = np.stack([sig * ci.white_map(ci.rng_for(2, c, ci.STREAM_NOISE), wl.npix) for c in range(R)])
        w0 = np.stack([ci.white_alm(ci.rng_for(2, c, ci.STREAM_W0), lmax) for c in range(R)])
        w1 = np.stack([ci.white_map(ci.rng_for(2, c, ci.STREAM_W1), wl.npix) for c in range(R)])
    amp = None
    if args.chain_columns:
        # columns 2k and 2k+1: mean field and fluctuation of chain k at its
        # own amplitude q_k ~ U[0.8, 1.25] (C_l -> q_k C_l)
        if R % 2:
            sys.exit("bench.py: --chain-columns needs an even --nrhs")
        amp = np.repeat(ci.rng_for(4, 0, ci.STREAM_PARAMS).uniform(0.8, 1.25, R // 2), 2)
        noise[1::2] = 0.0
        A[1::2] = 0.0
        w0[0::2] = 0.0
        w1[0::2] = 0.0
    prob = crsht.Problem(cl, bl, ninv, 2, amp)
    tuning = None
    if not args.no_tune:
        # tile shapes for this plan, column count and precision (set-up, like the preconditioner)
        tuning = crsht.autotune(plan, R, crsht.CR_MIXED if args.prec == "mixed" else crsht.CR_F64)
        print("tile shapes: %s" % tuning, file=sys.stderr, flush=True)
    use_block = (args.precond or "block") == "block"
    ce = args.check_every or (6 if use_block else 16)
    pc = crsht.CR_PC_BLOCK if use_block else crsht.CR_PC_JACOBI
    pc_setup_s = None
    if use_block:
        # per noise model (plan-level precomputation): timed, reported, outside the solve steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        crsht.block_precond_build(plan, crsht.Problem(cl, bl, ninv, 2))
        pc_setup_s = time.perf_counter() - t0
        print("block preconditioner built in %.2f s" % pc_setup_s, file=sys.stderr, flush=True)
    # inputs: d = Y B a_true + n per column (synthesised on the GPU), w0, w1
    d = crsht.synth(plan, torch.from_numpy(A).to(dev))
    d += torch.from_numpy(noise).to(dev)
    w0 = torch.from_numpy(w0).to(dev)
    w1 = torch.from_numpy(w1).to(dev)
    del A, noise
    out = torch.empty(plan.alm_shape(R), dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()

    prec = crsht.CR_MIXED if mixed else crsht.CR_F64

    def solve(n, p, o):
        return crsht.solve(plan, prob if n == R else crsht.Problem(cl, bl, ninv, 2, None if amp is None else amp[:n]),
                           d[:n], w0[:n], w1[:n], nrhs=n, tol=wl.tol, maxiter=20000, out=o, check_every=ce, prec=p,
                           inner_tol=inner_tol, precond=pc)

    def timed_form(n, p, reps, label):
        """warm-up solve (captures the graphs) and `reps` timed solves of n columns"""
        o = out[:n]
        solve(n, p, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, st = solve(n, p, o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        r = {"form": label, "nrhs": n, "solves_per_s": n / t, "ms_per_solve_call": t * 1e3,
             "iters_per_solve": sum(x.iters for x in st) / n,
             "rel_resid_true_max": max(x.rel_resid_true for x in st),
             "all_converged": all(x.status == 0 for x in st)}
        print("%s: %.2f solves/s, iters %s" % (label, r["solves_per_s"], [x.iters for x in st]), file=sys.stderr,
              flush=True)
        return r

    for _ in range(warmup):
        _, st = solve(R, prec, out)
        print("warmup: iters %s resid %s" % ([x.iters for x in st], ["%.2e" % x.rel_resid_true for x in st]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        _, st = solve(R, prec, out)
        stats.append(st)
        print("step %d: iters %s refinements %s resid %s" % (k, [x.iters for x in st], [x.refinements for x in st],
                                                             ["%.2e" % x.rel_resid_true for x in st]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves = steps * R
    tot_iters = sum(sum(x.iters for x in st) for st in stats)
    what = ("T+Q+U (spin-0 and spin-2) constrained-realization PCG solve, C^EE = 0.05 C^TT, C^BB = 0.005 C^TT, "
            "TE correlation 0.3, sigma_QU = sqrt(2) sigma_T" if tqu else "T-only constrained-realization PCG solve")
    res = {
        "metric": "constrained-realization CG solves/s at Nside=512, lmax=1535; SHT pairs/s",
        "value": solves / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": dt / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "%s, Nside %d, lmax %d, hit-pattern noise, "
                               "|b|<20deg mask, FWHM 10', true residual %g, %d columns per solve, %s"
                               % (what, nside, lmax, wl.tol, R, "bf16x3 MFMA Legendre + FP64 vectors and residual "
                                  "replacement" if mixed else "FP64"),
                   "nside": nside, "lmax": lmax, "nrhs": R, "ncomp": nc, "tol": wl.tol, "inner_tol": inner_tol,
                   "check_every": ce,
                   "preconditioner": "per-m blocks (built once per noise model)" if use_block else "Jacobi",
                   "precision": "CR_MIXED" if mixed else "CR_F64"},
        "sht_pairs_per_s": tot_iters * nc / dt,
        "iters_per_solve": tot_iters / solves,
        "rel_resid_true_max": max(x.rel_resid_true for st in stats for x in st),
        "all_converged": all(x.status == 0 for st in stats for x in st),
    }
    if tqu:
        res["config"]["sht_pairs_note"] = "one SHT pair per field: 3 per T+Q+U column and iteration"
    if amp is not None:
        res["config"]["workload"] += ("; the columns are %d chains x (mean field, fluctuation), chain k at "
                                      "C_l q_k, q_k ~ U[0.8, 1.25]" % (R // 2))
        res["config"]["chain_amplitudes"] = [float(v) for v in amp[::2]]
    if pc_setup_s is not None:
        res["precond_setup_s"] = pc_setup_s
        pb, nb, nh = plan.precond_info()
        res["precond_storage"] = {"bytes": pb, "blocks": nb, "fp16_blocks": nh}
    if tuning is not None:
        res["tile_shapes"] = tuning
    if kernels:
        res.update(kernel_roofline(args, plan, lambda: solve(R, prec, out), nside, lmax, R, nc, mixed, use_block, tqu))
    if compare:
        # the comparison forms at the same residual, preconditioner and sky
        forms = {}
        if mixed:
            forms["f64_same_columns"] = timed_form(R, crsht.CR_F64, 1, "plain FP64 PCG, %d columns" % R)
            if R > 1:
                forms["mixed_1_column"] = timed_form(1, crsht.CR_MIXED, 3, "mixed PCG, 1 column")
        forms["f64_1_column"] = timed_form(1, crsht.CR_F64, 1, "plain FP64 PCG, 1 column")
        res["forms"] = forms
        res["transforms"] = transform_rates(plan, R, nc, lmax, dev)
    plan.close()
    return res


def transform_rates(plan, R: int, nc: int, lmax: int, dev):
    """SHT pairs/s (synthesis + adjoint of R columns, inputs resident) per
    precision: FP64, bf16x3 (the PCG inner operator) and bf16x6 (the
    user-visible reduced-precision transforms)."""
    import torch
    from paper_2306_15511_amd import crsht
    import crinputs as ci
    rng = np.random.default_rng([7, R])
    a = np.stack([ci.white_alm(rng, lmax) for _ in range(R * nc)]).reshape(plan.alm_shape(R))
    A = torch.from_numpy(a).to(dev)
    mp = crsht.synth(plan, A)
    al = torch.empty_like(A)
    out = {}
    for name, prec in (("f64", crsht.CR_F64), ("bf16x3", crsht.CR_MIXED), ("bf16x6", crsht.CR_BF16X6)):
        crsht.synth(plan, A, out=mp, prec=prec)
        crsht.adjoint(plan, mp, out=al, prec=prec)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            crsht.synth(plan, A, out=mp, prec=prec)
            crsht.adjoint(plan, mp, out=al, prec=prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"ms_per_pair_call": dt * 1e3, "sht_pairs_per_s": R * nc / dt}
    return out


def kernel_roofline(args, plan, one_solve, nside, lmax, R, nc, mixed, use_block, tqu):
    """per-kernel launch times: one more (untimed) solve with HIP events
    around every launch of the tracked kernels (direct launches, no graph
    replay), and the roofline fraction of each against its algorithmic work"""
    from paper_2306_15511_amd import crsht
    crsht.timing_enable(plan, True)
    _, st = one_solve()
    tm = {k: crsht.timing_read(plan, k) for k in range(7)}
    crsht.timing_enable(plan, False)
    print("kernel-timing step: iters %s" % [x.iters for x in st], file=sys.stderr, flush=True)
    # algorithmic work per timed unit (one launch; an FP64 adjoint unit is a whole transform)
    T = legendre_triples(nside, lmax, lmax)
    # Legendre sums of one column (E and O, complex): float2 in the mixed
    # operator's ring pass, double2 in the FP64 one (the FP64 operator, and the
    # true residuals of the mixed path)
    eo32 = 2 * nside * (lmax + 1) * 2 * 8
    # scalar Legendre columns per transform: a T+Q+U column is 9 in the
    # synthesis and 7 in the adjoint; the ring pass sees nc maps per column
    cs, ca = (9 * R, 7 * R) if tqu else (R, R)
    # the FP32 fused pass of T plans reads and writes the sums only at the
    # (ring pair, m) where the pair's Legendre values are live (E and O,
    # float2 each)
    eo32_pass = 2 * plan.live_pair_m * 2 * 8 if not tqu else 2 * eo32
    kinfo = {
        2: ("k_ring<float2, RING_FUSED> (azimuthal FFT pass, N^-1 fused, FP32)", "hbm",
            nc * R * eo32_pass + nc * plan.npix * 8, HBM_PEAK_GBS, "GB/s", "ring.hip"),
        6: ("k_ring<double2, RING_FUSED> (azimuthal FFT pass, N^-1 fused, FP64)", "hbm",
            nc * R * 2 * 2 * eo32 + nc * plan.npix * 8, HBM_PEAK_GBS, "GB/s", "ring.hip"),
    }
    if mixed:
        # average work per launch: columns go in launches of at most 16
        kinfo[3] = ("k_synth_mfma (bf16x3 MFMA Legendre synthesis)", "mfma", 4 * T * cs / -(-cs // 16),
                    BF16_MFMA_PEAK_TFLOPS, "TFLOP/s", "legendre_mfma.hip")
        kinfo[4] = ("k_adj_mfma (bf16x3 MFMA Legendre adjoint; in the solve also q and <p, q>)", "mfma", 4 * T * ca / -(-ca // 16),
                    BF16_MFMA_PEAK_TFLOPS, "TFLOP/s", "legendre_mfma.hip")

    # FP64 Legendre kernels: the plain path, and in the mixed path the FP64
    # true residuals of the refinement and the right-hand side; with two or
    # more columns they run on the FP64 matrix cores in launches of up to 8
    # columns (FP64 vector units for a single column)
    def fp64_groups(n):
        return [min(8, n - c) for c in range(0, n, 8)] if n >= 2 else [1]
    gs, ga = fp64_groups(cs), fp64_groups(ca)
    f64m = cs >= 2
    kinfo[0] = ("k_legendre_synth_mfma (FP64 MFMA Legendre synthesis, whole transform)" if f64m
                else "k_legendre_synth (FP64 VALU)",
                "mfma" if f64m else "alu", sum((3 + 4 * g) * T for g in gs) / (1 if f64m else len(gs)),
                FP64_MATRIX_PEAK_TFLOPS if f64m else FP64_VECTOR_PEAK_TFLOPS, "TFLOP/s", "legendre.hip")
    kinfo[1] = ("k_legendre_adj_mfma (FP64 MFMA Legendre adjoint, whole transform)" if ca >= 2
                else "k_legendre_adj (FP64 VALU, whole transform)", "mfma" if ca >= 2 else "alu",
                sum((3 + 4 * g) * T for g in ga),
                FP64_MATRIX_PEAK_TFLOPS if ca >= 2 else FP64_VECTOR_PEAK_TFLOPS, "TFLOP/s", "legendre.hip")
    if use_block:
        # the n x n entries of the stored scaled inverses (FP16 or FP32 per
        # block, as the build chose) + their FP32 diagonal scales + r read
        # (FP64) + z written (FP32 in the mixed T solve, else FP64)
        pcb = plan.precond_info()[0]
        zb = 8 if (mixed and not tqu) else 16
        kinfo[5] = ("k_pc_apply (block preconditioner, FP16 blocks on FP16 MFMA, FP32 blocks on FP32 MFMA)", "hbm",
                    pcb + 4 * plan.vlen + R * plan.vlen * (16 + zb), HBM_PEAK_GBS, "GB/s", "blockpc.hip")
    roofs = {}
    for kid, (name, bound, work, peak, unit, src) in kinfo.items():
        ms, nl = tm[kid]
        if nl == 0:
            continue
        avg = ms / nl * 1e-3
        achieved = work / avg / (1e9 if unit == "GB/s" else 1e12)
        tr = TRAFFIC.get(name.split(" (")[0]) if (not tqu and R == 16 and nside == 512) else None
        traffic = None
        if tr is not None and tr["src"] == src_hash(src):
            traffic = tr["bytes"]
        roofs[name] = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                       "traffic": traffic, "work_per_launch": work, "avg_launch_ms": avg * 1e3,
                       "launches": nl, "total_ms": ms}
    dom = max(roofs, key=lambda k: roofs[k]["total_ms"])
    roof = dict(roofs[dom])
    roof["kernel"] = dom
    return {"roofline": roof, "kernels": roofs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nrhs", type=int, default=None, help="columns per solve (default 16; 2 for --workload tqu)")
    ap.add_argument("--nside", type=int, default=512)
    ap.add_argument("--lmax", type=int, default=None)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=None,
                    help="PCG iterations between host convergence checks (default 6 with the block "
                         "preconditioner, 16 with Jacobi)")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="mixed path: FP64 residual replacement each time the residual fell by this factor "
                         "(default 1e-3; 1e-2 for T+Q+U, the faster setting measured for each)")
    ap.add_argument("--prec", choices=["f64", "mixed"], default="mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64-compare", action="store_true",
                    help="headline: skip the FP64 and single-column comparison forms")
    ap.add_argument("--no-tqu-line", action="store_true", help="headline: skip the T+Q+U line")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tile shapes (no crsht_autotune before the timed steps)")
    ap.add_argument("--workload", choices=["headline", "tqu", "batched64", "chains", "probe-operator",
                                           "probe-precond", "copy"], default="headline")
    ap.add_argument("--chains", type=int, default=4, help="--workload chains: number of chains")
    ap.add_argument("--noise-scale", type=float, default=1.0,
                    help="--workload chains: noise standard deviation relative to the headline sky")
    ap.add_argument("--chain-columns", action="store_true",
                    help="headline/tqu: the columns are the mean-field and fluctuation systems of nrhs/2 chains, "
                         "each at its own amplitude q ~ U[0.8, 1.25] (one solve for all)")
    ap.add_argument("--precond", choices=["block", "jacobi"], default=None,
                    help="default: block (per-m blocks, one set per component)")
    ap.add_argument("--ncomp", type=int, choices=[1, 3], default=1, help="probe workloads: 3 = T+Q+U")
    ap.add_argument("--reps", type=int, default=3, help="probe workloads: repetitions")
    ap.add_argument("--mib", type=int, default=1024, help="copy: buffer size in MiB")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark measures one GPU only; --gpus %d is not supported "
              "(independent chains would shard one per GPU with no communication)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload in ("probe-operator", "probe-precond", "copy"):
        probe(args)
        return
    if args.workload == "batched64":
        if args.inner_tol is None:
            args.inner_tol = 1e-3
        bench_batched(args)
        return
    if args.workload == "chains":
        if args.inner_tol is None:
            args.inner_tol = 1e-3
        bench_chains(args)
        return
    tqu = args.workload == "tqu"
    R = args.nrhs if args.nrhs else (2 if tqu else 16)
    res = solve_line(args, tqu, R, args.steps, args.warmup, compare=not args.no_f64_compare)
    if not tqu and not args.no_tqu_line:
        # the second line: T+Q+U, 2 columns, same sky (one warm-up, two timed solves)
        t = solve_line(args, True, 2, 2, 1, compare=False, kernels=False)
        res["tqu_line"] = {k: t[k] for k in ("value", "unit", "ms_per_step", "steps", "dtype", "config",
                                             "sht_pairs_per_s", "iters_per_solve", "rel_resid_true_max",
                                             "all_converged", "precond_setup_s") if k in t}
    if not args.no_cpu_baseline:
        f1 = res.get("forms", {}).get("f64_1_column")
        if f1 is not None:
            it, src = int(round(f1["iters_per_solve"])), "the FP64 GPU solve's count for one column"
        else:
            it, src = int(round(res["iters_per_solve"])), "the benchmarked solves' mean count"
        res["cpu_baseline"] = cpu_baseline(ci_workload(args), it, src, tqu)
    print(json.dumps(res))


def ci_workload(args):
    import crinputs as ci
    nside = args.nside
    lmax = 3 * nside - 1 if args.lmax is None else args.lmax
    return ci.workload_masked_t(nside, lmax, fwhm_arcmin=10.0, cfg=2)


if __name__ == "__main__":
    main()
