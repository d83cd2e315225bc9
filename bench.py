#!/usr/bin/env python3
"""Benchmark: constrained-realization PCG solves/s and SHT pairs/s on one MI355X.

Workload (temperature, HEALPix Nside 512, lmax 1535): C_l = A/(l(l+1)) with a
100 uK pixel rms, Gaussian beam FWHM 10 arcmin, anisotropic white noise
sigma_p = 30 uK / sqrt(h_p) with h_p = 1 + 4 sin^2(ecliptic-like latitude),
N^-1 = 0 in the band |b| < 20 deg, data d = Y B a_true + n, fresh w0/w1; one
step = one full constrained-realization solve (right-hand side, Jacobi
diagonal and all PCG iterations, FP64) to relative residual 1e-6, for
`--nrhs` independent columns at once. Inputs are resident on the GPU before
timing starts.

Prints one JSON line (see the keys below). --gpus N with N > 1 is refused:
this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0


def legendre_triples(nside: int, lmax: int, mmax: int) -> int:
    """(l, m, ring pair) points of one Legendre pass."""
    return sum(lmax - m + 1 for m in range(mmax + 1)) * (2 * nside)


def cpu_baseline(wl, iters: int):
    """Oracle (numpy FP64) SHT pair on a bounded sample: the Legendre and
    azimuthal steps of one synthesis + adjoint restricted to every 8th ring
    pair, scaled to the full ring count; solves/s = 1/(t_pair * iters)."""
    from oracle import sht as osht
    from oracle.legendre import lambda_rows
    import crinputs as ci
    S = osht.SHT(wl.nside, wl.lmax)
    R = S.rings
    nr = R.nrings
    sel = np.arange(0, nr, 16)        # 1 in 16 rings = 1 in 8 ring pairs
    a = ci.white_alm(np.random.default_rng(1), wl.lmax)
    x = np.random.default_rng(2).standard_normal(S.npix)
    t0 = time.perf_counter()
    # Legendre synthesis on the sampled rings
    z, st = R.z[sel], R.sin_theta[sel]
    F = np.zeros((S.mmax + 1, sel.size), dtype=np.complex128)
    for l, lam in lambda_rows(S.lmax, S.mmax, z, st):
        top = lam.shape[0] - 1
        F[:top + 1] += lam * a[S._idx(l, top)][:, None]
    # azimuthal synthesis + adjoint on the sampled rings
    m = np.arange(S.mmax + 1)
    G = np.empty_like(F)
    for j, k in enumerate(sel):
        n, f0 = int(R.nphi[k]), int(R.first[k])
        c = np.zeros(n, dtype=np.complex128)
        np.add.at(c, m % n, np.where(m == 0, 1.0, 2.0) * F[:, j] * np.exp(1j * m * R.phi0[k]))
        _ = (n * np.fft.ifft(c)).real
        X = np.fft.fft(x[f0:f0 + n])
        G[:, j] = np.exp(-1j * m * R.phi0[k]) * X[m % n]
    # Legendre adjoint on the sampled rings
    out = np.zeros(S.nalm, dtype=np.complex128)
    for l, lam in lambda_rows(S.lmax, S.mmax, z, st):
        top = lam.shape[0] - 1
        out[S._idx(l, top)] = np.sum(lam * G[:top + 1], axis=1)
    t = time.perf_counter() - t0
    t_pair = t * nr / sel.size
    cores = len(os.sched_getaffinity(0))
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        used = max([d.get("num_threads", 1) for d in info] or [1])
        cores = min(cores, used) if used else cores
    except Exception:
        pass
    return {"value": 1.0 / (t_pair * max(iters, 1)), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": "numpy FP64 oracle SHT pair (Legendre + FFT synthesis and adjoint) on %d of %d rings "
                      "(%.1f s), scaled to all rings: %.1f s per SHT pair; solves/s = 1/(s per pair x %d GPU "
                      "iterations)" % (sel.size, nr, t, t_pair, iters),
            "sht_pairs_per_s": 1.0 / t_pair}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--nside", type=int, default=512)
    ap.add_argument("--lmax", type=int, default=None)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--prec", choices=["f64", "mixed"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported "
              "(independent chains would shard one per GPU with no communication)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_15511_amd import crsht
    import crinputs as ci

    nside = args.nside
    lmax = 3 * nside - 1 if args.lmax is None else args.lmax
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=10.0, cfg=2)
    wl.tol = args.tol
    R = args.nrhs
    dev = torch.device("cuda:0")
    plan = crsht.Plan(nside, lmax, nrhs_max=R)
    z, phi = plan.pixel_coords()
    ninv = torch.from_numpy(wl.ninv(z, phi)).to(dev)
    cl, bl = wl.cl(), wl.bl()
    prob = crsht.Problem(cl, bl, ninv, 2)
    # inputs: d = Y B a_true + n per column (synthesised on the GPU), w0, w1
    ls, _ = ci.alm_lm_arrays(lmax)
    A = np.stack([bl[ls] * ci.signal_alm(ci.rng_for(2, c, ci.STREAM_SIGNAL), cl, lmax) for c in range(R)])
    d = crsht.synth(plan, torch.from_numpy(A).to(dev))
    noise = np.stack([wl.sigma_map(z, phi) * ci.white_map(ci.rng_for(2, c, ci.STREAM_NOISE), wl.npix)
                      for c in range(R)])
    d += torch.from_numpy(noise).to(dev)
    w0 = torch.from_numpy(np.stack([ci.white_alm(ci.rng_for(2, c, ci.STREAM_W0), lmax) for c in range(R)])).to(dev)
    w1 = torch.from_numpy(np.stack([ci.white_map(ci.rng_for(2, c, ci.STREAM_W1), wl.npix)
                                    for c in range(R)])).to(dev)
    out = torch.empty((R, plan.nalm), dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()

    prec = crsht.CR_MIXED if args.prec == "mixed" else crsht.CR_F64

    def step():
        return crsht.solve(plan, prob, d, w0, w1, nrhs=R, tol=wl.tol, maxiter=20000, out=out, check_every=16,
                           prec=prec, inner_tol=1e-2)

    for _ in range(args.warmup):
        _, st = step()
        print("warmup: iters %s resid %s" % ([s.iters for s in st], ["%.2e" % s.rel_resid_true for s in st]),
              file=sys.stderr, flush=True)
    crsht.timing_enable(plan, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    stats = []
    for k in range(args.steps):
        _, st = step()
        iters.append(max(s.iters for s in st))
        stats.append(st)
        print("step %d: iters %s refinements %s resid %s" % (k, [s.iters for s in st], [s.refinements for s in st],
                                                             ["%.2e" % s.rel_resid_true for s in st]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_syn, n_syn = crsht.timing_read(plan, crsht.KERNEL_LEGENDRE_SYNTH)
    ms_adj, n_adj = crsht.timing_read(plan, crsht.KERNEL_LEGENDRE_ADJOINT)
    ms_ring, n_ring = crsht.timing_read(plan, crsht.KERNEL_RING)
    crsht.timing_enable(plan, False)

    solves = args.steps * R
    sps = solves / dt
    tot_iters = sum(sum(s.iters for s in st) for st in stats)
    # operator applications per solve = iterations + final true-residual check(s)
    pairs_per_s = tot_iters / dt
    T = legendre_triples(nside, lmax, lmax)
    flops_syn = (3 + 4 * R) * T        # recurrence (mul + FMA) + complex contraction per column
    avg_syn = ms_syn / max(n_syn, 1) * 1e-3
    avg_adj = ms_adj / max(n_adj, 1) * 1e-3
    achieved = flops_syn / avg_syn / 1e12 if avg_syn > 0 else 0.0
    res = {
        "metric": "constrained-realization CG solves/s at Nside=512, lmax=1535; SHT pairs/s",
        "value": sps,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "T-only CR solve, Nside %d, lmax %d, hit-pattern noise, |b|<20deg mask, "
                               "FWHM 10', tol %g, FP64 PCG" % (nside, lmax, wl.tol),
                   "nside": nside, "lmax": lmax, "nrhs": R, "tol": wl.tol, "precision": "CR_F64"},
        "sht_pairs_per_s": pairs_per_s,
        "iters_per_solve": tot_iters / solves,
        "rel_resid_true_max": max(s.rel_resid_true for st in stats for s in st),
        "kernel_ms": {"legendre_synth": avg_syn * 1e3, "legendre_adjoint": avg_adj * 1e3,
                      "ring": ms_ring / max(n_ring, 1)},
        "roofline": {"bound": "alu", "kernel": "k_legendre_synth (FP64 VALU)", "achieved": achieved,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "flops_per_launch": flops_syn, "launches": n_syn},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, int(round(tot_iters / solves)))
    print(json.dumps(res))
    plan.close()


if __name__ == "__main__":
    main()
