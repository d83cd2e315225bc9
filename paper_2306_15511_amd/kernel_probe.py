"""Short fixed workloads for hardware-counter runs (rocprofv3 --pmc).

    python -m paper_2306_15511_amd.kernel_probe operator --nside 512 --nrhs 16 --prec mixed --reps 3
    python -m paper_2306_15511_amd.kernel_probe precond --nside 512 --nrhs 16 --reps 3
    python -m paper_2306_15511_amd.kernel_probe copy --mib 1024 --reps 3

`operator` applies the constrained-realization operator (Legendre synthesis,
fused ring pass, Legendre adjoint, vector epilogue) `reps` times on the
benchmark workload, in FP64 or with the bf16x3 MFMA Legendre steps;
`precond` builds the per-m block preconditioner of that workload and applies
it `reps` times (--ncomp 3: the T+Q+U workload); `copy` copies a float64
buffer of known size so the FETCH_SIZE / WRITE_SIZE counters can be
calibrated against exact bytes.
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["operator", "precond", "copy"])
    ap.add_argument("--ncomp", type=int, choices=[1, 3], default=1)
    ap.add_argument("--nside", type=int, default=512)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--prec", choices=["f64", "mixed"], default="f64")
    a = ap.parse_args()
    dev = torch.device("cuda:0")
    if a.what == "copy":
        n = a.mib * 1024 * 1024 // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(a.reps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied %d bytes x %d" % (n * 8, a.reps))
        return
    import crinputs as ci
    from paper_2306_15511_amd import crsht
    lmax = 3 * a.nside - 1
    wl = ci.workload_masked_t(a.nside, lmax, fwhm_arcmin=10.0, cfg=2)
    plan = crsht.Plan(a.nside, lmax, nrhs_max=a.nrhs, ncomp=a.ncomp)
    z, phi = plan.pixel_coords()
    nt = wl.ninv(z, phi)
    if a.ncomp == 3:
        cl = np.ascontiguousarray(ci.cl_tqu(lmax, wl.amp, 0.3))
        prob = crsht.Problem(cl, wl.bl(), torch.from_numpy(np.stack([nt, nt / 2.0, nt / 2.0])).to(dev), 2)
    else:
        prob = crsht.Problem(wl.cl(), wl.bl(), torch.from_numpy(nt).to(dev), 2)
    rng = np.random.default_rng(0)
    x = np.stack([ci.white_alm(rng, lmax) for _ in range(a.nrhs * a.ncomp)])
    x = torch.from_numpy(x.reshape(plan.alm_shape(a.nrhs))).to(dev)
    if a.what == "precond":
        crsht.block_precond_build(plan, prob)
        for _ in range(a.reps):
            crsht.block_precond_apply(plan, x)
        torch.cuda.synchronize()
        print("applied block preconditioner x %d at nside %d, %d columns" % (a.reps, a.nside, a.nrhs))
        plan.close()
        return
    prec = crsht.CR_MIXED if a.prec == "mixed" else crsht.CR_F64
    for _ in range(a.reps):
        crsht.apply(plan, prob, x, prec=prec)
    torch.cuda.synchronize()
    print("applied operator x %d at nside %d" % (a.reps, a.nside))
    plan.close()


if __name__ == "__main__":
    main()
