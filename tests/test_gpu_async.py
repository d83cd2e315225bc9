"""GPU checks of the stream-ordered solve cr_solve_async (through the C ABI):
the mixed-precision solve equals cr_solve's (the refinement decisions that
cr_solve takes on the host from scalars read back are taken on the device);
two solves enqueued on one stream without any synchronisation in between,
their statistics read from device memory after one synchronisation, the
solutions checked by the oracle's residual; the call returns before the
solve has run; FP64 and T+Q+U forms; a maxiter too small reports CR_NOCONV."""
import time

import numpy as np
import pytest
import torch

import crinputs as ci
from oracle import cr, cr_tqu, healpix
from oracle import sht as osht
from tests.gpu_helpers import masked_problem, real_rel, tc

pytestmark = pytest.mark.gpu


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


def _oracle_resid(op, x, b):
    return op.norm(b - op.apply(x)) / op.norm(b)


@pytest.mark.parametrize("precond", ["jacobi", "block"])
def test_async_mixed_equals_sync(precond):
    m = _m()
    print("case async mixed vs cr_solve", precond, flush=True)
    nside, R = 32, 3
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax, nrhs_max=R)
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), 2)
    pc = m.CR_PC_BLOCK if precond == "block" else m.CR_PC_JACOBI
    if precond == "block":
        m.block_precond_build(plan, gp)
    rng = np.random.default_rng(7)
    D = tc(np.stack([d * (1.0 + 0.1 * c) for c in range(R)]))
    W0 = tc(np.stack([ci.white_alm(rng, wl.lmax) for _ in range(R)]))
    W1 = tc(rng.standard_normal((R, P.ninv.size)))
    kw = dict(nrhs=R, tol=1e-6, prec=m.CR_MIXED, inner_tol=1e-2, max_refine=50, check_every=6, precond=pc)
    s1, st1 = m.solve(plan, gp, D, W0, W1, maxiter=2000, **kw)
    s2, sd = m.solve_async(plan, gp, D, W0, W1, maxiter=2000, **kw)
    torch.cuda.synchronize()
    st2 = m.decode_stats(sd, R)
    for c in range(R):
        e = real_rel(op, s2[c].cpu().numpy(), s1[c].cpu().numpy())
        print("column %d: iters %d / %d, replacements %d / %d, residual %.3e / %.3e, rel diff %.2e" % (
            c, st1[c].iters, st2[c].iters, st1[c].refinements, st2[c].refinements, st1[c].rel_resid_true,
            st2[c].rel_resid_true, e), flush=True)
        assert st2[c].status == 0
        assert st2[c].iters == st1[c].iters and st2[c].refinements == st1[c].refinements
        assert e <= 1e-12
        assert abs(st2[c].rel_resid_true - st1[c].rel_resid_true) <= 1e-12


def test_two_async_solves_one_stream_one_sync():
    m = _m()
    print("case two async solves, one sync (nside 256)", flush=True)
    nside = 256
    wl = ci.workload_masked_t(nside)
    z, phi = healpix.pixel_coords(nside)
    S = osht.SHT(nside, wl.lmax, fast=True)
    P = cr.Problem(nside, wl.lmax, wl.cl(), wl.bl(), wl.ninv(z, phi))
    op = cr.CROperator(P, S)
    d = S.synth(op.b * wl.signal()) + wl.noise(z, phi)
    rng = np.random.default_rng(256)
    w0 = np.stack([ci.white_alm(rng, wl.lmax) for _ in range(2)])
    w1 = rng.standard_normal((2, P.ninv.size))
    plan = m.Plan(nside, wl.lmax, nrhs_max=2)
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), 2)
    m.block_precond_build(plan, gp)
    dd, W0, W1 = tc(d), tc(w0), tc(w1)
    kw = dict(tol=1e-6, maxiter=60, prec=m.CR_MIXED, inner_tol=1e-3, check_every=6, precond=m.CR_PC_BLOCK)
    # warm-up: captures the graphs of this configuration
    m.solve_async(plan, gp, dd, W0[:1], W1[:1], **kw)
    torch.cuda.synchronize()
    out_a = torch.empty((1, plan.nalm), dtype=torch.complex128, device="cuda:0")
    out_b = torch.empty((1, plan.nalm), dtype=torch.complex128, device="cuda:0")
    st_a = torch.full((24,), 255, dtype=torch.uint8, device="cuda:0")
    st_b = torch.full((24,), 255, dtype=torch.uint8, device="cuda:0")
    t0 = time.perf_counter()
    m.solve_async(plan, gp, dd, W0[:1], W1[:1], out=out_a, stats=st_a, **kw)
    m.solve_async(plan, gp, None, W0[1:], W1[1:], out=out_b, stats=st_b, **kw)
    t_enqueue = time.perf_counter() - t0
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    sa, sb = m.decode_stats(st_a, 1)[0], m.decode_stats(st_b, 1)[0]
    print("enqueue %.1f ms, enqueue + run %.1f ms; iters %d / %d, replacements %d / %d" % (
        1e3 * t_enqueue, 1e3 * t_total, sa.iters, sb.iters, sa.refinements, sb.refinements), flush=True)
    assert t_enqueue < 0.5 * t_total          # the calls returned before the solves had run
    assert sa.status == 0 and sb.status == 0
    ra = _oracle_resid(op, out_a[0].cpu().numpy(), op.rhs(d, w0[0], w1[0]))
    rb = _oracle_resid(op, out_b[0].cpu().numpy(), op.rhs(None, w0[1], w1[1]))
    print("oracle residuals %.3e %.3e (library %.3e %.3e)" % (ra, rb, sa.rel_resid_true, sb.rel_resid_true),
          flush=True)
    assert ra <= 1e-6 and rb <= 1e-6
    assert abs(ra - sa.rel_resid_true) <= 1e-9 and abs(rb - sb.rel_resid_true) <= 1e-9


def test_async_fp64_jacobi_and_noconv():
    m = _m()
    print("case async fp64", flush=True)
    nside = 16
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), 2)
    w0, w1 = wl.w0(), wl.w1()
    s, sd = m.solve_async(plan, gp, tc(d), tc(w0), tc(w1), tol=1e-10, maxiter=2000, check_every=8)
    torch.cuda.synchronize()
    st = m.decode_stats(sd, 1)[0]
    res = _oracle_resid(op, s[0].cpu().numpy(), op.rhs(d, w0, w1))
    print("fp64: iters %d, oracle residual %.2e, library %.2e" % (st.iters, res, st.rel_resid_true), flush=True)
    assert st.status == 0 and res <= 1.5e-10 and st.refinements == 0
    s, sd = m.solve_async(plan, gp, tc(d), tc(w0), tc(w1), tol=1e-10, maxiter=8, check_every=8)
    torch.cuda.synchronize()
    st = m.decode_stats(sd, 1)[0]
    print("maxiter 8: status %d, iters %d, residual %.2e" % (st.status, st.iters, st.rel_resid_true), flush=True)
    assert st.status == m.CR_NOCONV and st.iters == 8
    res = _oracle_resid(op, s[0].cpu().numpy(), op.rhs(d, w0, w1))
    assert abs(res - st.rel_resid_true) <= 1e-12 + 1e-9 * res


def test_async_tqu_mixed():
    m = _m()
    print("case async tqu mixed", flush=True)
    nside = 8
    wl = ci.workload_masked_t(nside)
    z, phi = healpix.pixel_coords(nside)
    nt = wl.ninv(z, phi)
    cl = np.ascontiguousarray(ci.cl_tqu(wl.lmax, wl.amp, 0.3))
    P = cr_tqu.ProblemTQU(nside, wl.lmax, cl, wl.bl(), nt, nt / 2.0, 2)
    op = cr_tqu.CROperatorTQU(P)
    rng = np.random.default_rng(88)
    npix = 12 * nside * nside
    d = rng.standard_normal((3, npix)) * 50.0
    w0 = np.stack([ci.white_alm(rng, wl.lmax) for _ in range(3)])
    w1 = rng.standard_normal((3, npix))
    plan = m.Plan(nside, wl.lmax, ncomp=3)
    gp = m.Problem(cl, wl.bl(), tc(np.stack([nt, nt / 2.0, nt / 2.0])), 2)
    s, sd = m.solve_async(plan, gp, tc(d), tc(w0), tc(w1), tol=1e-6, maxiter=3000, prec=m.CR_MIXED,
                          check_every=8)
    torch.cuda.synchronize()
    st = m.decode_stats(sd, 1)[0]
    x = s.cpu().numpy()[0]
    b = op.rhs(d, w0, w1)
    res = op.norm(b - op.apply(x)) / op.norm(b)
    print("tqu mixed: iters %d, replacements %d, oracle residual %.2e" % (st.iters, st.refinements, res),
          flush=True)
    assert st.status == 0 and res <= 1.5e-6
