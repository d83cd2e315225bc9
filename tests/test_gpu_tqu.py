"""GPU parity of T+Q+U plans (C ABI) against the oracle of oracle/cr_tqu.py and
oracle/spin2.py: spin-0 + spin-2 synthesis and its adjoint, the Jacobi
diagonal, right-hand side and operator with the 3x3 spectra blocks, PCG
solves (FP64 and mixed with FP64 residual replacement) and the chi^2 gradient.

FP64 tolerance: the spin-2 functions are formed from scalar Legendre sums with
the ring factors 1/sin^2 and cos/sin^2 applied afterwards; the polar rings
(sin^2 ~ 2 / (3 nside^2)) amplify rounding of the sums by up to that factor,
which stays far below 1e-10 at the sizes here."""
import math

import numpy as np
import pytest
import torch

import crinputs as ci
from oracle import cr, cr_tqu, healpix
from tests.gpu_helpers import rel, tc

pytestmark = pytest.mark.gpu
TOL = 1e-10
MIXED_TOL = 1e-4
# Q, U on rings with sin^2 theta < 0.01 in the mixed path: FP64 Legendre sums
# and combination, then FP32 spectra and FP32 ring FFT (a few float roundings
# of the ring's own scale)
POLAR_TOL = 1e-5


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


def _problem(nside, lmax=None, te=0.3):
    lmax = 3 * nside - 1 if lmax is None else lmax
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=60.0 * 64 / nside, cfg=2)
    z, phi = healpix.pixel_coords(nside)
    nt = wl.ninv(z, phi)
    P = cr_tqu.ProblemTQU(nside, lmax, ci.cl_tqu(lmax, wl.amp, te), wl.bl(), nt, nt / 2.0)
    return wl, P, cr_tqu.CROperatorTQU(P)


def _gpu_problem(m, P):
    ninv = np.stack([P.ninv_t, P.ninv_p, P.ninv_p])
    return m.Problem(np.ascontiguousarray(P.cl), P.bl, tc(ninv), P.lmin)


def _alm3(rng, lmax, op):
    return op.project(np.stack([ci.white_alm(rng, lmax) for _ in range(3)]))


def _data(rng, op, P):
    """d = Y B s + n for a draw s of the prior (3 maps)."""
    npix = op.sht.npix
    s = op._block(np.linalg.cholesky(_cov_blocks(P))[op.ls], _alm3(rng, P.lmax, op))
    noise = rng.standard_normal((3, npix)) / np.sqrt(np.maximum(op._ninv(), 1e-30)) * (op._ninv() > 0)
    return op.synth(op.b * op.project(s)) + noise


def _cov_blocks(P):
    C = np.zeros((P.lmax + 1, 3, 3))
    C[:, 0, 0], C[:, 1, 1], C[:, 2, 2] = P.cl[0], P.cl[1], P.cl[2]
    C[:, 0, 1] = C[:, 1, 0] = P.cl[3]
    C[:2] = np.eye(3)   # unused modes (projected out)
    return C


def real_rel3(op, a, b):
    d = a - b
    return math.sqrt(max(op.dot(d, d), 0.0)) / math.sqrt(max(op.dot(b, b), 1e-300))


@pytest.mark.parametrize("nside", [4, 8, 32])
def test_tqu_synth_adjoint(nside):
    m = _m()
    print("case tqu transforms nside", nside, flush=True)
    wl, P, op = _problem(nside)
    plan = m.Plan(nside, P.lmax, nrhs_max=2, ncomp=3)
    rng = np.random.default_rng(nside)
    A = np.stack([_alm3(rng, P.lmax, op) for _ in range(2)])
    maps = m.synth(plan, tc(A)).cpu().numpy()
    assert maps.shape == (2, 3, op.sht.npix)
    for c in range(2):
        ref = op.synth(A[c])
        for k in range(3):
            assert rel(maps[c, k], ref[k]) < TOL, (c, k, rel(maps[c, k], ref[k]))
    M = rng.standard_normal((2, 3, op.sht.npix))
    got = m.adjoint(plan, tc(M)).cpu().numpy()
    for c in range(2):
        ref = op.adjoint(M[c])
        for k in range(3):
            assert rel(got[c, k], ref[k]) < TOL, (c, k, rel(got[c, k], ref[k]))


@pytest.mark.parametrize("nside", [4, 8, 16])
def test_tqu_precond_rhs_apply(nside):
    m = _m()
    print("case tqu operator nside", nside, flush=True)
    wl, P, op = _problem(nside)
    plan = m.Plan(nside, P.lmax, nrhs_max=2, ncomp=3)
    gp = _gpu_problem(m, P)
    assert rel(m.precond(plan, gp).cpu().numpy(), op.diag()) < TOL
    rng = np.random.default_rng(7)
    d = _data(rng, op, P)
    w0 = np.stack([ci.white_alm(rng, P.lmax) for _ in range(3)])
    w1 = rng.standard_normal((3, op.sht.npix))
    for args in ((d, w0, w1), (d, None, None), (None, w0, None), (None, None, w1)):
        ref = op.rhs(*args)
        got = m.rhs(plan, gp, *[None if v is None else tc(v) for v in args]).cpu().numpy()[0]
        assert real_rel3(op, got, ref) < TOL
    X = np.stack([_alm3(rng, P.lmax, op) for _ in range(2)])
    got = m.apply(plan, gp, tc(X)).cpu().numpy()
    for c in range(2):
        assert real_rel3(op, got[c], op.apply(X[c])) < TOL


def test_tqu_solve_matches_oracle_pcg():
    m = _m()
    nside = 4
    wl, P, op = _problem(nside, 11)
    plan = m.Plan(nside, P.lmax, ncomp=3)
    gp = _gpu_problem(m, P)
    rng = np.random.default_rng(11)
    d = _data(rng, op, P)
    w0 = np.stack([ci.white_alm(rng, P.lmax) for _ in range(3)])
    w1 = rng.standard_normal((3, op.sht.npix))
    s, st = m.solve(plan, gp, tc(d), tc(w0), tc(w1), tol=1e-13, maxiter=5000)
    assert st[0].status == 0 and st[0].rel_resid_true <= 1e-13
    xo, info = cr.pcg(op, op.rhs(d, w0, w1), 1e-13, 5000)
    assert info.converged
    assert real_rel3(op, s.cpu().numpy()[0], xo) < TOL


@pytest.mark.parametrize("nside", [16, 32])
def test_tqu_solve_oracle_residual(nside):
    m = _m()
    print("case tqu solve nside", nside, flush=True)
    wl, P, op = _problem(nside)
    plan = m.Plan(nside, P.lmax, nrhs_max=2, ncomp=3)
    gp = _gpu_problem(m, P)
    rng = np.random.default_rng(nside + 1)
    d = np.stack([_data(rng, op, P) for _ in range(2)])
    w0 = np.stack([np.stack([ci.white_alm(rng, P.lmax) for _ in range(3)]) for _ in range(2)])
    w1 = rng.standard_normal((2, 3, op.sht.npix))
    s, st = m.solve(plan, gp, tc(d), tc(w0), tc(w1), nrhs=2, tol=1e-8, maxiter=20000)
    for c in range(2):
        b = op.rhs(d[c], w0[c], w1[c])
        res = real_rel3(op, op.apply(s.cpu().numpy()[c]), b)
        print("col", c, "iters", st[c].iters, "res", res, flush=True)
        assert st[c].status == 0
        assert res <= 1.5e-8
        assert abs(res - st[c].rel_resid_true) < 1e-10


@pytest.mark.parametrize("nside", [8, 16, 32, 64])
def test_tqu_mixed_transforms(nside):
    # Nside 8: no ring pair with sin^2 theta < 0.01; 16, 32, 64: 1, 3, 7
    # polar pairs take FP64 Legendre sums inside the mixed transforms
    m = _m()
    print("case tqu mixed transforms nside", nside, flush=True)
    wl, P, op = _problem(nside)
    plan = m.Plan(nside, P.lmax, ncomp=3)
    rng = np.random.default_rng(3)
    a = _alm3(rng, P.lmax, op)
    got = m.synth(plan, tc(a), prec=m.CR_MIXED).cpu().numpy()
    ref = op.synth(a)
    errs = [rel(got[k], ref[k]) for k in range(3)]
    M = rng.standard_normal((3, op.sht.npix))
    ga = m.adjoint(plan, tc(M), prec=m.CR_MIXED).cpu().numpy()
    ra = op.adjoint(M)
    errs += [rel(ga[k], ra[k]) for k in range(3)]
    print("mixed rel errors (T, Q, U maps; T, E, B alm)", errs, flush=True)
    assert max(errs) < MIXED_TOL
    # the polar rings (FP64 sums, FP32 ring FFT) on their own
    R = op.sht.rings
    for k in range(R.z.size):
        if R.sin_theta[k] ** 2 >= 0.01:
            continue
        f, n = int(R.first[k]), int(R.nphi[k])
        for c in (1, 2):
            e = rel(got[c, f:f + n], ref[c, f:f + n])
            assert e < POLAR_TOL, (k, c, e)


def test_tqu_mixed_solve_oracle_residual():
    m = _m()
    nside = 32
    wl, P, op = _problem(nside)
    plan = m.Plan(nside, P.lmax, ncomp=3)
    gp = _gpu_problem(m, P)
    rng = np.random.default_rng(5)
    d = _data(rng, op, P)
    w0 = np.stack([ci.white_alm(rng, P.lmax) for _ in range(3)])
    w1 = rng.standard_normal((3, op.sht.npix))
    s, st = m.solve(plan, gp, tc(d), tc(w0), tc(w1), tol=1e-6, maxiter=20000, prec=m.CR_MIXED)
    b = op.rhs(d, w0, w1)
    res = real_rel3(op, op.apply(s.cpu().numpy()[0]), b)
    print("mixed tqu iters", st[0].iters, "refinements", st[0].refinements, "res", res, flush=True)
    assert st[0].status == 0
    assert res <= 1.05e-6
    assert abs(res - st[0].rel_resid_true) <= 1e-9


@pytest.mark.parametrize("nside", [8, 16])
def test_tqu_grad_chi2(nside):
    m = _m()
    wl, P, op = _problem(nside)
    plan = m.Plan(nside, P.lmax, nrhs_max=2, ncomp=3)
    gp = _gpu_problem(m, P)
    rng = np.random.default_rng(9)
    d = np.stack([_data(rng, op, P) for _ in range(2)])
    a = np.stack([_alm3(rng, P.lmax, op) for _ in range(2)])
    g, chi2 = m.grad_chi2(plan, gp, tc(d), tc(a))
    g = g.cpu().numpy()
    n = op._ninv()
    for c in range(2):
        r = d[c] - op.synth(op.b * a[c])
        ref_chi2 = float(np.sum(n * r * r))
        ref_g = op.project(-2.0 * op.b * op.adjoint(n * r))
        assert abs(chi2[c] - ref_chi2) <= 1e-10 * ref_chi2
        assert real_rel3(op, g[c], ref_g) < TOL


def test_tqu_rejects_unsupported():
    m = _m()
    wl, P, op = _problem(4, 11)
    plan = m.Plan(4, 11, ncomp=3)
    bad = m.Problem(np.ascontiguousarray(P.cl), P.bl, tc(np.stack([P.ninv_t] * 3)), 1)
    with pytest.raises(m.CrshtError):
        m.precond(plan, bad)
    cl = np.array(P.cl)
    cl[3, 5] = 2.0 * math.sqrt(cl[0, 5] * cl[1, 5])    # |TE| > sqrt(TT EE): not positive definite
    with pytest.raises(m.CrshtError):
        m.precond(plan, m.Problem(cl, P.bl, tc(np.stack([P.ninv_t] * 3)), 2))


def test_tqu_nside128_full_maps():
    m = _m()
    nside = 128
    print("case tqu nside128", flush=True)
    wl, P, op = _problem(nside)
    plan = m.Plan(nside, P.lmax, ncomp=3)
    rng = np.random.default_rng(128)
    a = _alm3(rng, P.lmax, op)
    got = m.synth(plan, tc(a)).cpu().numpy()
    ref = op.synth(a)
    errs = [rel(got[k], ref[k]) for k in range(3)]
    gm = m.synth(plan, tc(a), prec=m.CR_MIXED).cpu().numpy()
    errs_m = [rel(gm[k], ref[k]) for k in range(3)]
    M = rng.standard_normal((3, op.sht.npix))
    ga = m.adjoint(plan, tc(M)).cpu().numpy()
    ra = op.adjoint(M)
    errs += [rel(ga[k], ra[k]) for k in range(3)]
    gam = m.adjoint(plan, tc(M), prec=m.CR_MIXED).cpu().numpy()
    errs_m += [rel(gam[k], ra[k]) for k in range(3)]
    print("fp64", errs, "mixed", errs_m, flush=True)
    assert max(errs) < TOL
    assert max(errs_m) < MIXED_TOL


def test_tqu_nside512_sampled_rings_and_adjointness():
    # the T+Q+U benchmark size: sampled rings of Q and U against the oracle,
    # adjointness of the three-component transform pair
    m = _m()
    from oracle import spin2
    nside, lmax = 512, 1535
    print("case tqu nside512", flush=True)
    plan = m.Plan(nside, lmax, ncomp=3)
    pol = spin2.PolSHT(nside, lmax)
    rng = np.random.default_rng(512)
    ls, ms = ci.alm_lm_arrays(lmax)
    a = np.stack([ci.white_alm(rng, lmax) for _ in range(3)])
    a[:, ls < 2] = 0.0
    a[:, ms == 0] = a[:, ms == 0].real
    got = m.synth(plan, tc(a)).cpu().numpy()
    gm = m.synth(plan, tc(a), prec=m.CR_MIXED).cpu().numpy()
    rings = [0, 1, 2, 37, 300, 511, 512, 900, 1023, 1500, 2045, 2046]
    ref = pol.synth_rings(a[1], a[2], rings)
    R = pol.s.rings
    for k in rings:
        f, n = int(R.first[k]), int(R.nphi[k])
        # Q and U divide Legendre sums that cancel near the poles by
        # sin^2 theta, which amplifies split-bf16 rounding there (measured
        # 1.7e-5 / sin theta on ring 0 and 9e-6 / sin theta on ring 37 with
        # bf16x3 sums on every ring): rings with sin^2 < 0.01 take FP64 sums
        # (POLAR_TOL), the others keep the 1e-4 bound
        s2 = 1.0 - R.z[k] ** 2
        bound_m = POLAR_TOL if s2 < 0.01 else MIXED_TOL
        for q in range(2):
            e = rel(got[1 + q, f:f + n], ref[k][q])
            assert e < TOL, (k, q, e)
            em = rel(gm[1 + q, f:f + n], ref[k][q])
            print("ring %d sin^2 %.2e: mixed rel error %.2e (bound %.2e)" % (k, s2, em, bound_m), flush=True)
            assert em < bound_m, (k, q, em)
    y = rng.standard_normal((3, pol.npix))
    ya = m.adjoint(plan, tc(y)).cpu().numpy()
    lhs = float(np.sum(got * y))
    from oracle.sht import dot
    rhs = sum(dot(a[k], ya[k], lmax, lmax) for k in range(3))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(got) * np.linalg.norm(y)


def test_tqu_nside1024_16_columns_sampled():
    # the largest T+Q+U workload (Nside 1024, lmax 2047, 16 columns: 8 chains
    # x mean and fluctuation): sampled rings of T, Q, U of the first and last
    # column against the oracle (FP64 and mixed), adjointness of the transform
    # pair and symmetry of the FP64 operator on two columns, and the block
    # preconditioner (built at this size) symmetric and positive
    m = _m()
    from oracle import sht as osht, spin2
    nside, lmax, ncol = 1024, 2047, 16
    print("case tqu nside1024 x16", flush=True)
    plan = m.Plan(nside, lmax, nrhs_max=ncol, ncomp=3)
    rng = np.random.default_rng(1024)
    ls, ms = ci.alm_lm_arrays(lmax)
    a = (rng.standard_normal((ncol, 3, ls.size)) + 1j * rng.standard_normal((ncol, 3, ls.size))) / math.sqrt(2.0)
    a[:, :, ls < 2] = 0.0
    a[:, :, ms == 0] = a[:, :, ms == 0].real
    da = tc(a)
    del a
    npix = 12 * nside * nside
    rings = [0, 1, 700, 2047, 3000, 4094]
    pol = spin2.PolSHT(nside, lmax)
    R = pol.s.rings
    cols = [0, ncol - 1]
    # Q and U carry the 1/sin^2 cancellation of the spin-2 sums (module
    # docstring): FP64 rounding u of the Legendre sums reaches Q, U amplified
    # by up to 1/sin^2 (1.6e6 on the first ring here), so their bound on a
    # ring is max(TOL, 8 u / sin^2); the mixed path is held to MIXED_TOL on
    # rings with sin^2 > 0.01 and to POLAR_TOL on the others (FP64 sums)
    u = np.finfo(np.float64).eps / 2
    for prec in (m.CR_F64, m.CR_MIXED):
        got = m.synth(plan, da, prec=prec)
        sel = {k: got[cols, :, int(R.first[k]):int(R.first[k]) + int(R.nphi[k])].cpu().numpy() for k in rings}
        del got
        worst = {}
        for ci_, c in enumerate(cols):
            ac = da[c].cpu().numpy()
            rt = osht.synth_rings(pol.s, ac[0], rings)
            rp = pol.synth_rings(ac[1], ac[2], rings)
            for k in rings:
                s2 = float(R.sin_theta[k]) ** 2
                for comp, ref in ((0, rt[k]), (1, rp[k][0]), (2, rp[k][1])):
                    e = rel(sel[k][ci_, comp], ref)
                    worst[k] = max(worst.get(k, 0.0), e)
                    if prec == m.CR_F64:
                        tol = TOL if comp == 0 else max(TOL, 8 * u / s2)
                        assert e < tol, (prec, c, k, comp, e, tol)
                    elif s2 > 1e-2:
                        assert e < MIXED_TOL, (prec, c, k, comp, e)
                    else:
                        assert e < POLAR_TOL, (prec, c, k, comp, e)
        print("prec", prec, "worst rel error per sampled ring", {k: "%.1e" % v for k, v in worst.items()}, flush=True)
    # adjointness and operator symmetry on two columns (FP64)
    x = da[:2].contiguous()
    y = torch.from_numpy(rng.standard_normal((2, 3, npix))).to(x.device)
    ya = m.adjoint(plan, y)
    sx = m.synth(plan, x)
    lhs = float(torch.sum(sx * y))
    mw = torch.from_numpy(np.where(ms == 0, 1.0, 2.0)).to(x.device)
    rhs = float(torch.sum(mw * (x.real * ya.real + x.imag * ya.imag)))
    assert abs(lhs - rhs) <= 1e-11 * float(torch.linalg.vector_norm(sx)) * float(torch.linalg.vector_norm(y))
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=10.0, cfg=2)
    z, phi = plan.pixel_coords()
    nt = wl.ninv(z, phi)
    gp = m.Problem(np.ascontiguousarray(ci.cl_tqu(lmax, wl.amp, 0.3)), wl.bl(),
                   tc(np.stack([nt, nt / 2.0, nt / 2.0])), 2)
    u = da[2:4].contiguous()
    ax, au = m.apply(plan, gp, x), m.apply(plan, gp, u)
    d1 = float(torch.sum(mw * (u.real * ax.real + u.imag * ax.imag)))
    d2 = float(torch.sum(mw * (x.real * au.real + x.imag * au.imag)))
    print("operator symmetry", d1, d2, flush=True)
    assert abs(d1 - d2) <= 1e-10 * abs(d1)
    m.block_precond_build(plan, gp)
    px, pu = m.block_precond_apply(plan, x), m.block_precond_apply(plan, u)
    e1 = float(torch.sum(mw * (u.real * px.real + u.imag * px.imag)))
    e2 = float(torch.sum(mw * (x.real * pu.real + x.imag * pu.imag)))
    ex = float(torch.sum(mw * (x.real * px.real + x.imag * px.imag)))
    print("block preconditioner symmetry", e1, e2, "positivity", ex, flush=True)
    assert abs(e1 - e2) <= 1e-5 * math.sqrt(abs(ex) * abs(float(torch.sum(mw * (u.real * pu.real + u.imag * pu.imag)))))
    assert ex > 0


def test_tqu_nside1024_16_columns_mixed_solve():
    # the largest T+Q+U workload end to end: Nside 1024, lmax 2047, 16 columns
    # (8 chains x mean field and fluctuation), split-bf16 Legendre sums with
    # FP64 polar rings inside FP64 residual replacement, block preconditioner,
    # relative residual 1e-6. The residual of the returned solution is taken
    # again with the FP64 operator and right-hand side entry points.
    m = _m()
    nside, lmax, R = 1024, 2047, 16
    print("case tqu nside1024 x16 mixed solve", flush=True)
    plan = m.Plan(nside, lmax, nrhs_max=R, ncomp=3)
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=10.0, cfg=2)
    z, phi = plan.pixel_coords()
    nt = wl.ninv(z, phi)
    sig = torch.from_numpy(wl.sigma_map(z, phi)).cuda()
    cl = np.ascontiguousarray(ci.cl_tqu(lmax, wl.amp, 0.3))
    bl = wl.bl()
    gp = m.Problem(cl, bl, tc(np.stack([nt, nt / 2.0, nt / 2.0])), 2)
    ls, _ = ci.alm_lm_arrays(lmax)
    # columns 2k (mean field: data, no white terms) and 2k+1 (fluctuation:
    # white terms only), 8 sky draws
    A = np.zeros((R, 3, ls.size), dtype=np.complex128)
    for c in range(0, R, 2):
        A[c] = bl[ls] * ci.signal_alm_tqu(ci.rng_for(4, c, ci.STREAM_SIGNAL), cl, lmax)
    d = m.synth(plan, tc(A))
    del A
    g = torch.Generator(device="cuda")
    g.manual_seed(1024)
    qu = torch.tensor([1.0, 2 ** 0.5, 2 ** 0.5], dtype=torch.float64, device="cuda").view(3, 1)
    for c in range(0, R, 2):
        d[c] += qu * sig * torch.randn((3, sig.numel()), generator=g, dtype=torch.float64, device="cuda")
    d[1::2] = 0.0
    w0 = torch.zeros(plan.alm_shape(R), dtype=torch.complex128, device="cuda")
    w1 = torch.zeros((R, 3, sig.numel()), dtype=torch.float64, device="cuda")
    for c in range(1, R, 2):
        for k in range(3):
            w0[c, k] = tc(ci.white_alm(ci.rng_for(4, c, ci.STREAM_W0 + 10 * k), lmax))
        w1[c] = torch.randn((3, sig.numel()), generator=g, dtype=torch.float64, device="cuda")
    m.block_precond_build(plan, gp)
    import time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = m.solve(plan, gp, d, w0, w1, nrhs=R, tol=1e-6, maxiter=3000, prec=m.CR_MIXED, inner_tol=1e-2,
                    precond=m.CR_PC_BLOCK, check_every=6)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("mixed solve %.2f s, iters %s, refinements %s, rel true residual max %.2e"
          % (dt, [s.iters for s in st], [s.refinements for s in st], max(s.rel_resid_true for s in st)), flush=True)
    assert all(s.status == 0 for s in st)
    b = m.rhs(plan, gp, d, w0, w1, nrhs=R)
    del d, w0, w1
    r = b - m.apply(plan, gp, x)
    _, ms = ci.alm_lm_arrays(lmax)
    mw = torch.from_numpy(np.where(ms == 0, 1.0, 2.0)).cuda()
    for c in range(R):
        nr = float(torch.sum(mw * (r[c].real ** 2 + r[c].imag ** 2)).sqrt())
        nb = float(torch.sum(mw * (b[c].real ** 2 + b[c].imag ** 2)).sqrt())
        assert nr <= 1.05e-6 * nb, (c, nr / nb)
        assert abs(nr / nb - st[c].rel_resid_true) <= 1e-8, (c, nr / nb, st[c].rel_resid_true)


def test_tqu_column_amplitudes():
    # T+Q+U columns at amp[c] times all four spectra: solve against the
    # oracle's PCG on the scaled problem
    m = _m()
    nside = 4
    print("case tqu column amplitudes", flush=True)
    wl, P, op = _problem(nside, 11)
    amp = np.array([0.7, 1.4])
    plan = m.Plan(nside, P.lmax, nrhs_max=2, ncomp=3)
    gp = m.Problem(np.ascontiguousarray(P.cl), P.bl, tc(np.stack([P.ninv_t, P.ninv_p, P.ninv_p])), P.lmin, amp)
    rng = np.random.default_rng(12)
    d = np.stack([_data(rng, op, P) for _ in range(2)])
    w0 = np.stack([np.stack([ci.white_alm(rng, P.lmax) for _ in range(3)]) for _ in range(2)])
    w1 = rng.standard_normal((2, 3, op.sht.npix))
    s, st = m.solve(plan, gp, tc(d), tc(w0), tc(w1), nrhs=2, tol=1e-13, maxiter=5000)
    for c in range(2):
        Pc = cr_tqu.ProblemTQU(nside, P.lmax, P.cl * amp[c], P.bl, P.ninv_t, P.ninv_p, P.lmin)
        oc = cr_tqu.CROperatorTQU(Pc)
        xo, info = cr.pcg(oc, oc.rhs(d[c], w0[c], w1[c]), 1e-13, 5000)
        assert info.converged and st[c].status == 0
        assert real_rel3(oc, s.cpu().numpy()[c], xo) < TOL


def test_tqu_lnpi_and_joint_step():
    # ln pi of a T+Q+U state (at q = 1 and rescaled) and the joint move
    # (accepted, then rejected) against the oracle with the same numbers
    from oracle import joint
    m = _m()
    nside = 4
    print("case tqu joint step", flush=True)
    wl, P, op = _problem(nside, 11)
    plan = m.Plan(nside, P.lmax, ncomp=3)
    gp = _gpu_problem(m, P)
    rng = np.random.default_rng(19)
    d = _data(rng, op, P)
    npix = op.sht.npix
    w0 = np.stack([ci.white_alm(rng, P.lmax) for _ in range(3)])
    w1 = rng.standard_normal((3, npix))
    tol = 1e-12
    a, _ = cr.pcg(op, op.rhs(d=d), 1e-13)
    f, _ = cr.pcg(op, op.rhs(w0=w0, w1=w1), 1e-13)
    lp = joint.lnpi_tqu(op, d, a, f)
    assert abs(m.lnpi(plan, gp, 1.0, tc(d), tc(a), tc(f)) - lp) <= 1e-10 * abs(lp)
    op13 = cr_tqu.CROperatorTQU(cr_tqu.ProblemTQU(nside, P.lmax, P.cl * 1.3, P.bl, P.ninv_t, P.ninv_p, P.lmin))
    lp13 = joint.lnpi_tqu(op13, d, a, f)
    assert abs(m.lnpi(plan, gp, 1.3, tc(d), tc(a), tc(f)) - lp13) <= 1e-10 * abs(lp13)
    st = joint.ChainState(1.0, a, f, lp)
    ch = m.Chain(1.0, lp, tc(a), tc(f))
    for xi, u in ((0.4, 1e-300), (60.0, 1.0 - 1e-12)):
        w0n = np.stack([ci.white_alm(rng, P.lmax) for _ in range(3)])
        w1n = rng.standard_normal((3, npix))
        res = m.joint_step(plan, gp, tc(d), ch, xi, u, tc(w0n), tc(w1n), sigma_lnq=0.05, tol=tol)
        new, r = joint.joint_step_tqu(P, d, st, xi, u, w0n, w1n, 0.05, tol)
        print("lnA gpu %.12e oracle %.12e accepted %s/%s" % (res.lnA, r.lnA, res.accepted, r.accepted), flush=True)
        assert res.accepted == r.accepted
        assert res.q_new == r.q_new
        assert abs(res.lnA - r.lnA) <= 1e-8 + 1e-13 * abs(r.lnpi_new)   # absolute: ln A decides the move
        assert abs(ch.q - new.q) <= 1e-15 * new.q and abs(ch.lnpi - new.lnpi) <= 1e-9 * abs(new.lnpi)
        opn = cr_tqu.CROperatorTQU(cr_tqu.ProblemTQU(nside, P.lmax, P.cl * new.q, P.bl, P.ninv_t, P.ninv_p, P.lmin))
        assert real_rel3(opn, ch.ahat.cpu().numpy(), new.ahat) < 1e-8
        assert real_rel3(opn, ch.fhat.cpu().numpy(), new.fhat) < 1e-8
        st = new
    assert ch.q == st.q
