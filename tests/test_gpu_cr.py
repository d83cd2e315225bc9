"""GPU parity of the constrained-realization pieces (C ABI) against the oracle:
Jacobi diagonal, right-hand side, operator, PCG solves (dense Cholesky at small
Nside, oracle residual at larger), batched columns, special cases, status."""
import math

import numpy as np
import pytest
import torch

import crinputs as ci
from oracle import cr, dense, healpix
from tests.gpu_helpers import masked_problem, real_rel, rel, tc

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


def _gpu_problem(m, P):
    return m.Problem(P.cl, P.bl, tc(P.ninv), P.lmin)


@pytest.mark.parametrize("nside", [4, 8, 32])
def test_precond_rhs_apply(nside):
    m = _m()
    print("case", nside, flush=True)
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax, nrhs_max=2)
    gp = _gpu_problem(m, P)
    assert rel(m.precond(plan, gp).cpu().numpy(), op.diag()) < TOL
    w0, w1 = wl.w0(), wl.w1()
    for args in ((d, w0, w1), (d, None, None), (None, w0, None), (None, None, w1)):
        ref = op.rhs(*args)
        got = m.rhs(plan, gp, *[None if v is None else tc(v) for v in args]).cpu().numpy()[0]
        assert rel(got, ref) < TOL
    rng = np.random.default_rng(5)
    X = np.stack([ci.white_alm(rng, wl.lmax) for _ in range(2)])
    got = m.apply(plan, gp, tc(X)).cpu().numpy()
    for c in range(2):
        assert rel(got[c], op.apply(X[c])) < TOL


@pytest.mark.parametrize("nside", [4, 8])
def test_solve_matches_dense_cholesky(nside):
    m = _m()
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    gp = _gpu_problem(m, P)
    w0, w1 = wl.w0(), wl.w1()
    s, st = m.solve(plan, gp, tc(d), tc(w0), tc(w1), tol=1e-13, maxiter=5000)
    assert st[0].status == 0 and st[0].rel_resid_true <= 1e-13
    D = dense.DenseY(nside, wl.lmax, lmin=2)
    ref = D.cr_solve(P.cl, P.bl, P.ninv, op.rhs(d, w0, w1))
    assert real_rel(op, s.cpu().numpy()[0], ref) < TOL


def test_solve_nside32_oracle_residual_and_iterations():
    m = _m()
    nside = 32
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    gp = _gpu_problem(m, P)
    w0, w1 = wl.w0(), wl.w1()
    s, st = m.solve(plan, gp, tc(d), tc(w0), tc(w1), tol=1e-8, maxiter=20000)
    x = s.cpu().numpy()[0]
    b = op.rhs(d, w0, w1)
    res = real_rel(op, op.apply(x), b)       # oracle-evaluated residual of the GPU solution
    assert res <= 1.5e-8
    assert abs(res - st[0].rel_resid_true) < 1e-10
    xo, info = cr.pcg(op, b, 1e-8, 20000)
    assert abs(info.iters - st[0].iters) <= max(2, info.iters // 50)
    print("iters gpu", st[0].iters, "oracle", info.iters, "diff", real_rel(op, x, xo), flush=True)
    assert real_rel(op, x, xo) < 1e-5


def test_batched_columns_independent():
    m = _m()
    nside = 8
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax, nrhs_max=3)
    gp = _gpu_problem(m, P)
    rng = np.random.default_rng(9)
    W0 = np.stack([ci.white_alm(rng, wl.lmax) for _ in range(3)])
    W1 = np.stack([rng.standard_normal(P.ninv.size) for _ in range(3)])
    D3 = np.stack([d, 2 * d, -d])
    s, st = m.solve(plan, gp, tc(D3), tc(W0), tc(W1), nrhs=3, tol=1e-12)
    Dd = dense.DenseY(nside, wl.lmax, lmin=2)
    for c in range(3):
        ref = Dd.cr_solve(P.cl, P.bl, P.ninv, op.rhs(D3[c], W0[c], W1[c]))
        assert st[c].status == 0
        assert real_rel(op, s.cpu().numpy()[c], ref) < 1e-9


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_separate_terms(prec):
    # CR_SEPARATE: per column the mean field (d term) and the fluctuation (w0,
    # w1 terms) as two solutions; each against the oracle's dense solution of
    # its own right-hand side (FP64) or the oracle-evaluated residual (mixed),
    # with per-column amplitudes applied to both; their sum solves the full
    # right-hand side
    m = _m()
    nside = 8
    print("case separate terms", prec, flush=True)
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax, nrhs_max=4)
    amp = np.array([1.0, 1.7])
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), P.lmin, amp)
    rng = np.random.default_rng(13)
    W0 = np.stack([ci.white_alm(rng, wl.lmax) for _ in range(2)])
    W1 = np.stack([rng.standard_normal(P.ninv.size) for _ in range(2)])
    D2 = np.stack([d, -0.5 * d])
    pr = m.CR_F64 if prec == "f64" else m.CR_MIXED
    tol = 1e-12 if prec == "f64" else 1e-8
    s, st = m.solve(plan, gp, tc(D2), tc(W0), tc(W1), nrhs=2, tol=tol, prec=pr, terms=m.CR_SEPARATE)
    assert tuple(s.shape[:2]) == (2, 2) and len(st) == 4
    s = s.cpu().numpy()
    Dd = dense.DenseY(nside, wl.lmax, lmin=2)
    for c in range(2):
        cl_c = P.cl * amp[c]
        opc = cr.CROperator(cr.Problem(P.nside, P.lmax, cl_c, P.bl, P.ninv, P.lmin))
        bs = (opc.rhs(D2[c], None, None), opc.rhs(None, W0[c], W1[c]))
        for k, b in enumerate(bs):
            assert st[2 * c + k].status == 0
            if prec == "f64":
                ref = Dd.cr_solve(cl_c, P.bl, P.ninv, b)
                assert real_rel(opc, s[c, k], ref) < 1e-9, (c, k)
            else:
                res = real_rel(opc, opc.apply(s[c, k]), b)
                assert res <= 1.05e-8, (c, k, res)
        full = opc.rhs(D2[c], W0[c], W1[c])
        nb = [math.sqrt(opc.dot(b, b)) for b in bs]
        bound = 1.05 * tol * (nb[0] + nb[1]) / math.sqrt(opc.dot(full, full))
        assert real_rel(opc, opc.apply(s[c, 0] + s[c, 1]), full) <= bound
    with pytest.raises(m.CrshtError):   # 2 nrhs columns must fit the plan
        m.solve(plan, gp, tc(np.stack([d] * 3)), tc(np.stack([W0[0]] * 3)), None, nrhs=3, terms=m.CR_SEPARATE)


def test_fully_masked_gives_prior_draw():
    m = _m()
    nside = 8
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    gp = m.Problem(P.cl, P.bl, torch.zeros(P.ninv.size, dtype=torch.float64, device="cuda"), 2)
    w0 = wl.w0()
    s, st = m.solve(plan, gp, tc(d), tc(w0), tc(wl.w1()), tol=1e-14)
    ref = op.project(op.shalf * w0)
    assert rel(s.cpu().numpy()[0], ref) < 1e-12


def test_rhs_override_and_nonconvergence_status():
    m = _m()
    nside = 8
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    gp = _gpu_problem(m, P)
    b = op.rhs(d, wl.w0(), wl.w1())
    s, st = m.solve(plan, gp, rhs_vec=tc(b[None, :]), tol=1e-12)
    Dd = dense.DenseY(nside, wl.lmax, lmin=2)
    assert real_rel(op, s.cpu().numpy()[0], Dd.cr_solve(P.cl, P.bl, P.ninv, b)) < 1e-9
    s1, st1 = m.solve(plan, gp, rhs_vec=tc(b[None, :]), tol=1e-12, maxiter=1)
    assert st1[0].status == m.CR_NOCONV and st1[0].iters == 1


def test_invalid_spectrum_rejected():
    m = _m()
    nside = 4
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax)
    cl = P.cl.copy()
    cl[5] = -1.0
    gp = m.Problem(cl, P.bl, tc(P.ninv), 2)
    with pytest.raises(m.CrshtError):
        m.solve(plan, gp, tc(d))
    _ = math, healpix


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_column_amplitudes(prec):
    # per-column amplitudes (column c with C_l amp[c]): right-hand side and
    # operator of every column against the oracle's problem at amp[c] C_l;
    # solves (Jacobi, and the block preconditioner built at C_l) against the
    # dense Cholesky solution at amp[c] C_l; the same columns without amp
    # unchanged; a chain call given amplitudes is rejected
    m = _m()
    nside = 8
    print("case column amplitudes", prec, flush=True)
    wl, P, op, d = masked_problem(nside)
    amp = np.array([0.8, 1.0, 1.25])
    plan = m.Plan(nside, wl.lmax, nrhs_max=3)
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), P.lmin, amp)
    rng = np.random.default_rng(21)
    W0 = np.stack([ci.white_alm(rng, wl.lmax) for _ in range(3)])
    W1 = np.stack([rng.standard_normal(P.ninv.size) for _ in range(3)])
    D3 = np.stack([d, 0.5 * d, -d])
    ops = [cr.CROperator(cr.Problem(nside, wl.lmax, P.cl * a, P.bl, P.ninv, P.lmin)) for a in amp]
    Dd = dense.DenseY(nside, wl.lmax, lmin=2)
    if prec == "f64":
        got = m.rhs(plan, gp, tc(D3), tc(W0), tc(W1), nrhs=3).cpu().numpy()
        X = np.stack([ci.white_alm(rng, wl.lmax) for _ in range(3)])
        ax = m.apply(plan, gp, tc(X)).cpu().numpy()
        for c in range(3):
            assert rel(got[c], ops[c].rhs(D3[c], W0[c], W1[c])) < TOL
            assert rel(ax[c], ops[c].apply(X[c])) < TOL
    pr = m.CR_F64 if prec == "f64" else m.CR_MIXED
    tol = 1e-12 if prec == "f64" else 1e-8
    m.block_precond_build(plan, _gpu_problem(m, P))
    for pc in (m.CR_PC_JACOBI, m.CR_PC_BLOCK):
        s, st = m.solve(plan, gp, tc(D3), tc(W0), tc(W1), nrhs=3, tol=tol, prec=pr, precond=pc, max_refine=50)
        print("precond", pc, "iters", [x.iters for x in st], flush=True)
        for c in range(3):
            ref = Dd.cr_solve(P.cl * amp[c], P.bl, P.ninv, ops[c].rhs(D3[c], W0[c], W1[c]))
            assert st[c].status == 0
            assert real_rel(ops[c], s.cpu().numpy()[c], ref) < (1e-9 if prec == "f64" else 1e-6)
            x = s.cpu().numpy()[c]
            assert real_rel(ops[c], ops[c].apply(x), ops[c].rhs(D3[c], W0[c], W1[c])) <= 1.5 * tol
    # without amplitudes: every column at C_l
    s0, _ = m.solve(plan, _gpu_problem(m, P), tc(D3), tc(W0), tc(W1), nrhs=3, tol=1e-12)
    ref = Dd.cr_solve(P.cl, P.bl, P.ninv, op.rhs(D3[2], W0[2], W1[2]))
    assert real_rel(op, s0.cpu().numpy()[2], ref) < 1e-9
    ch = m.Chain(1.0, 0.0, tc(W0[0]), tc(W0[1]))
    with pytest.raises(RuntimeError):
        m.joint_step(plan, gp, tc(d), ch, 0.1, 0.5, tc(W0[0]), tc(W1[0]))
    with pytest.raises(RuntimeError):
        m.solve(plan, m.Problem(P.cl, P.bl, tc(P.ninv), P.lmin, np.array([1.0, -1.0, 1.0])), tc(D3), tc(W0),
                tc(W1), nrhs=3, tol=1e-8)
