"""Graph-captured PCG iteration blocks (cr_opts.use_graph): every replay must
give exactly what direct launches give. Each solve replays its captured block
many times, with the host's convergence checks, residual replacements and
scalar reads (eager work and synchronisations) between replays; consecutive
solves reuse or re-capture the graph. The kernels reduce in a fixed order, so
the comparison is bit for bit."""
import numpy as np
import pytest
import torch

import crinputs as ci
from tests.gpu_helpers import masked_problem, tc

pytestmark = pytest.mark.gpu


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


def _inputs(wl, d, nrhs):
    w0 = np.stack([ci.white_alm(np.random.default_rng(10 + c), wl.lmax) for c in range(nrhs)])
    w1 = np.stack([np.random.default_rng(20 + c).standard_normal(d.size) for c in range(nrhs)])
    D = np.stack([d] * nrhs)
    return tc(D), tc(w0), tc(w1)


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_graph_solves_identical_to_direct(prec):
    m = _m()
    nside = 32
    print("case graph", prec, flush=True)
    wl, P, op, d = masked_problem(nside)
    plan = m.Plan(nside, wl.lmax, nrhs_max=3)
    gp = m.Problem(P.cl, P.bl, tc(P.ninv), P.lmin)
    p = m.CR_MIXED if prec == "mixed" else m.CR_F64
    D, W0, W1 = _inputs(wl, d, 3)
    ref, st_ref = m.solve(plan, gp, D, W0, W1, nrhs=3, tol=1e-8, maxiter=20000, prec=p, use_graph=False)
    ref = ref.clone()
    for rep in range(2):   # second run replays the cached graph
        got, st = m.solve(plan, gp, D, W0, W1, nrhs=3, tol=1e-8, maxiter=20000, prec=p, use_graph=True)
        assert torch.equal(got, ref), rep
        assert [s.iters for s in st] == [s.iters for s in st_ref]
        assert [s.rel_resid_true for s in st] == [s.rel_resid_true for s in st_ref]
    # a different column count re-captures; results still match direct launches
    one, st1 = m.solve(plan, gp, D[:1], W0[:1], W1[:1], nrhs=1, tol=1e-8, maxiter=20000, prec=p, use_graph=True)
    one_ref, _ = m.solve(plan, gp, D[:1], W0[:1], W1[:1], nrhs=1, tol=1e-8, maxiter=20000, prec=p,
                         use_graph=False)
    assert torch.equal(one, one_ref)
    got, _ = m.solve(plan, gp, D, W0, W1, nrhs=3, tol=1e-8, maxiter=20000, prec=p, use_graph=True)
    assert torch.equal(got, ref)


def test_graph_tqu_mixed_identical_to_direct():
    m = _m()
    from tests.test_gpu_tqu import _gpu_problem, _problem, _data
    nside = 16
    wl, P, op = _problem(nside)
    plan = m.Plan(nside, P.lmax, nrhs_max=2, ncomp=3)
    gp = _gpu_problem(m, P)
    rng = np.random.default_rng(3)
    d = tc(np.stack([_data(rng, op, P) for _ in range(2)]))
    w0 = tc(np.stack([np.stack([ci.white_alm(rng, P.lmax) for _ in range(3)]) for _ in range(2)]))
    w1 = tc(rng.standard_normal((2, 3, op.sht.npix)))
    ref, st_ref = m.solve(plan, gp, d, w0, w1, nrhs=2, tol=1e-7, maxiter=20000, prec=m.CR_MIXED, use_graph=False)
    ref = ref.clone()
    for rep in range(2):
        got, st = m.solve(plan, gp, d, w0, w1, nrhs=2, tol=1e-7, maxiter=20000, prec=m.CR_MIXED, use_graph=True)
        assert torch.equal(got, ref), rep
        assert [s.iters for s in st] == [s.iters for s in st_ref]
