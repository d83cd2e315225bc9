"""The allocation-free synthesis (sht_synth_noalloc, through the C ABI)
against the plan-workspace synthesis sht_synth: the same kernels on the same
inputs, so the maps agree to the FP64 bar of 1e-10 (measured: bit for bit),
on two calls in a row with the second on a smaller input (a smaller plan and
fewer columns) that must not see the first call's scratch contents; both
precisions; inputs beyond the static scratch rejected with CR_ESCRATCH."""
import numpy as np
import pytest
import torch

import crinputs as ci
from tests.gpu_helpers import rel, tc

pytestmark = pytest.mark.gpu


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


def _case(m, plan, lmax, ncols, seed, prec):
    rng = np.random.default_rng(seed)
    a = tc(np.stack([ci.white_alm(rng, lmax) for _ in range(ncols)]))
    ref = m.synth(plan, a, prec=prec)
    out = torch.full_like(ref, float("nan"))
    got = m.synth_noalloc(plan, a, out, prec=prec)
    torch.cuda.synchronize()
    e = max(rel(got[c].cpu().numpy(), ref[c].cpu().numpy()) for c in range(ncols))
    print("noalloc vs synth: %d columns, prec %d, rel %.2e, identical %s" % (ncols, prec, e, torch.equal(got, ref)),
          flush=True)
    return e


def test_noalloc_synthesis_matches_synth_twice_second_smaller():
    m = _m()
    print("case noalloc nside512 then nside32", flush=True)
    big = m.Plan(512, 1535, nrhs_max=3)
    small = m.Plan(32, 95, nrhs_max=2)
    # first call: the largest FP64 input that fits (one column at Nside 512)
    assert _case(m, big, 1535, 1, 1, m.CR_F64) < 1e-10
    # second call, smaller input: a smaller plan and fewer scratch bytes
    assert _case(m, small, 95, 2, 2, m.CR_F64) < 1e-10
    # the mixed path: three columns at Nside 512, then one at Nside 32
    assert _case(m, big, 1535, 3, 3, m.CR_MIXED) < 1e-10
    assert _case(m, small, 95, 1, 4, m.CR_MIXED) < 1e-10
    # beyond the scratch: two FP64 columns at Nside 512
    a = torch.zeros((2, big.nalm), dtype=torch.complex128, device="cuda:0")
    out = torch.empty((2, big.npix), dtype=torch.float64, device="cuda:0")
    with pytest.raises(m.CrshtError) as ei:
        m.synth_noalloc(big, a, out)
    assert ei.value.code == m.CR_ESCRATCH
    big.close()
    small.close()
