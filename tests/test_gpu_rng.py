"""Device white draws (cr_white) against the Philox4x32-10 reference
(tests/philox_ref.py): every value of several columns, T and T+Q+U layouts,
determinism, and moments at a larger size."""
import numpy as np
import pytest
import torch

import crinputs as ci
from tests.philox_ref import white_alm, white_map

pytestmark = pytest.mark.gpu


def _m():
    from paper_2306_15511_amd import crsht as m
    return m


@pytest.mark.parametrize("ncomp", [1, 3])
def test_white_matches_reference(ncomp):
    m = _m()
    nside, lmax, n = 8, 23, 3
    print("case white ncomp", ncomp, flush=True)
    plan = m.Plan(nside, lmax, nrhs_max=n, ncomp=ncomp)
    seed, counter = 0x1234_5678_9ABC_DEF0, (7 << 32) | 11
    w0, w1 = m.white(plan, n, seed, counter)
    a = w0.cpu().numpy().reshape(n * ncomp, -1)
    x = w1.cpu().numpy().reshape(n * ncomp, -1)
    _, ms = ci.alm_lm_arrays(lmax)
    for c in range(n * ncomp):
        assert np.max(np.abs(a[c] - white_alm(ms, c, seed, counter))) < 1e-12, c
        assert np.max(np.abs(x[c] - white_map(plan.npix, c, seed, counter))) < 1e-12, c
    v0, v1 = m.white(plan, n, seed, counter)
    assert torch.equal(v0, w0) and torch.equal(v1, w1)
    u0, _ = m.white(plan, n, seed, counter + 1, pix=False)
    assert not torch.allclose(u0, w0)


def test_white_moments_nside256():
    m = _m()
    plan = m.Plan(256, 767, nrhs_max=2)
    w0, w1 = m.white(plan, 2, 42, 0)
    n = w1.numel()
    assert abs(float(w1.mean())) < 5.0 / n ** 0.5
    assert abs(float(w1.var()) - 1.0) < 5.0 * (2.0 / n) ** 0.5
    _, ms = ci.alm_lm_arrays(767)
    sel = torch.from_numpy(ms > 0).to(w0.device)
    re = w0[:, sel].real
    assert abs(float(re.var()) - 0.5) < 5.0 * (2.0 / re.numel()) ** 0.5
