"""CPU pins of the chain driver's host-side pieces: the integrated
autocorrelation time against the closed form of an AR(1) process, the white
a_lm draw's layout and variances, and the per-bin spectrum scaling."""
import numpy as np

from paper_2306_15511_amd import chains


def test_integrated_autocorr_time_of_ar1():
    # x_t = rho x_{t-1} + sqrt(1 - rho^2) e_t has rho_k = rho^k and
    # tau = 1 + 2 sum rho^k = (1 + rho) / (1 - rho)
    rng = np.random.default_rng(3)
    for rho in (0.0, 0.5, 0.8):
        n = 200_000
        e = rng.standard_normal(n)
        x = np.empty(n)
        x[0] = e[0]
        for t in range(1, n):
            x[t] = rho * x[t - 1] + np.sqrt(1.0 - rho * rho) * e[t]
        tau = chains.integrated_autocorr_time(x)
        want = (1.0 + rho) / (1.0 - rho)
        assert abs(tau - want) < 0.08 * want, (rho, tau, want)
    assert chains.integrated_autocorr_time(np.ones(10)) == 1.0


def test_white_alm_layout_and_variance():
    lmax = 40
    a = chains.white_alm(np.random.default_rng(1), lmax)
    ms = np.concatenate([np.full(lmax - m + 1, m) for m in range(lmax + 1)])
    assert a.size == ms.size and np.all(a[ms == 0].imag == 0.0)
    big = np.concatenate([chains.white_alm(np.random.default_rng(s), lmax) for s in range(200)])
    mm = np.tile(ms, 200)
    assert abs(np.var(big[mm > 0].real) - 0.5) < 0.02 and abs(np.var(big[mm == 0].real) - 1.0) < 0.05


def test_bin_scaled_spectrum():
    class P:   # the fields bin_scaled reads
        cl = np.arange(1.0, 11.0)
        bl = np.ones(10)
        ninv = None
        lmin = 2
    out = chains.bin_scaled(P, [2, 5, 8], [np.log(2.0), np.log(0.5)])
    want = P.cl.copy()
    want[2:5] *= 2.0
    want[5:8] *= 0.5
    assert np.allclose(np.asarray(out.cl), want)
