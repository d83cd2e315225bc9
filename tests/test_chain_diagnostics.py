"""CPU pins of the chain driver's host-side pieces: the integrated
autocorrelation time and the correlation length (first lag with zeta < 0.1)
against the closed forms of an AR(1) process, zeta against its definition
summed pair by pair, the white a_lm draw's layout and variances, and the
per-bin spectrum scaling."""
import math

import numpy as np
from scipy.signal import lfilter

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


def _ar1(rng, rho, n):
    e = rng.standard_normal(n) * math.sqrt(1.0 - rho * rho)
    return lfilter([1.0], [1.0, -rho], e)


def test_autocorrelation_matches_pairwise_definition():
    # zeta(D) = mean over i of (x_i - mu)(x_{i+D} - mu) / sigma^2, written out
    x = _ar1(np.random.default_rng(7), 0.6, 300) + 3.0
    mu, sd = x.mean(), x.std()
    want = [np.mean([(x[i] - mu) * (x[i + d] - mu) for i in range(x.size - d)]) / sd ** 2 for d in range(x.size)]
    assert np.allclose(chains.autocorrelation(x), want, rtol=0, atol=1e-12)


def test_correlation_length_of_ar1():
    # zeta(D) = rho^D: the first D with rho^D < 0.1 is 4 for rho = 0.5
    # (0.125, 0.0625), 7 for rho = 0.7 (0.118, 0.082) and 11 for rho = 0.8
    # (0.107, 0.086); the estimate's standard deviation at 1e6 samples is
    # about 0.002 (Bartlett), well inside those gaps; white noise: 1
    rng = np.random.default_rng(11)
    for rho, want in ((0.5, 4), (0.7, 7), (0.8, 11)):
        assert chains.correlation_length(_ar1(rng, rho, 1_000_000)) == want, rho
    assert chains.correlation_length(rng.standard_normal(100_000)) == 1
    assert chains.correlation_length(np.ones(10)) == 10
