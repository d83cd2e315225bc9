"""Seeded synthetic workloads for the constrained-realization solve.

This module is shared by the CPU oracle (under ``oracle/``), the tests and the
benchmark. It holds only the *problem definitions* (spectra, beams, noise
patterns, masks) and the random draws. It performs none of the method's
arithmetic: no spherical-harmonic transform, no pixel geometry, no solve.
Quantities that depend on pixel positions take the pixel coordinates as
arguments, so each caller supplies them from its own geometry code.

Conventions (paper: simplified data model r = B a + n, Sect. 2.2.1; the
constrained-realization equation and its white-noise terms w0, w1):

* a_lm of a real field are stored for m >= 0 only, m-major (for m = 0..mmax,
  l = m..lmax), as complex128.
* A unit-variance complex draw has Re, Im ~ N(0, 1/2) for m > 0 and a real
  N(0, 1) value for m = 0; this makes every real degree of freedom unit
  variance under the inner product <a,c> = sum_l a_l0 c_l0
  + 2 sum_{m>0} Re(a_lm conj(c_lm)).
* Maps are float64 in HEALPix RING order, units of micro-Kelvin.

Seeds follow ``numpy.random.default_rng([230615511, cfg, prob, stream])`` with
streams 0 = signal a_lm, 1 = noise map, 2 = w0, 3 = w1, 4 = Metropolis draws,
5 = per-problem parameters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 230615511
STREAM_SIGNAL, STREAM_NOISE, STREAM_W0, STREAM_W1, STREAM_MH, STREAM_PARAMS = range(6)

ARCMIN = math.pi / (180.0 * 60.0)
DEG = math.pi / 180.0
OBLIQUITY = 23.44 * DEG


def rng_for(cfg: int, prob: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, cfg, prob, stream])


def nalm(lmax: int, mmax: int | None = None) -> int:
    mmax = lmax if mmax is None else mmax
    return (mmax + 1) * (lmax + 1) - (mmax * (mmax + 1)) // 2


def alm_lm_arrays(lmax: int, mmax: int | None = None):
    """(l, m) of every stored coefficient in m-major order."""
    mmax = lmax if mmax is None else mmax
    ls, ms = [], []
    for m in range(mmax + 1):
        ls.append(np.arange(m, lmax + 1))
        ms.append(np.full(lmax + 1 - m, m))
    return np.concatenate(ls), np.concatenate(ms)


# --------------------------------------------------------------------------
# Spectra and beams
# --------------------------------------------------------------------------

def amplitude_for_rms(lmax: int, rms_uk: float = 100.0, lmin: int = 2) -> float:
    """Amplitude A of C_l = A/(l(l+1)) whose expected unbeamed pixel variance
    sum_l (2l+1)/(4 pi) C_l equals rms_uk**2."""
    ell = np.arange(lmin, lmax + 1, dtype=np.float64)
    return 4.0 * math.pi * rms_uk ** 2 / float(np.sum((2 * ell + 1) / (ell * (ell + 1))))


def cl_powerlaw(lmax: int, amp: float, lmin: int = 2) -> np.ndarray:
    """C_l = amp / (l (l+1)) for l >= lmin, 0 below."""
    cl = np.zeros(lmax + 1)
    ell = np.arange(lmin, lmax + 1, dtype=np.float64)
    cl[lmin:] = amp / (ell * (ell + 1))
    return cl


def cl_tqu(lmax: int, amp: float, te_corr: float = 0.3, lmin: int = 2) -> np.ndarray:
    """[4][lmax+1] spectra TT, EE, BB, TE of the polarised workload:
    C^TT = A/(l(l+1)), C^EE = 0.05 C^TT, C^BB = 0.005 C^TT,
    C^TE = te_corr sqrt(C^TT C^EE) (zero below lmin)."""
    tt = cl_powerlaw(lmax, amp, lmin)
    ee, bb = 0.05 * tt, 0.005 * tt
    return np.stack([tt, ee, bb, te_corr * np.sqrt(tt * ee)])


def gaussian_beam(lmax: int, fwhm_rad: float) -> np.ndarray:
    """b_l = exp(-l(l+1) sigma_b^2 / 2), sigma_b = FWHM / sqrt(8 ln 2); no pixel window."""
    sig = fwhm_rad / math.sqrt(8.0 * math.log(2.0))
    ell = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * ell * (ell + 1) * sig * sig)


# --------------------------------------------------------------------------
# Random draws
# --------------------------------------------------------------------------

def white_alm(rng: np.random.Generator, lmax: int, mmax: int | None = None, lmin: int = 0) -> np.ndarray:
    """Unit-variance real-field complex draw (m = 0 real), zero for l < lmin."""
    ls, ms = alm_lm_arrays(lmax, mmax)
    n = ls.size
    g = rng.standard_normal((2, n))
    out = (g[0] + 1j * g[1]) / math.sqrt(2.0)
    m0 = ms == 0
    out[m0] = g[0][m0]
    out[ls < lmin] = 0.0
    return out


def white_map(rng: np.random.Generator, npix: int) -> np.ndarray:
    return rng.standard_normal(npix)


def signal_alm(rng: np.random.Generator, cl: np.ndarray, lmax: int, mmax: int | None = None) -> np.ndarray:
    """a_lm = sqrt(C_l) * unit draw (C_l <= 0 gives 0)."""
    ls, _ = alm_lm_arrays(lmax, mmax)
    return np.sqrt(np.clip(cl, 0.0, None))[ls] * white_alm(rng, lmax, mmax)


def signal_alm_tqu(rng: np.random.Generator, cl4: np.ndarray, lmax: int) -> np.ndarray:
    """(a_T, a_E, a_B) [3][nalm] drawn from the 3x3 blocks of cl4 = (TT, EE,
    BB, TE): a_T = sqrt(TT) g1, a_E = TE/sqrt(TT) g1 + sqrt(EE - TE^2/TT) g2,
    a_B = sqrt(BB) g3 with unit real-field draws g (0 where TT <= 0)."""
    ls, _ = alm_lm_arrays(lmax)
    tt, ee, bb, te = (np.asarray(c, dtype=np.float64) for c in cl4)
    ok = tt > 0
    st = np.sqrt(np.where(ok, tt, 0.0))
    x = np.where(ok, te / np.where(ok, st, 1.0), 0.0)
    y = np.sqrt(np.clip(ee - x * x, 0.0, None))
    g = [white_alm(rng, lmax) for _ in range(3)]
    return np.stack([st[ls] * g[0], x[ls] * g[0] + y[ls] * g[1], np.sqrt(np.clip(bb, 0.0, None))[ls] * g[2]])


# --------------------------------------------------------------------------
# Noise and mask patterns, given pixel coordinates (z = cos theta, phi)
# --------------------------------------------------------------------------

def ecliptic_like_latitude(z: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """beta = asin(z cos eps - y sin eps): latitude after a rotation by the
    obliquity eps about the x axis; y = sin(theta) sin(phi)."""
    y = np.sqrt(np.clip(1.0 - z * z, 0.0, None)) * np.sin(phi)
    return np.arcsin(np.clip(z * math.cos(OBLIQUITY) - y * math.sin(OBLIQUITY), -1.0, 1.0))


def hit_pattern(z: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """h_p = 1 + 4 sin^2(beta) in [1, 5]."""
    return 1.0 + 4.0 * np.sin(ecliptic_like_latitude(z, phi)) ** 2


def band_mask(z: np.ndarray, b_deg: float | None = None, sin_b: float | None = None) -> np.ndarray:
    """1 outside the constant-latitude band |lat| < b (kept), 0 inside
    (the constant-latitude mask of the paper's Appendix A: a pixel is masked
    when |theta - pi/2| < b, strictly)."""
    if sin_b is None:
        sin_b = 0.0 if b_deg is None else math.sin(b_deg * DEG)
    return (np.abs(z) >= sin_b).astype(np.float64)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    nside: int
    lmax: int
    cfg: int
    prob: int = 0
    amp: float = 0.0
    fwhm_rad: float = 0.0
    sigma_uk: float = 10.0          # uniform white noise sigma (when hits is False)
    anisotropic: bool = False       # sigma_p = sigma0 / sqrt(h_p)
    sigma0_uk: float = 30.0
    mask_b_deg: float | None = None
    mask_sin_b: float | None = None
    tol: float = 1e-6
    lmin: int = 2
    extra: dict = field(default_factory=dict)

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside

    def cl(self) -> np.ndarray:
        return cl_powerlaw(self.lmax, self.amp, self.lmin)

    def bl(self) -> np.ndarray:
        return gaussian_beam(self.lmax, self.fwhm_rad)

    def sigma_map(self, z: np.ndarray, phi: np.ndarray) -> np.ndarray:
        if self.anisotropic:
            return self.sigma0_uk / np.sqrt(hit_pattern(z, phi))
        return np.full(z.shape, self.sigma_uk)

    def ninv(self, z: np.ndarray, phi: np.ndarray) -> np.ndarray:
        """Inverse noise variance per pixel, 0 where masked."""
        sig = self.sigma_map(z, phi)
        keep = band_mask(z, self.mask_b_deg, self.mask_sin_b)
        return keep / (sig * sig)

    def rng(self, stream: int) -> np.random.Generator:
        return rng_for(self.cfg, self.prob, stream)

    def signal(self) -> np.ndarray:
        return signal_alm(self.rng(STREAM_SIGNAL), self.cl(), self.lmax)

    def noise(self, z: np.ndarray, phi: np.ndarray) -> np.ndarray:
        return self.sigma_map(z, phi) * white_map(self.rng(STREAM_NOISE), self.npix)

    def w0(self) -> np.ndarray:
        return white_alm(self.rng(STREAM_W0), self.lmax)

    def w1(self) -> np.ndarray:
        return white_map(self.rng(STREAM_W1), self.npix)


def workload_plain_t(nside: int = 16, lmax: int | None = None) -> Workload:
    """Plain method, temperature only, FP64: Nside 16, lmax 47, full sky,
    uniform white noise sigma = 10 uK, Gaussian beam FWHM 5 deg, pixel rms
    100 uK, solve to 1e-8."""
    lmax = 3 * nside - 1 if lmax is None else lmax
    return Workload("plain_t_nside%d" % nside, nside, lmax, cfg=0,
                    amp=amplitude_for_rms(lmax), fwhm_rad=5.0 * DEG,
                    sigma_uk=10.0, tol=1e-8)


def workload_masked_t(nside: int = 256, lmax: int | None = None, fwhm_arcmin: float = 30.0,
                      cfg: int = 1) -> Workload:
    """Temperature, anisotropic noise sigma_p = 30 uK / sqrt(h_p),
    h_p = 1 + 4 sin^2(ecliptic-like latitude), N^-1 = 0 in |b| < 20 deg,
    C_l = A/(l(l+1)) with pixel rms 100 uK; solve to 1e-6."""
    lmax = 3 * nside - 1 if lmax is None else lmax
    return Workload("masked_t_nside%d" % nside, nside, lmax, cfg=cfg,
                    amp=amplitude_for_rms(lmax), fwhm_rad=fwhm_arcmin * ARCMIN,
                    anisotropic=True, sigma0_uk=30.0, mask_b_deg=20.0, tol=1e-6)


def workload_headline_t() -> Workload:
    """Nside 512, lmax 1535, temperature part of the differentiation
    workload: hit pattern and 20 deg band mask as above, FWHM 10 arcmin."""
    return workload_masked_t(512, 1535, fwhm_arcmin=10.0, cfg=2)


def workload_batched(j: int) -> Workload:
    """Problem j of the 64 uneven batched solves: Nside = (64,128,256,512)[j//16],
    lmax = 3 Nside - 1, amplitude U[0.5,2] x A(lmax), white sigma U[5,50] uK,
    band mask of sky fraction f ~ U[0, 0.3] (masked iff |z| < f), FWHM
    30 arcmin x 256/Nside, solve to 1e-6."""
    nside = (64, 128, 256, 512)[j // 16]
    lmax = 3 * nside - 1
    r = rng_for(3, j, STREAM_PARAMS)
    qa, sig, f = r.uniform(0.5, 2.0), r.uniform(5.0, 50.0), r.uniform(0.0, 0.3)
    return Workload("batched_%02d" % j, nside, lmax, cfg=3, prob=j,
                    amp=qa * amplitude_for_rms(lmax), fwhm_rad=30.0 * ARCMIN * 256.0 / nside,
                    sigma_uk=sig, mask_sin_b=f, tol=1e-6)
