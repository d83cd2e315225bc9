"""Normalised associated Legendre functions lambda_lm(z) = Delta_lm P_lm(z).

Definition (paper, App. A): Y_lm = P~_lm e^{i m phi}, P~_lm = Delta_lm P_lm(cos theta),
Delta_lm = (-1)^m sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), with P_lm the associated
Legendre functions without the Condon-Shortley phase, so Y_lm carries exactly
one factor (-1)^m (the convention of SciPy's ``sph_harm_y``).

Evaluation: the textbook three-term recurrence for the normalised functions,

    lambda_00     = 1 / sqrt(4 pi)
    lambda_mm     = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1}
    lambda_lm     = a_lm (z lambda_{l-1,m} - b_lm lambda_{l-2,m}),   l > m
    a_lm          = sqrt((4 l^2 - 1) / (l^2 - m^2))
    b_lm          = sqrt(((l-1)^2 - m^2) / (4 (l-1)^2 - 1))

(for l = m+1 the b term vanishes, giving lambda_{m+1,m} = sqrt(2m+3) z lambda_mm).
sin^m(theta) underflows double precision near the poles at large m, so every
value is carried as an extended-exponent number f * 2^e (f a double, e an
int64), renormalised after each step; only the final values are rounded to
double (values below the double range become 0 or subnormal, which is below
any tolerance used here).
"""
from __future__ import annotations

import math

import numpy as np

_ZERO_EXP = -(1 << 40)   # exponent given to an exact zero


def _norm(f: np.ndarray, e: np.ndarray):
    mant, ex = np.frexp(f)
    e2 = e + ex.astype(np.int64)
    e2 = np.where(mant == 0.0, _ZERO_EXP, e2)
    return mant, e2


def _to_double(f: np.ndarray, e: np.ndarray) -> np.ndarray:
    ee = np.clip(e, -2000, 2000).astype(np.int32)
    return np.ldexp(f, ee)


def lambda_rows_x(lmax: int, mmax: int, z: np.ndarray, sin_theta: np.ndarray):
    """Generator over l = 0..lmax yielding (l, f, e) with f, e of shape
    (min(l, mmax)+1, nz): lambda_lm(z[k]) = f[m, k] * 2**e[m, k] exactly as
    carried (no underflow)."""
    z = np.asarray(z, dtype=np.float64)
    st = np.asarray(sin_theta, dtype=np.float64)
    nz = z.size
    nm = mmax + 1
    # extended-exponent state for rows m: current (l-1) and previous (l-2)
    f1 = np.zeros((nm, nz)); e1 = np.full((nm, nz), _ZERO_EXP, dtype=np.int64)
    f0 = np.zeros((nm, nz)); e0 = np.full((nm, nz), _ZERO_EXP, dtype=np.int64)
    # diagonal lambda_mm, advanced with m
    fd, ed = _norm(np.full(nz, 1.0 / math.sqrt(4.0 * math.pi)), np.zeros(nz, dtype=np.int64))
    for l in range(lmax + 1):
        top = min(l, mmax)
        fn = np.zeros((top + 1, nz)); en = np.full((top + 1, nz), _ZERO_EXP, dtype=np.int64)
        if l <= mmax:
            if l > 0:
                fd, ed = _norm(-math.sqrt((2.0 * l + 1.0) / (2.0 * l)) * st * fd, ed)
            fn[l], en[l] = fd, ed
        nr = min(l, nm)          # rows m < l use the three-term recurrence
        if nr > 0:
            m = np.arange(nr, dtype=np.float64)[:, None]
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            lm1 = l - 1.0
            b = np.sqrt(np.clip(lm1 * lm1 - m * m, 0.0, None) / (4.0 * lm1 * lm1 - 1.0)) if l > 1 else np.zeros_like(m)
            emax = np.maximum(e1[:nr], e0[:nr])
            t1 = np.ldexp(z[None, :] * f1[:nr], np.clip(e1[:nr] - emax, -2000, 0).astype(np.int32))
            t0 = np.ldexp(b * f0[:nr], np.clip(e0[:nr] - emax, -2000, 0).astype(np.int32))
            fn[:nr], en[:nr] = _norm(a * (t1 - t0), emax)
        # shift the state
        f0[:top + 1], e0[:top + 1] = f1[:top + 1], e1[:top + 1]
        f1[:top + 1], e1[:top + 1] = fn, en
        yield l, fn, en


def lambda_rows(lmax: int, mmax: int, z: np.ndarray, sin_theta: np.ndarray):
    """Generator over l = 0..lmax yielding (l, lam) with lam of shape
    (min(l, mmax)+1, nz): lam[m, k] = lambda_lm(z[k]) rounded to double."""
    for l, f, e in lambda_rows_x(lmax, mmax, z, sin_theta):
        yield l, _to_double(f, e)


def log10_abs_lambda(l: int, m: int, z: float) -> float:
    """log10 |lambda_lm(z)| from the extended-exponent value (valid far below
    the double range)."""
    st = math.sqrt(max(0.0, (1.0 - z) * (1.0 + z)))
    for ll, f, e in lambda_rows_x(l, m, np.array([z]), np.array([st])):
        if ll == l:
            return math.log10(abs(float(f[m, 0]))) + float(e[m, 0]) * math.log10(2.0)
    raise AssertionError

def lambda_table(lmax: int, mmax: int, z: np.ndarray, sin_theta: np.ndarray) -> np.ndarray:
    """Dense table lam[l, m, k] (zero for m > l). For small problems only."""
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros((lmax + 1, mmax + 1, z.size))
    for l, lam in lambda_rows(lmax, mmax, z, sin_theta):
        out[l, :lam.shape[0]] = lam
    return out


def lambda_single(l: int, m: int, z: float) -> float:
    """lambda_lm at one point (closed-form checks)."""
    st = math.sqrt(max(0.0, (1.0 - z) * (1.0 + z)))
    for ll, lam in lambda_rows(l, m, np.array([z]), np.array([st])):
        if ll == l:
            return float(lam[m, 0])
    raise AssertionError
