"""Plain-C Legendre sums of the oracle (``legendre_sums.c``), loaded by ctypes.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

The C file evaluates the same recurrence and the same two sums as
``legendre.lambda_rows`` and ``sht.SHT.legendre_synth`` /
``legendre_adjoint`` (paper App. A normalisation), as plain loops over
(m, ring, l) so that the transforms of the Nside 512 and 1024 workloads take
seconds instead of minutes. It is compiled with gcc (strict IEEE double: no
-ffast-math, no FMA contraction on the x86-64 baseline) the first time it is
needed, or by ``build()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "legendre_sums.c")
LIB = os.path.join(HERE, "liblegendre_sums.so")

_lib = None


def build() -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle C build failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oc_legendre_synth.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
    lib.oc_legendre_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_int, dp]
    lib.oc_lambda_m.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
    for f in (lib.oc_legendre_synth, lib.oc_legendre_adjoint, lib.oc_lambda_m):
        f.restype = None
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def legendre_synth(lmax: int, mmax: int, z, sin_theta, alm) -> np.ndarray:
    """F[m, r] = sum_l lambda_lm(z_r) alm[l, m] (complex, [mmax+1, nring])."""
    lib = _load()
    z, st = _f64(z), _f64(sin_theta)
    a = np.ascontiguousarray(alm, dtype=np.complex128)
    F = np.empty((mmax + 1, z.size), dtype=np.complex128)
    lib.oc_legendre_synth(lmax, mmax, z.size, _p(z), _p(st), _p(a.view(np.float64)), _p(F.view(np.float64)))
    return F


def legendre_adjoint(lmax: int, mmax: int, z, sin_theta, G, square: bool = False) -> np.ndarray:
    """out[l, m] = sum_r lambda_lm(z_r) G[m, r] (complex, m-major)."""
    lib = _load()
    z, st = _f64(z), _f64(sin_theta)
    g = np.ascontiguousarray(G, dtype=np.complex128)
    n = (mmax + 1) * (lmax + 1) - (mmax * (mmax + 1)) // 2
    out = np.empty(n, dtype=np.complex128)
    lib.oc_legendre_adjoint(lmax, mmax, z.size, _p(z), _p(st), _p(g.view(np.float64)), 1 if square else 0,
                            _p(out.view(np.float64)))
    return out


def lambda_m(lmax: int, m: int, z, sin_theta) -> np.ndarray:
    """lambda_lm(z_k) for one m: array [lmax - m + 1, nz]."""
    lib = _load()
    z, st = _f64(z), _f64(sin_theta)
    out = np.empty((lmax - m + 1, z.size))
    lib.oc_lambda_m(lmax, m, z.size, _p(z), _p(st), _p(out))
    return out
