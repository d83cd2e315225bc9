"""Python binding of libcrsht (include/crsht.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every computation runs in
the library's HIP kernels. a_lm tensors are complex128 of shape [nalm] or
[nrhs, nalm] (m-major, m >= 0); maps are float64 [npix] or [nrhs, npix] in
HEALPix RING order. Plans with ncomp = 3 (T, E, B / T, Q, U) take a_lm of
shape [3, nalm] or [nrhs, 3, nalm] and maps [3, npix] or [nrhs, 3, npix]. The library must be built (``python -m
paper_2306_15511_amd.build``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CRSHT_LIB") or os.path.join(_HERE, "libcrsht.so")

CR_OK, CR_EINVAL, CR_ENOMEM, CR_EDEVICE, CR_ENOTSUP, CR_ESCRATCH = 0, -1, -2, -3, -4, -5
CR_NOCONV, CR_BREAKDOWN = 1, 2
CR_F64, CR_MIXED, CR_BF16X6 = 0, 1, 3
CR_PC_JACOBI, CR_PC_BLOCK = 0, 1
CR_SUM, CR_SEPARATE = 0, 4


class CrshtError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__("%s failed: %s (%d)" % (where, strerror(code), code))
        self.code = code


class _Info(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int), ("lmax", ctypes.c_int), ("mmax", ctypes.c_int), ("ncomp", ctypes.c_int),
                ("nrhs_max", ctypes.c_int), ("nrings", ctypes.c_int), ("npix", ctypes.c_int64),
                ("nalm", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64), ("precond_bytes", ctypes.c_int64),
                ("precond_blocks", ctypes.c_int), ("precond_half_blocks", ctypes.c_int),
                ("live_pair_m", ctypes.c_int64)]


class _Problem(ctypes.Structure):
    _fields_ = [("cl", ctypes.POINTER(ctypes.c_double)), ("bl", ctypes.POINTER(ctypes.c_double)),
                ("ninv", ctypes.c_void_p), ("lmin", ctypes.c_int), ("amp", ctypes.POINTER(ctypes.c_double))]


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("prec", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int), ("check_every", ctypes.c_int),
                ("precond", ctypes.c_int), ("use_graph", ctypes.c_int), ("terms", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("refinements", ctypes.c_int),
                ("rel_resid_true", ctypes.c_double)]


class _Tuning(ctypes.Structure):
    _fields_ = [("nclasses", ctypes.c_int), ("fft_len", ctypes.c_int * 8), ("ring_div", ctypes.c_int * 8),
                ("f64_synth_cols", ctypes.c_int), ("f64_adj_cols", ctypes.c_int), ("from_cache", ctypes.c_int),
                ("ms_default", ctypes.c_double), ("ms_tuned", ctypes.c_double)]


class _Chain(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("lnpi", ctypes.c_double), ("ahat", ctypes.c_void_p),
                ("fhat", ctypes.c_void_p)]


class _Draws(ctypes.Structure):
    _fields_ = [("xi", ctypes.c_double), ("u", ctypes.c_double), ("w0", ctypes.c_void_p),
                ("w1", ctypes.c_void_p), ("sigma_lnq", ctypes.c_double)]


class _StepOut(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int), ("lnA", ctypes.c_double), ("q_new", ctypes.c_double),
                ("lnpi_new", ctypes.c_double), ("mean_stats", _Stats), ("fluct_stats", _Stats)]


class _BinChain(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int), ("edges", ctypes.POINTER(ctypes.c_int)),
                ("theta", ctypes.POINTER(ctypes.c_double)), ("lnpi", ctypes.c_double), ("ahat", ctypes.c_void_p),
                ("fhat", ctypes.c_void_p)]


class _HmcDraws(ctypes.Structure):
    _fields_ = [("p0", ctypes.POINTER(ctypes.c_double)), ("u", ctypes.c_double), ("w0", ctypes.c_void_p),
                ("w1", ctypes.c_void_p), ("eps", ctypes.c_double), ("nleap", ctypes.c_int)]


class _HmcOut(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int), ("status", ctypes.c_int), ("dH", ctypes.c_double),
                ("lnpi_new", ctypes.c_double), ("solves", ctypes.c_int), ("iters", ctypes.c_int),
                ("fluct_stats", _Stats)]


class _GibbsOut(ctypes.Structure):
    _fields_ = [("q_new", ctypes.c_double), ("t", ctypes.c_double), ("mean_stats", _Stats),
                ("fluct_stats", _Stats)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcrsht.so is not built (%s); run python -m paper_2306_15511_amd.build" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, vp, i, d = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "crsht_plan_create": ([i, i, i, i, i, ctypes.POINTER(ctypes.c_void_p)], i),
        "crsht_plan_destroy": ([P], None),
        "crsht_strerror": ([i], ctypes.c_char_p),
        "crsht_plan_info": ([P, ctypes.POINTER(_Info)], i),
        "crsht_pixel_coords": ([P, vp, vp], i),
        "sht_synth": ([P, i, vp, vp, i, vp], i),
        "sht_synth_noalloc": ([P, i, vp, vp, i, vp], i),
        "sht_synth_adjoint": ([P, i, vp, vp, i, vp], i),
        "sht_analysis": ([P, i, vp, vp, i, vp], i),
        "cr_precond": ([P, ctypes.POINTER(_Problem), vp, vp], i),
        "cr_block_precond_build": ([P, ctypes.POINTER(_Problem), vp], i),
        "cr_block_precond_apply": ([P, i, vp, vp, vp], i),
        "cr_rhs": ([P, ctypes.POINTER(_Problem), i, vp, vp, vp, vp, vp], i),
        "cr_apply": ([P, ctypes.POINTER(_Problem), i, vp, vp, i, vp], i),
        "cr_solve": ([P, ctypes.POINTER(_Problem), i, vp, vp, vp, vp, vp, ctypes.POINTER(_Opts),
                      ctypes.POINTER(_Stats), vp], i),
        "cr_solve_async": ([P, ctypes.POINTER(_Problem), i, vp, vp, vp, vp, vp, ctypes.POINTER(_Opts), vp, vp], i),
        "cr_lnpi": ([P, ctypes.POINTER(_Problem), d, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp], i),
        "joint_cl_step": ([P, ctypes.POINTER(_Problem), vp, ctypes.POINTER(_Chain), ctypes.POINTER(_Draws),
                           ctypes.POINTER(_Opts), ctypes.POINTER(_StepOut), vp], i),
        "cr_lnpi_grad_fixed": ([P, ctypes.POINTER(_Problem), vp, i, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), vp, vp,
                                ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), vp, ctypes.POINTER(_Stats), vp], i),
        "hmc_cl_step": ([P, ctypes.POINTER(_Problem), vp, ctypes.POINTER(_BinChain), ctypes.POINTER(_HmcDraws),
                         ctypes.POINTER(_Opts), ctypes.POINTER(_HmcOut), vp], i),
        "gibbs_cl_step_batch": ([P, ctypes.POINTER(_Problem), vp, i, ctypes.POINTER(_Chain),
                                 ctypes.POINTER(ctypes.c_double), vp, vp, ctypes.POINTER(_Opts),
                                 ctypes.POINTER(_GibbsOut), vp], i),
        "gibbs_bins_step": ([P, ctypes.POINTER(_Problem), vp, ctypes.POINTER(_BinChain),
                             ctypes.POINTER(ctypes.c_double), vp, vp, ctypes.POINTER(_Opts),
                             ctypes.POINTER(ctypes.c_double), vp, vp], i),
        "cr_white": ([P, i, ctypes.c_uint64, ctypes.c_uint64, vp, vp, vp], i),
        "joint_cl_step_batch": ([P, ctypes.POINTER(_Problem), vp, i, ctypes.POINTER(_Chain),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), d, vp, vp,
                                 ctypes.POINTER(_Opts), ctypes.POINTER(_StepOut), vp], i),
        "gibbs_cl_step": ([P, ctypes.POINTER(_Problem), vp, ctypes.POINTER(_Chain), d, vp, vp,
                           ctypes.POINTER(_Opts), ctypes.POINTER(_GibbsOut), vp], i),
        "cr_solve_batched": ([ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(_Problem), i,
                              ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                              ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                              ctypes.POINTER(_Opts), ctypes.POINTER(_Stats), vp], i),
        "sht_synth_grad": ([P, i, vp, vp, i, vp], i),
        "cr_grad_chi2": ([P, ctypes.POINTER(_Problem), i, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp], i),
        "cr_grad_lnpi": ([P, ctypes.POINTER(_Problem), vp, vp, vp, i, ctypes.POINTER(ctypes.c_int),
                          ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(_Stats), vp], i),
        "crsht_autotune": ([P, i, i, ctypes.POINTER(_Tuning), vp], i),
        "crsht_get_tuning": ([P, ctypes.POINTER(_Tuning)], i),
        "crsht_set_tuning": ([P, ctypes.POINTER(_Tuning)], i),
        "crsht_timing_enable": ([P, i], i),
        "crsht_timing_read": ([P, i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()

EXPORTED = ("crsht_plan_create", "crsht_plan_destroy", "crsht_strerror", "crsht_plan_info", "crsht_pixel_coords",
            "sht_synth", "sht_synth_noalloc", "sht_synth_adjoint", "sht_analysis", "cr_precond", "cr_rhs", "cr_apply", "cr_solve",
            "cr_solve_async",
            "cr_white", "cr_lnpi", "joint_cl_step", "joint_cl_step_batch", "gibbs_cl_step", "gibbs_cl_step_batch", "gibbs_bins_step", "hmc_cl_step", "cr_lnpi_grad_fixed",
            "cr_solve_batched", "sht_synth_grad", "cr_grad_chi2", "cr_grad_lnpi",
            "cr_block_precond_build", "cr_block_precond_apply", "crsht_timing_enable", "crsht_timing_read",
            "crsht_autotune", "crsht_get_tuning", "crsht_set_tuning")


def lib():
    return _lib


def strerror(code: int) -> str:
    return _lib.crsht_strerror(int(code)).decode()


def _check(rc: int, where: str):
    if rc < 0:
        raise CrshtError(rc, where)
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _nrhs(t, per: int, dtype) -> int:
    if t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    if t.numel() % per or t.numel() == 0:
        raise ValueError("tensor size %d is not a multiple of %d" % (t.numel(), per))
    return t.numel() // per


class Plan:
    """Geometry, tables and workspace for one (nside, lmax, mmax, nrhs_max)."""

    def __init__(self, nside: int, lmax: int, mmax: int = -1, nrhs_max: int = 1, ncomp: int = 1):
        h = ctypes.c_void_p()
        _check(_lib.crsht_plan_create(nside, lmax, mmax, ncomp, nrhs_max, ctypes.byref(h)), "crsht_plan_create")
        self._h = h
        info = _Info()
        _check(_lib.crsht_plan_info(h, ctypes.byref(info)), "crsht_plan_info")
        self.nside, self.lmax, self.mmax = info.nside, info.lmax, info.mmax
        self.nrhs_max, self.nrings = info.nrhs_max, info.nrings
        self.npix, self.nalm = int(info.npix), int(info.nalm)
        self.ncomp = int(info.ncomp)
        self.vlen = self.ncomp * self.nalm      # coefficients per column
        self.mlen = self.ncomp * self.npix      # map values per column
        self.workspace_bytes = int(info.workspace_bytes)
        self.live_pair_m = int(info.live_pair_m)   # (ring pair, m) with live Legendre values

    def precond_info(self):
        """(bytes of the stored block-preconditioner inverses one application
        reads, blocks, blocks stored in FP16); zeros if none is built."""
        info = _Info()
        _check(_lib.crsht_plan_info(self._h, ctypes.byref(info)), "crsht_plan_info")
        return int(info.precond_bytes), int(info.precond_blocks), int(info.precond_half_blocks)

    def alm_shape(self, nrhs: int):
        return (nrhs, self.nalm) if self.ncomp == 1 else (nrhs, self.ncomp, self.nalm)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.crsht_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pixel_coords(self):
        import numpy as np
        z = np.empty(self.npix)
        phi = np.empty(self.npix)
        _check(_lib.crsht_pixel_coords(self._h, z.ctypes.data_as(ctypes.c_void_p), phi.ctypes.data_as(ctypes.c_void_p)),
               "crsht_pixel_coords")
        return z, phi


KERNEL_LEGENDRE_SYNTH, KERNEL_LEGENDRE_ADJOINT, KERNEL_RING = 0, 1, 2
KERNEL_MFMA_SYNTH, KERNEL_MFMA_ADJOINT = 3, 4
KERNEL_BLOCK_PC = 5


def timing_enable(plan: Plan, on: bool = True):
    _check(_lib.crsht_timing_enable(plan.handle, 1 if on else 0), "crsht_timing_enable")


def timing_read(plan: Plan, kernel: int):
    """(total milliseconds, launches) of a tracked kernel since timing_enable."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.crsht_timing_read(plan.handle, kernel, ctypes.byref(ms), ctypes.byref(n)), "crsht_timing_read")
    return ms.value, n.value


# ---------------------------------------------------------------- tile shapes
def _tuning_dict(t: _Tuning) -> dict:
    n = t.nclasses
    return {"fft_len": list(t.fft_len[:n]), "ring_div": list(t.ring_div[:n]), "f64_synth_cols": t.f64_synth_cols,
            "f64_adj_cols": t.f64_adj_cols, "from_cache": bool(t.from_cache), "ms_default": t.ms_default,
            "ms_tuned": t.ms_tuned}


def autotune(plan: Plan, nrhs: int, prec: int = CR_F64) -> dict:
    """crsht_autotune: measure (or read from CRSHT_TUNE_CACHE) and keep the
    fastest tile shapes of the plan for nrhs columns in precision prec."""
    t = _Tuning()
    _check(_lib.crsht_autotune(plan.handle, nrhs, prec, ctypes.byref(t), _stream()), "crsht_autotune")
    return _tuning_dict(t)


def get_tuning(plan: Plan) -> dict:
    t = _Tuning()
    _check(_lib.crsht_get_tuning(plan.handle, ctypes.byref(t)), "crsht_get_tuning")
    return _tuning_dict(t)


def set_tuning(plan: Plan, ring_div=None, f64_synth_cols: int | None = None, f64_adj_cols: int | None = None):
    """crsht_set_tuning: force shapes (unspecified fields keep their values)."""
    t = _Tuning()
    _check(_lib.crsht_get_tuning(plan.handle, ctypes.byref(t)), "crsht_get_tuning")
    if ring_div is not None:
        for k, v in enumerate(ring_div):
            t.ring_div[k] = int(v)
    if f64_synth_cols is not None:
        t.f64_synth_cols = int(f64_synth_cols)
    if f64_adj_cols is not None:
        t.f64_adj_cols = int(f64_adj_cols)
    _check(_lib.crsht_set_tuning(plan.handle, ctypes.byref(t)), "crsht_set_tuning")


# ---------------------------------------------------------------- transforms
def synth(plan: Plan, alm: torch.Tensor, out: torch.Tensor | None = None, prec: int = CR_F64) -> torch.Tensor:
    n = _nrhs(alm, plan.vlen, torch.complex128)
    if out is None:
        out = torch.empty(tuple(alm.shape[:-1]) + (plan.npix,), dtype=torch.float64, device=alm.device)
    _check(_lib.sht_synth(plan.handle, n, _ptr(alm), _ptr(out), prec, _stream()), "sht_synth")
    return out


def synth_noalloc(plan: Plan, alm: torch.Tensor, out: torch.Tensor, prec: int = CR_F64) -> torch.Tensor:
    """sht_synth_noalloc: sht_synth with the library's static device scratch
    (no allocation by the call); `out` is the caller's map tensor."""
    n = _nrhs(alm, plan.vlen, torch.complex128)
    _check(_lib.sht_synth_noalloc(plan.handle, n, _ptr(alm), _ptr(out), prec, _stream()), "sht_synth_noalloc")
    return out


def adjoint(plan: Plan, m: torch.Tensor, out: torch.Tensor | None = None, prec: int = CR_F64) -> torch.Tensor:
    n = _nrhs(m, plan.mlen, torch.float64)
    if out is None:
        out = torch.empty(tuple(m.shape[:-1]) + (plan.nalm,), dtype=torch.complex128, device=m.device)
    _check(_lib.sht_synth_adjoint(plan.handle, n, _ptr(m), _ptr(out), prec, _stream()), "sht_synth_adjoint")
    return out


def analysis(plan: Plan, m: torch.Tensor, n_iter: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    n = _nrhs(m, plan.mlen, torch.float64)
    if out is None:
        out = torch.empty(tuple(m.shape[:-1]) + (plan.nalm,), dtype=torch.complex128, device=m.device)
    _check(_lib.sht_analysis(plan.handle, n, _ptr(m), _ptr(out), n_iter, _stream()), "sht_analysis")
    return out


# ---------------------------------------------------------------- CR system
@dataclass
class Problem:
    """cl, bl: host float64 arrays of lmax+1; ninv: device float64 [npix].
    Plans with ncomp = 3: cl [4, lmax+1] (TT, EE, BB, TE), ninv [3, npix]
    (T, Q, U), lmin >= 2. amp: optional host float64 array, one amplitude
    per column (column c solves with amp[c] C_l; rhs, apply and solve only)."""
    cl: object
    bl: object
    ninv: torch.Tensor
    lmin: int = 2
    amp: object = None

    def _c(self, q: float = 1.0):
        import numpy as np
        self._cl = np.ascontiguousarray(self.cl, dtype=np.float64)
        self._bl = np.ascontiguousarray(self.bl, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        amp = None
        if self.amp is not None:
            self._amp = np.ascontiguousarray(self.amp, dtype=np.float64)
            amp = self._amp.ctypes.data_as(dp)
        return _Problem(self._cl.ctypes.data_as(dp), self._bl.ctypes.data_as(dp), _ptr(self.ninv), self.lmin, amp)


@dataclass
class Stats:
    status: int
    iters: int
    refinements: int
    rel_resid_true: float


def precond(plan: Plan, prob: Problem) -> torch.Tensor:
    out = torch.empty(plan.alm_shape(1)[1:], dtype=torch.float64, device=prob.ninv.device)
    p = prob._c()
    _check(_lib.cr_precond(plan.handle, ctypes.byref(p), _ptr(out), _stream()), "cr_precond")
    return out


def block_precond_build(plan: Plan, prob: Problem):
    """Build the per-m block preconditioner of prob into the plan (used by
    solves with precond=CR_PC_BLOCK)."""
    p = prob._c()
    _check(_lib.cr_block_precond_build(plan.handle, ctypes.byref(p), _stream()), "cr_block_precond_build")
    torch.cuda.synchronize()


def block_precond_apply(plan: Plan, r: torch.Tensor) -> torch.Tensor:
    """z = M^-1 r with the plan's block preconditioner."""
    n = _nrhs(r, plan.vlen, torch.complex128)
    z = torch.empty_like(r)
    _check(_lib.cr_block_precond_apply(plan.handle, n, _ptr(r), _ptr(z), _stream()), "cr_block_precond_apply")
    return z


def rhs(plan: Plan, prob: Problem, d=None, w0=None, w1=None, nrhs: int = 1) -> torch.Tensor:
    out = torch.empty(plan.alm_shape(nrhs), dtype=torch.complex128, device=prob.ninv.device)
    p = prob._c()
    _check(_lib.cr_rhs(plan.handle, ctypes.byref(p), nrhs, _ptr(d), _ptr(w0), _ptr(w1), _ptr(out), _stream()),
           "cr_rhs")
    return out


def apply(plan: Plan, prob: Problem, x: torch.Tensor, prec: int = CR_F64) -> torch.Tensor:
    n = _nrhs(x, plan.vlen, torch.complex128)
    out = torch.empty_like(x)
    p = prob._c()
    _check(_lib.cr_apply(plan.handle, ctypes.byref(p), n, _ptr(x), _ptr(out), prec, _stream()), "cr_apply")
    return out


def solve(plan: Plan, prob: Problem, d=None, w0=None, w1=None, rhs_vec=None, nrhs: int = 1, tol: float = 1e-6,
          maxiter: int = 10000, prec: int = CR_F64, inner_tol: float = 1e-2, max_refine: int = 50,
          check_every: int = 8, out: torch.Tensor | None = None, use_graph: bool = True,
          precond: int = CR_PC_JACOBI, terms: int = CR_SUM):
    """Returns (s [nrhs, nalm] complex128 ([nrhs, 3, nalm] for ncomp = 3), [Stats]).
    use_graph: replay each block of check_every iterations as a captured HIP graph.
    terms = CR_SEPARATE: s [nrhs, 2, ...] (mean field, fluctuation) and 2 nrhs Stats."""
    nsol = 2 * nrhs if terms == CR_SEPARATE else nrhs
    if out is None:
        shape = plan.alm_shape(nrhs)
        if terms == CR_SEPARATE:
            shape = (nrhs, 2) + tuple(shape[1:])
        out = torch.empty(shape, dtype=torch.complex128, device=prob.ninv.device)
    p = prob._c()
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, check_every, int(precond), int(use_graph), int(terms))
    st = (_Stats * nsol)()
    _check(_lib.cr_solve(plan.handle, ctypes.byref(p), nrhs, _ptr(d), _ptr(w0), _ptr(w1), _ptr(rhs_vec), _ptr(out),
                         ctypes.byref(o), st, _stream()), "cr_solve")
    return out, [Stats(s.status, s.iters, s.refinements, s.rel_resid_true) for s in st]


def solve_async(plan: Plan, prob: Problem, d=None, w0=None, w1=None, rhs_vec=None, nrhs: int = 1,
                tol: float = 1e-6, maxiter: int = 60, prec: int = CR_F64, inner_tol: float = 1e-2,
                max_refine: int = 50, check_every: int = 6, out: torch.Tensor | None = None,
                stats: torch.Tensor | None = None, use_graph: bool = True, precond: int = CR_PC_JACOBI):
    """cr_solve_async: the whole solve enqueued on the current stream, nothing
    waits. Returns (s, stats_dev) with stats_dev a device tensor of nrhs
    cr_stats (24 bytes each, as uint8); read it with decode_stats after a
    synchronisation."""
    if out is None:
        out = torch.empty(plan.alm_shape(nrhs), dtype=torch.complex128, device=prob.ninv.device)
    if stats is None:
        stats = torch.empty(nrhs * ctypes.sizeof(_Stats), dtype=torch.uint8, device=prob.ninv.device)
    if stats.numel() < nrhs * ctypes.sizeof(_Stats):
        raise ValueError("stats needs %d bytes" % (nrhs * ctypes.sizeof(_Stats)))
    p = prob._c()
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, check_every, int(precond), int(use_graph))
    _check(_lib.cr_solve_async(plan.handle, ctypes.byref(p), nrhs, _ptr(d), _ptr(w0), _ptr(w1), _ptr(rhs_vec),
                               _ptr(out), ctypes.byref(o), _ptr(stats), _stream()), "cr_solve_async")
    return out, stats


def decode_stats(stats: torch.Tensor, nrhs: int) -> list:
    """Host copies of the cr_stats an asynchronous solve wrote to the device."""
    raw = bytes(stats[:nrhs * ctypes.sizeof(_Stats)].cpu().numpy().tobytes())
    arr = (_Stats * nrhs).from_buffer_copy(raw)
    return [Stats(x.status, x.iters, x.refinements, x.rel_resid_true) for x in arr]


def solve_batched(plans, probs, d=None, w0=None, w1=None, tol: float = 1e-6, maxiter: int = 20000,
                  prec: int = CR_F64, inner_tol: float = 1e-2, max_refine: int = 0, check_every: int = 16,
                  out=None, use_graph: bool = True, precond: int = CR_PC_JACOBI):
    """Independent single-column problems (own plan each). d, w0, w1: lists of
    tensors (or None). Returns (list of s [nalm] complex128, [Stats])."""
    n = len(plans)
    if len(probs) != n:
        raise ValueError("one problem per plan")
    if out is None:
        out = [torch.empty(pl.alm_shape(1)[1:], dtype=torch.complex128, device=pr.ninv.device)
               for pl, pr in zip(plans, probs)]
    VP = ctypes.c_void_p * n

    def arr(ts):
        if ts is None:
            return None
        return VP(*[(_ptr(t).value if t is not None else None) for t in ts])

    hp = VP(*[pl.handle.value for pl in plans])
    pa = (_Problem * n)(*[pr._c() for pr in probs])
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, check_every, int(precond), int(use_graph))
    st = (_Stats * n)()
    _check(_lib.cr_solve_batched(hp, pa, n, arr(d), arr(w0), arr(w1), VP(*[_ptr(t).value for t in out]),
                                 ctypes.byref(o), st, _stream()), "cr_solve_batched")
    return out, [Stats(x.status, x.iters, x.refinements, x.rel_resid_true) for x in st]


def lnpi(plan: Plan, fid: Problem, q: float, d: torch.Tensor, ahat: torch.Tensor, fhat: torch.Tensor) -> float:
    p = fid._c()
    v = ctypes.c_double()
    _check(_lib.cr_lnpi(plan.handle, ctypes.byref(p), q, _ptr(d), _ptr(ahat), _ptr(fhat), ctypes.byref(v),
                        _stream()), "cr_lnpi")
    return v.value


@dataclass
class Chain:
    q: float
    lnpi: float
    ahat: torch.Tensor
    fhat: torch.Tensor


@dataclass
class StepResult:
    accepted: bool
    lnA: float
    q_new: float
    lnpi_new: float
    mean_stats: Stats
    fluct_stats: Stats


def joint_step(plan: Plan, fid: Problem, d: torch.Tensor, chain: Chain, xi: float, u: float, w0: torch.Tensor,
               w1: torch.Tensor, sigma_lnq: float = 0.02, tol: float = 1e-6, maxiter: int = 10000,
               prec: int = CR_F64, inner_tol: float = 1e-2, max_refine: int = 50,
               use_graph: bool = True, precond: int = CR_PC_JACOBI) -> StepResult:
    p = fid._c()
    c = _Chain(chain.q, chain.lnpi, _ptr(chain.ahat), _ptr(chain.fhat))
    dr = _Draws(xi, u, _ptr(w0), _ptr(w1), sigma_lnq)
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, 8, int(precond), int(use_graph))
    r = _StepOut()
    _check(_lib.joint_cl_step(plan.handle, ctypes.byref(p), _ptr(d), ctypes.byref(c), ctypes.byref(dr),
                              ctypes.byref(o), ctypes.byref(r), _stream()), "joint_cl_step")
    chain.q, chain.lnpi = c.q, c.lnpi

    def st(s):
        return Stats(s.status, s.iters, s.refinements, s.rel_resid_true)

    return StepResult(bool(r.accepted), r.lnA, r.q_new, r.lnpi_new, st(r.mean_stats), st(r.fluct_stats))


def white(plan: Plan, nrhs: int, seed: int, counter: int, alm: bool = True, pix: bool = True,
          device: torch.device | None = None):
    """(w0 [nrhs, (3,) nalm] complex, w1 [nrhs, (3,) npix]) unit white draws on
    the device (cr_white); either is None when not asked for."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    w0 = torch.empty(plan.alm_shape(nrhs), dtype=torch.complex128, device=dev) if alm else None
    shape = (nrhs, 3, plan.npix) if plan.ncomp == 3 else (nrhs, plan.npix)
    w1 = torch.empty(shape, dtype=torch.float64, device=dev) if pix else None
    _check(_lib.cr_white(plan.handle, nrhs, seed & (2 ** 64 - 1), counter & (2 ** 64 - 1), _ptr(w0), _ptr(w1),
                         _stream()), "cr_white")
    return w0, w1


def joint_step_batch(plan: Plan, fid: Problem, d: torch.Tensor, chains: list, xi, u, w0: torch.Tensor,
                     w1: torch.Tensor, sigma_lnq: float = 0.02, tol: float = 1e-6, maxiter: int = 10000,
                     prec: int = CR_F64, inner_tol: float = 1e-2, max_refine: int = 50, use_graph: bool = True,
                     precond: int = CR_PC_JACOBI) -> list:
    """Joint moves of several chains at once (joint_cl_step_batch); w0
    [n, nalm] and w1 [n, npix] on the device; every chain updated in place."""
    n = len(chains)
    p = fid._c()
    arr = (_Chain * n)(*[_Chain(c.q, c.lnpi, _ptr(c.ahat), _ptr(c.fhat)) for c in chains])
    x, uu = _f64(xi), _f64(u)
    if x.size != n or uu.size != n:
        raise ValueError("xi and u need one entry per chain")
    dp = ctypes.POINTER(ctypes.c_double)
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, 8, int(precond), int(use_graph))
    outs = (_StepOut * n)()
    _check(_lib.joint_cl_step_batch(plan.handle, ctypes.byref(p), _ptr(d), n, arr, x.ctypes.data_as(dp),
                                    uu.ctypes.data_as(dp), sigma_lnq, _ptr(w0), _ptr(w1), ctypes.byref(o), outs,
                                    _stream()), "joint_cl_step_batch")

    def st(s_):
        return Stats(s_.status, s_.iters, s_.refinements, s_.rel_resid_true)

    res = []
    for c, ch in enumerate(chains):
        ch.q, ch.lnpi = arr[c].q, arr[c].lnpi
        r = outs[c]
        res.append(StepResult(bool(r.accepted), r.lnA, r.q_new, r.lnpi_new, st(r.mean_stats), st(r.fluct_stats)))
    return res


@dataclass
class GibbsResult:
    q_new: float
    t: float
    mean_stats: Stats
    fluct_stats: Stats


def gibbs_shape(lmax: int, lmin: int = 2) -> float:
    """Shape alpha = k/2 - 1 of the inverse-gamma amplitude conditional,
    k = sum_{l=lmin}^{lmax} (2l + 1) real degrees of freedom."""
    k = sum(2 * l + 1 for l in range(lmin, lmax + 1))
    return 0.5 * k - 1.0


def gibbs_step(plan: Plan, fid: Problem, d: torch.Tensor, chain: Chain, g: float, w0: torch.Tensor,
               w1: torch.Tensor, tol: float = 1e-6, maxiter: int = 10000, prec: int = CR_F64,
               inner_tol: float = 1e-2, max_refine: int = 50, use_graph: bool = True,
               precond: int = CR_PC_JACOBI) -> GibbsResult:
    """Standard Gibbs amplitude move (gibbs_cl_step); g ~ Gamma(gibbs_shape(lmax, lmin), 1)."""
    p = fid._c()
    c = _Chain(chain.q, chain.lnpi, _ptr(chain.ahat), _ptr(chain.fhat))
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, 8, int(precond), int(use_graph))
    r = _GibbsOut()
    _check(_lib.gibbs_cl_step(plan.handle, ctypes.byref(p), _ptr(d), ctypes.byref(c), float(g), _ptr(w0), _ptr(w1),
                              ctypes.byref(o), ctypes.byref(r), _stream()), "gibbs_cl_step")
    chain.q, chain.lnpi = c.q, c.lnpi

    def st(s):
        return Stats(s.status, s.iters, s.refinements, s.rel_resid_true)

    return GibbsResult(r.q_new, r.t, st(r.mean_stats), st(r.fluct_stats))


def gibbs_step_batch(plan: Plan, fid: Problem, d: torch.Tensor, chains: list, g, w0: torch.Tensor,
                     w1: torch.Tensor, tol: float = 1e-6, maxiter: int = 10000, prec: int = CR_F64,
                     inner_tol: float = 1e-2, max_refine: int = 50, use_graph: bool = True,
                     precond: int = CR_PC_JACOBI) -> list:
    """Gibbs moves of several chains at once (gibbs_cl_step_batch); w0 [n,
    nalm] and w1 [n, npix] on the device; every chain updated in place."""
    n = len(chains)
    p = fid._c()
    arr = (_Chain * n)(*[_Chain(c.q, c.lnpi, _ptr(c.ahat), _ptr(c.fhat)) for c in chains])
    gg = _f64(g)
    if gg.size != n:
        raise ValueError("g needs one entry per chain")
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, 8, int(precond), int(use_graph))
    outs = (_GibbsOut * n)()
    _check(_lib.gibbs_cl_step_batch(plan.handle, ctypes.byref(p), _ptr(d), n, arr,
                                    gg.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(w0), _ptr(w1),
                                    ctypes.byref(o), outs, _stream()), "gibbs_cl_step_batch")

    def st(s_):
        return Stats(s_.status, s_.iters, s_.refinements, s_.rel_resid_true)

    res = []
    for c, ch in enumerate(chains):
        ch.q, ch.lnpi = arr[c].q, arr[c].lnpi
        r = outs[c]
        res.append(GibbsResult(r.q_new, r.t, st(r.mean_stats), st(r.fluct_stats)))
    return res


@dataclass
class BinChain:
    """Chain over per-bin log-amplitudes theta (C_l = C_l^fid exp(theta_k) on
    [edges[k], edges[k+1]))."""
    edges: object            # host int array, nbins + 1
    theta: object            # host float64 array, nbins (updated in place)
    lnpi: float
    ahat: torch.Tensor
    fhat: torch.Tensor


@dataclass
class HmcResult:
    accepted: bool
    status: int
    dH: float
    lnpi_new: float
    solves: int
    iters: int
    fluct_stats: Stats


def _i32(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.float64)


def lnpi_grad_fixed(plan: Plan, fid: Problem, d: torch.Tensor, edges, theta0, theta, f0: torch.Tensor,
                    a0: torch.Tensor | None = None, tol: float = 1e-10, maxiter: int = 20000, prec: int = CR_F64,
                    inner_tol: float = 1e-2, max_refine: int = 50, check_every: int = 8, use_graph: bool = True,
                    precond: int = CR_PC_JACOBI):
    """(d ln pi / d theta [nbins] numpy, ln pi, mean field [nalm], Stats) at a
    fixed whitened fluctuation (cr_lnpi_grad_fixed)."""
    import numpy as np
    e, t0, t1 = _i32(edges), _f64(theta0), _f64(theta)
    nb = e.size - 1
    g = np.zeros(nb)
    v = ctypes.c_double()
    st = (_Stats * 1)()
    ahat = torch.empty(plan.alm_shape(1)[1:], dtype=torch.complex128, device=d.device)
    p = fid._c()
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, check_every, int(precond), int(use_graph))
    dp = ctypes.POINTER(ctypes.c_double)
    _check(_lib.cr_lnpi_grad_fixed(plan.handle, ctypes.byref(p), _ptr(d), nb,
                                   e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), t0.ctypes.data_as(dp),
                                   t1.ctypes.data_as(dp), _ptr(f0), _ptr(a0), ctypes.byref(o), ctypes.byref(v),
                                   g.ctypes.data_as(dp), _ptr(ahat), st, _stream()), "cr_lnpi_grad_fixed")
    return g, v.value, ahat, Stats(st[0].status, st[0].iters, st[0].refinements, st[0].rel_resid_true)


def gibbs_bins_step(plan: Plan, fid: Problem, d: torch.Tensor, chain: BinChain, g, w0: torch.Tensor,
                    w1: torch.Tensor, tol: float = 1e-6, maxiter: int = 10000, prec: int = CR_F64,
                    inner_tol: float = 1e-2, max_refine: int = 50, use_graph: bool = True,
                    precond: int = CR_PC_JACOBI):
    """Standard Gibbs move of per-bin amplitudes (gibbs_bins_step): returns
    (t [nbins] numpy, mean-field Stats, fluctuation Stats); chain.theta and
    chain.lnpi updated in place."""
    import numpy as np
    e = _i32(chain.edges)
    th = _f64(chain.theta)
    gg = _f64(g)
    nb = e.size - 1
    if gg.size != nb:
        raise ValueError("g needs one entry per bin")
    dp = ctypes.POINTER(ctypes.c_double)
    c = _BinChain(nb, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), th.ctypes.data_as(dp), chain.lnpi,
                  _ptr(chain.ahat), _ptr(chain.fhat))
    t = np.zeros(nb)
    sts = (_Stats * 2)()
    p = fid._c()
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, 8, int(precond), int(use_graph))
    _check(_lib.gibbs_bins_step(plan.handle, ctypes.byref(p), _ptr(d), ctypes.byref(c), gg.ctypes.data_as(dp),
                                _ptr(w0), _ptr(w1), ctypes.byref(o), t.ctypes.data_as(dp), sts, _stream()),
           "gibbs_bins_step")
    chain.theta = th.copy()
    chain.lnpi = c.lnpi
    mk = [Stats(x.status, x.iters, x.refinements, x.rel_resid_true) for x in sts]
    return t, mk[0], mk[1]


def hmc_step(plan: Plan, fid: Problem, d: torch.Tensor, chain: BinChain, p0, u: float, w0: torch.Tensor,
             w1: torch.Tensor, eps: float, nleap: int, tol: float = 1e-6, maxiter: int = 10000,
             prec: int = CR_F64, inner_tol: float = 1e-2, max_refine: int = 50, use_graph: bool = True,
             precond: int = CR_PC_JACOBI) -> HmcResult:
    """One HMC move of the bin log-amplitudes (hmc_cl_step); chain.theta and
    chain.lnpi are updated in place."""
    e = _i32(chain.edges)
    th = _f64(chain.theta)
    pp = _f64(p0)
    dp = ctypes.POINTER(ctypes.c_double)
    c = _BinChain(e.size - 1, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), th.ctypes.data_as(dp), chain.lnpi,
                  _ptr(chain.ahat), _ptr(chain.fhat))
    dr = _HmcDraws(pp.ctypes.data_as(dp), u, _ptr(w0), _ptr(w1), eps, int(nleap))
    p = fid._c()
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, 8, int(precond), int(use_graph))
    r = _HmcOut()
    _check(_lib.hmc_cl_step(plan.handle, ctypes.byref(p), _ptr(d), ctypes.byref(c), ctypes.byref(dr),
                            ctypes.byref(o), ctypes.byref(r), _stream()), "hmc_cl_step")
    chain.theta = th.copy()
    chain.lnpi = c.lnpi
    fs = r.fluct_stats
    return HmcResult(bool(r.accepted), r.status, r.dH, r.lnpi_new, r.solves, r.iters,
                     Stats(fs.status, fs.iters, fs.refinements, fs.rel_resid_true))


# ---------------------------------------------------------------- gradients
def synth_grad(plan: Plan, map_grad: torch.Tensor, out: torch.Tensor | None = None, prec: int = CR_F64):
    """w_m Y^T map_grad (torch.autograd convention for the complex m >= 0 leaf)."""
    n = _nrhs(map_grad, plan.mlen, torch.float64)
    if out is None:
        out = torch.empty(tuple(map_grad.shape[:-1]) + (plan.nalm,), dtype=torch.complex128, device=map_grad.device)
    _check(_lib.sht_synth_grad(plan.handle, n, _ptr(map_grad), _ptr(out), prec, _stream()), "sht_synth_grad")
    return out


class SynthFunction(torch.autograd.Function):
    """map = Y alm with the synthesis kernel forward and sht_synth_grad backward."""

    @staticmethod
    def forward(ctx, alm, plan, prec):
        ctx.plan, ctx.prec = plan, prec
        return synth(plan, alm.contiguous(), prec=prec)

    @staticmethod
    def backward(ctx, g):
        return synth_grad(ctx.plan, g.contiguous(), prec=ctx.prec), None, None


def synth_ad(plan: Plan, alm: torch.Tensor, prec: int = CR_F64) -> torch.Tensor:
    """Differentiable synthesis (torch.autograd)."""
    return SynthFunction.apply(alm, plan, prec)


def grad_chi2(plan: Plan, prob: Problem, d: torch.Tensor, a: torch.Tensor):
    """(g, chi2) with chi2 = (d - Y B a)^T N^-1 (d - Y B a) per column and g
    its gradient in the real-field inner product."""
    n = _nrhs(a, plan.vlen, torch.complex128)
    g = torch.empty_like(a)
    c = (ctypes.c_double * n)()
    p = prob._c()
    _check(_lib.cr_grad_chi2(plan.handle, ctypes.byref(p), n, _ptr(d), _ptr(a), _ptr(g), c, _stream()),
           "cr_grad_chi2")
    return g, [c[k] for k in range(n)]


def grad_lnpi(plan: Plan, prob: Problem, d: torch.Tensor, w0, w1, edges, tol: float = 1e-10, maxiter: int = 20000,
              prec: int = CR_F64, inner_tol: float = 1e-2, max_refine: int = 0, check_every: int = 8,
              use_graph: bool = True, precond: int = CR_PC_JACOBI):
    """(dlnpi/dtheta [nbins] numpy, ln pi, [Stats x 3]) for per-bin log-amplitudes
    of C_l on [edges[k], edges[k+1])."""
    import numpy as np
    e = np.ascontiguousarray(edges, dtype=np.int32)
    nb = e.size - 1
    g = np.zeros(nb)
    v = ctypes.c_double()
    st = (_Stats * 3)()
    p = prob._c()
    o = _Opts(tol, maxiter, prec, inner_tol, max_refine, check_every, int(precond), int(use_graph))
    _check(_lib.cr_grad_lnpi(plan.handle, ctypes.byref(p), _ptr(d), _ptr(w0), _ptr(w1), nb,
                             e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(o),
                             g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(v), st, _stream()),
           "cr_grad_lnpi")
    return g, v.value, [Stats(x.status, x.iters, x.refinements, x.rel_resid_true) for x in st]


def nalm(lmax: int, mmax: int | None = None) -> int:
    mmax = lmax if mmax is None else mmax
    return (mmax + 1) * (lmax + 1) - (mmax * (mmax + 1)) // 2


__all__ = ["Plan", "Problem", "Stats", "Chain", "StepResult", "synth", "adjoint", "analysis", "precond", "rhs",
           "block_precond_build", "block_precond_apply", "CR_PC_JACOBI", "CR_PC_BLOCK",
           "apply", "solve", "solve_batched", "lnpi", "white", "joint_step", "joint_step_batch", "gibbs_step", "gibbs_step_batch", "gibbs_shape", "GibbsResult",
           "BinChain", "HmcResult", "lnpi_grad_fixed", "hmc_step", "gibbs_bins_step", "synth_grad", "synth_ad", "SynthFunction", "grad_chi2", "grad_lnpi",
           "CR_F64", "CR_MIXED", "CrshtError", "strerror", "EXPORTED"]
_ = math
