"""Shared helpers of the GPU parity tests (inputs from crinputs, expected
values from the oracle; the HIP path only through the C-ABI binding)."""
import math

import numpy as np
import torch

import crinputs as ci
from oracle import cr, healpix, sht


def dev():
    return torch.device("cuda:0")


def tc(a):
    """numpy -> contiguous CUDA tensor (complex128 or float64)."""
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a).to(dev())


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def real_rel(op, a, b):
    """relative error in the real-field norm."""
    d = a - b
    nb = math.sqrt(max(op.dot(b, b), 1e-300))
    return math.sqrt(max(op.dot(d, d), 0.0)) / nb


def masked_problem(nside, lmax=None, cfg=1, fwhm_arcmin=30.0):
    wl = ci.workload_masked_t(nside, lmax, fwhm_arcmin=fwhm_arcmin, cfg=cfg)
    z, phi = healpix.pixel_coords(nside)
    ninv = wl.ninv(z, phi)
    P = cr.Problem(nside, wl.lmax, wl.cl(), wl.bl(), ninv)
    op = cr.CROperator(P)
    d = op.sht.synth(op.b * wl.signal()) + wl.noise(z, phi)
    return wl, P, op, d
