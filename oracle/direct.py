"""O1: Python side of the direct line-integral pair (oracle, test only).

Wraps `direct.c` (built to `_direct.so` by `build_direct()`).  FBP_dir
filters each detector row with the transfer function W(m) of `filters`
(rows zero-padded to w_p, filtered through a DFT, cropped back to w) and
then applies L*_dir: the direct discretisation of eq:recon.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import filters
from .geometry import centred, freqs

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_direct.so")
_lib = None


def build_direct():
    """Compile direct.c with gcc/OpenMP into oracle/_direct.so."""
    src = os.path.join(_HERE, "direct.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    )
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_direct()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        for name in ("lam_direct_fwd", "lam_direct_adj"):
            fn = getattr(lib, name)
            fn.argtypes = [dp, i, i, dp, i, ctypes.c_double, i, i, dp]
            fn.restype = None
        lib.lam_direct_adj_slices.argtypes = [dp, i, i, dp, i, ctypes.c_double, i, i, i, i, dp]
        lib.lam_direct_adj_slices.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def forward(f, geom):
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    th = np.ascontiguousarray(geom.theta, dtype=np.float64)
    d = np.empty((geom.n_theta, geom.h, geom.w))
    lib.lam_direct_fwd(_ptr(f), geom.nz, geom.n, _ptr(th), geom.n_theta, geom.phi,
                       geom.h, geom.w, _ptr(d))
    return d


def adjoint(d, geom, z_range=None):
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64)
    th = np.ascontiguousarray(geom.theta, dtype=np.float64)
    if z_range is None:
        f = np.empty((geom.nz, geom.n, geom.n))
        lib.lam_direct_adj(_ptr(d), geom.nz, geom.n, _ptr(th), geom.n_theta, geom.phi,
                           geom.h, geom.w, _ptr(f))
        return f
    z0, z1 = z_range
    f = np.empty((z1 - z0, geom.n, geom.n))
    lib.lam_direct_adj_slices(_ptr(d), geom.nz, geom.n, _ptr(th), geom.n_theta, geom.phi,
                              geom.h, geom.w, z0, z1, _ptr(f))
    return f


def filter_rows(d, geom, kind):
    """Rows filtered by W(m): zero-pad to w_p, DFT, multiply, inverse, crop."""
    d = np.asarray(d, dtype=np.float64)
    w, w_p = geom.w, geom.w_p
    pos = centred(w) % w_p  # padded index of each detector column
    buf = np.zeros(d.shape[:-1] + (w_p,))
    buf[..., pos] = d
    spec = np.fft.fft(buf, axis=-1)
    W = np.zeros(w_p)
    ms = freqs(w_p)
    W[ms % w_p] = filters.fbp_weight(ms, w_p, geom.n_theta, geom.phi, kind)
    out = np.fft.ifft(spec * W, axis=-1).real
    return out[..., pos]


def fbp(d, geom, kind=filters.SHEPP_LOGAN, z_range=None):
    return adjoint(filter_rows(d, geom, kind), geom, z_range)
