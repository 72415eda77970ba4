"""O2: the exact discrete Fourier pair L, L*, FBP (oracle, test only).

This is the definition the Fourier route approximates, written out as
non-uniform DFT sums.  It follows eq:fftfwd / eq:fftadj with the 3D
transform evaluated exactly (no USFFT), and eq:fftfwdsplit for the order
of summation (x3 first, then (x1, x2)), which changes nothing but speed.

Definitions (discrete conventions in `geometry`):

  A f(theta, l, m) = sum_x f(x) exp(-2 pi i x . xi(theta, m/w_p, l/h_p))
  L f(theta, v, u) = Re (1/(h_p w_p)) sum_{l, m} A f(theta, l, m)
                         exp(+2 pi i (m u / w_p + l v / h_p))
  G(theta, l, m)   = (1/(h_p w_p)) sum_{u, v} d(theta, v, u)
                         exp(-2 pi i (m u / w_p + l v / h_p))
  L* d(x)          = Re sum_{theta, l, m} G(theta, l, m) exp(+2 pi i x . xi)
  FBP d(x)         = Re sum_{theta, l, m} W(m) G(theta, l, m) exp(+2 pi i x . xi)

with l, m over the full symmetric ranges (Nyquist bins dropped) and W
from `filters.fbp_weight`.  No Hermitian halving is used here: every
frequency is summed explicitly and the real part taken at the end.
"""
import numpy as np

from . import filters
from .geometry import centred, freqs


def _phases(geom, l, sign):
    """exp(sign 2 pi i x1 xi1), exp(sign 2 pi i x2 xi2) for slab l.

    Returns P1, P2 of shape (n_theta * M, n): row s = (theta, m)."""
    ms = freqs(geom.w_p)
    ct = np.cos(geom.theta)[:, None]
    st = np.sin(geom.theta)[:, None]
    ku = (ms / geom.w_p)[None, :]
    kv = l / geom.h_p
    xi1 = (ku * ct + kv * st * np.sin(geom.phi)).reshape(-1)
    xi2 = (ku * st - kv * ct * np.sin(geom.phi)).reshape(-1)
    x = centred(geom.n)
    P1 = np.exp(sign * 2j * np.pi * xi1[:, None] * x[None, :])
    P2 = np.exp(sign * 2j * np.pi * xi2[:, None] * x[None, :])
    return P1, P2


def x3_phases(geom, sign):
    """E[z, l] = exp(sign 2 pi i x3 xi3), xi3 = l cos(phi) / h_p (eq:uneqspace)."""
    ls = freqs(geom.h_p)
    x3 = centred(geom.nz)
    return np.exp(sign * 2j * np.pi * np.outer(x3, ls) * np.cos(geom.phi) / geom.h_p)


def forward_spectra(f, geom):
    """A f(theta, l, m) over the full (l, m) ranges; shape (T, L, M)."""
    f = np.asarray(f, dtype=np.float64)
    assert f.shape == (geom.nz, geom.n, geom.n)
    ls = freqs(geom.h_p)
    ms = freqs(geom.w_p)
    E = x3_phases(geom, -1.0)
    # inner integral of eq:fftfwdsplit: sum over x3 for every (l, x2, x1)
    # (contiguous per slab, so that the products below run through BLAS)
    ghat = np.ascontiguousarray(np.einsum("zl,zyx->lyx", E, f, optimize=True))
    A = np.empty((geom.n_theta, len(ls), len(ms)), dtype=np.complex128)
    for li, l in enumerate(ls):
        P1, P2 = _phases(geom, l, -1.0)
        # sum_{x2, x1} P2[s, x2] ghat[x2, x1] P1[s, x1]
        A[:, li, :] = np.sum((P2 @ ghat[li]) * P1, axis=1).reshape(geom.n_theta, len(ms))
    return A


def spectra_to_detector(A, geom, rows=None, cols=None, imag=False):
    """(1/(h_p w_p)) sum_{l,m} A exp(2 pi i (m u/w_p + l v/h_p)) on the detector.

    rows/cols default to the h x w detector; pass centred coordinates to
    evaluate elsewhere (e.g. the whole padded period)."""
    ls = freqs(geom.h_p)
    ms = freqs(geom.w_p)
    u = centred(geom.w) if cols is None else np.asarray(cols)
    v = centred(geom.h) if rows is None else np.asarray(rows)
    Eu = np.exp(2j * np.pi * np.outer(ms, u) / geom.w_p)
    Ev = np.exp(2j * np.pi * np.outer(v, ls) / geom.h_p)
    d = np.einsum("vl,tlm,mu->tvu", Ev, A, Eu, optimize=True) / (geom.h_p * geom.w_p)
    return (d.real, d.imag) if imag else d.real


def forward(f, geom, rows=None, cols=None, imag=False):
    """L f (eq:fftfwd evaluated exactly)."""
    return spectra_to_detector(forward_spectra(f, geom), geom, rows, cols, imag)


def data_spectra(d, geom):
    """G(theta, l, m) = (1/(h_p w_p)) sum_{u,v} d exp(-2 pi i (m u/w_p + l v/h_p))."""
    d = np.asarray(d, dtype=np.float64)
    assert d.shape == (geom.n_theta, geom.h, geom.w)
    ls = freqs(geom.h_p)
    ms = freqs(geom.w_p)
    Fu = np.exp(-2j * np.pi * np.outer(centred(geom.w), ms) / geom.w_p)
    Fv = np.exp(-2j * np.pi * np.outer(ls, centred(geom.h)) / geom.h_p)
    return np.einsum("lv,tvu,um->tlm", Fv, d, Fu, optimize=True) / (geom.h_p * geom.w_p)


def data_spectra_fft(d, geom, half=False):
    """The same G computed with numpy's FFT of the zero-padded data.

    half=True keeps l >= 0 only (for large inputs); rows are then
    l = 0 .. h_p/2 - 1."""
    d = np.asarray(d, dtype=np.float64)
    T = geom.n_theta
    ms = freqs(geom.w_p)
    ls = np.arange(geom.h_p // 2) if half else freqs(geom.h_p)
    out = np.empty((T, len(ls), len(ms)), dtype=np.complex128)
    rows = centred(geom.h) % geom.h_p
    cols = centred(geom.w) % geom.w_p
    for t0 in range(0, T, 16):
        t1 = min(T, t0 + 16)
        pad = np.zeros((t1 - t0, geom.h_p, geom.w_p))
        pad[:, rows[:, None], cols[None, :]] = d[t0:t1]
        F = np.fft.fft2(pad) / (geom.h_p * geom.w_p)
        out[t0:t1] = F[:, (ls % geom.h_p)[:, None], (ms % geom.w_p)[None, :]]
    return out


def filter_spectra(G, geom, kind):
    """Multiply by the FBP weight W(m) of eq:recon (see `filters`)."""
    W = filters.fbp_weight(freqs(geom.w_p), geom.w_p, geom.n_theta, geom.phi, kind)
    return G * W[None, None, :]


def backproject_spectra(G, geom, imag=False):
    """Re sum_{theta,l,m} G exp(+2 pi i x . xi) on the whole volume."""
    ls = freqs(geom.h_p)
    n = geom.n
    g = np.empty((len(ls), n, n), dtype=np.complex128)
    for li, l in enumerate(ls):
        P1, P2 = _phases(geom, l, +1.0)
        Gl = G[:, li, :].reshape(-1)
        # g_l[x2, x1] = sum_s G[s] P2[s, x2] P1[s, x1]
        g[li] = (P2 * Gl[:, None]).T @ P1
    E = x3_phases(geom, +1.0)
    vol = np.einsum("zl,lyx->zyx", E, g, optimize=True)
    return (vol.real, vol.imag) if imag else vol.real


def backproject_columns(G, geom, ys, xs):
    """The same sum for selected columns (y, x) only: returns (nz, len(ys))."""
    ls = freqs(geom.h_p)
    ms = freqs(geom.w_p)
    ys = np.asarray(ys)
    xs = np.asarray(xs)
    x1 = xs - geom.n // 2
    x2 = ys - geom.n // 2
    ct = np.cos(geom.theta)[:, None]
    st = np.sin(geom.theta)[:, None]
    ku = (ms / geom.w_p)[None, :]
    g = np.empty((len(ls), len(xs)), dtype=np.complex128)
    for li, l in enumerate(ls):
        kv = l / geom.h_p
        xi1 = (ku * ct + kv * st * np.sin(geom.phi)).reshape(-1)
        xi2 = (ku * st - kv * ct * np.sin(geom.phi)).reshape(-1)
        ph = np.exp(2j * np.pi * (np.outer(xi1, x1) + np.outer(xi2, x2)))
        g[li] = G[:, li, :].reshape(-1) @ ph
    E = x3_phases(geom, +1.0)
    return (E @ g).real


def adjoint(d, geom, imag=False):
    """L* d (eq:fftadj evaluated exactly)."""
    return backproject_spectra(data_spectra(d, geom), geom, imag)


def fbp(d, geom, kind=filters.SHEPP_LOGAN):
    """FBP d = L* applied to W-filtered data (eq:recon)."""
    return backproject_spectra(filter_spectra(data_spectra(d, geom), geom, kind), geom)


def forward_bruteforce(f, geom):
    """L f straight from the definition: one loop over every term.

    For tiny grids only; used to pin the vectorised split above."""
    ls = freqs(geom.h_p)
    ms = freqs(geom.w_p)
    xs = centred(geom.n)
    zs = centred(geom.nz)
    us = centred(geom.w)
    vs = centred(geom.h)
    sp, cp = np.sin(geom.phi), np.cos(geom.phi)
    out = np.zeros((geom.n_theta, geom.h, geom.w))
    for t, th in enumerate(geom.theta):
        ct, st = np.cos(th), np.sin(th)
        for l in ls:
            for m in ms:
                ku, kv = m / geom.w_p, l / geom.h_p
                x1f = ku * ct + kv * st * sp
                x2f = ku * st - kv * ct * sp
                x3f = kv * cp
                acc = 0.0j
                for iz, z in enumerate(zs):
                    for iy, y in enumerate(xs):
                        for ix, x in enumerate(xs):
                            if f[iz, iy, ix] != 0.0:
                                acc += f[iz, iy, ix] * np.exp(
                                    -2j * np.pi * (x * x1f + y * x2f + z * x3f)
                                )
                for iv, v in enumerate(vs):
                    for iu, u in enumerate(us):
                        out[t, iv, iu] += (
                            acc * np.exp(2j * np.pi * (m * u / geom.w_p + l * v / geom.h_p))
                        ).real
    return out / (geom.h_p * geom.w_p)
