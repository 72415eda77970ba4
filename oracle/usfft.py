"""O3: the operators evaluated with a Gaussian USFFT (oracle, test only).

The paper evaluates the 3D transform onto the unequally spaced grid
of eq:uneqspace with an unequally spaced FFT built on a Gaussian psi
(Section "Laminography reconstruction", the three-step list after
eq:fftadj): (1) divide by psi in space, (2) FFT, (3) a convolution in
frequency that moves values to the unequally spaced points; the adjoint
runs the steps in reverse with the inverse FFT.  With the split of
eq:fftfwdsplit the x3 part is done first as an exact sum (xi3 depends
on the slab index l only) and the USFFT is two-dimensional, per slab.

Discrete form used here (per slab, grid of N_g x N_g cells, N_g >= 2 n):

  sample position in cells  X = N_g xi1, Y = N_g xi2 (not wrapped)
  frequency kernel          phi(t) = exp(-beta t^2), t in cells, taps
                            k = floor(X) - M + 1 ... floor(X) + M, used
                            periodically (index k mod N_g)
  beta                      pi (R - 1/2) / (R M), R = N_g / n
                            (the Gaussian width of Greengard & Lee 2004,
                            expressed in grid cells)
  psi correction per axis   sqrt(beta / pi) exp(pi^2 x^2 / (beta N_g^2))

  forward:  F = FFT_{N_g}(f / psi zero-padded), A f(s) = sum_taps phi F
  adjoint:  grid = sum_s c_s phi (spreading), g = IFFT_{N_g}(grid) * N_g^2,
            cropped to the n x n volume, times the same psi correction.

The two are exact transposes of each other at any M; their distance to
the exact sums of `nudft` is the USFFT approximation error.
"""
import numpy as np

from . import filters
from .geometry import centred, freqs
from .nudft import data_spectra, filter_spectra, spectra_to_detector, x3_phases


def gaussian_beta(n, N_g, M):
    R = N_g / n
    return np.pi * (R - 0.5) / (R * M)


def psi_correction(n, N_g, beta):
    x = centred(n).astype(np.float64)
    return np.sqrt(beta / np.pi) * np.exp(np.pi**2 * x**2 / (beta * N_g**2))


def slab_positions(geom, l, N_g):
    """Sample positions (X, Y) in grid cells for slab l; row s = (theta, m)."""
    ms = freqs(geom.w_p)
    ct = np.cos(geom.theta)[:, None]
    st = np.sin(geom.theta)[:, None]
    ku = (ms / geom.w_p)[None, :]
    kv = l / geom.h_p
    xi1 = ku * ct + kv * st * np.sin(geom.phi)
    xi2 = ku * st - kv * ct * np.sin(geom.phi)
    return (N_g * xi1).reshape(-1), (N_g * xi2).reshape(-1)


def _taps(X, M, beta):
    base = np.floor(X).astype(np.int64) - M + 1
    k = base[:, None] + np.arange(2 * M)[None, :]
    w = np.exp(-beta * (k - X[:, None]) ** 2)
    return k, w


def interp2d(F, X, Y, M, beta):
    """Step (3) forward: c_s = sum_{k1,k2} phi(k1 - X_s) phi(k2 - Y_s) F[k2, k1]."""
    N_g = F.shape[0]
    k1, w1 = _taps(X, M, beta)
    k2, w2 = _taps(Y, M, beta)
    out = np.zeros(len(X), dtype=np.complex128)
    for j in range(2 * M):
        rows = F[k2[:, j] % N_g]  # (S, N_g)
        vals = np.take_along_axis(rows, k1 % N_g, axis=1)  # (S, 2M)
        out += w2[:, j] * np.sum(w1 * vals, axis=1)
    return out


def spread2d(c, X, Y, N_g, M, beta):
    """Step (3) adjoint: grid[k2, k1] = sum_s c_s phi(k1 - X_s) phi(k2 - Y_s)."""
    k1, w1 = _taps(X, M, beta)
    k2, w2 = _taps(Y, M, beta)
    idx = ((k2 % N_g)[:, :, None] * N_g + (k1 % N_g)[:, None, :]).reshape(-1)
    wts = (w2[:, :, None] * w1[:, None, :] * c[:, None, None]).reshape(-1)
    re = np.bincount(idx, weights=wts.real, minlength=N_g * N_g)
    im = np.bincount(idx, weights=wts.imag, minlength=N_g * N_g)
    return (re + 1j * im).reshape(N_g, N_g)


def type2(f2, X, Y, N_g, M):
    """Equally -> unequally spaced: sum_x f2(x) exp(-2 pi i x . (X, Y)/N_g)."""
    n = f2.shape[0]
    beta = gaussian_beta(n, N_g, M)
    p = psi_correction(n, N_g, beta)
    F = np.zeros((N_g, N_g), dtype=np.complex128)
    idx = centred(n) % N_g
    F[np.ix_(idx, idx)] = f2 * p[:, None] * p[None, :]  # (1) divide by psi
    F = np.fft.fft2(F)  # (2) FFT
    return interp2d(F, X, Y, M, beta)  # (3) convolution


def type1(c, X, Y, n, N_g, M):
    """Unequally -> equally spaced: g(x) = sum_s c_s exp(+2 pi i x . (X, Y)/N_g)."""
    beta = gaussian_beta(n, N_g, M)
    p = psi_correction(n, N_g, beta)
    grid = spread2d(c, X, Y, N_g, M, beta)  # (3) adjoint convolution
    g = np.fft.ifft2(grid) * (N_g * N_g)  # (2) inverse FFT
    idx = centred(n) % N_g
    return g[np.ix_(idx, idx)] * p[:, None] * p[None, :]  # (1) divide by psi


def default_grid(n):
    N = 1
    while N < 2 * n:
        N *= 2
    return N


def forward_spectra(f, geom, M=12, N_g=None):
    N_g = default_grid(geom.n) if N_g is None else N_g
    ls = freqs(geom.h_p)
    ms = freqs(geom.w_p)
    E = x3_phases(geom, -1.0)
    ghat = np.einsum("zl,zyx->lyx", E, np.asarray(f, dtype=np.float64), optimize=True)
    A = np.empty((geom.n_theta, len(ls), len(ms)), dtype=np.complex128)
    for li, l in enumerate(ls):
        X, Y = slab_positions(geom, l, N_g)
        A[:, li, :] = type2(ghat[li], X, Y, N_g, M).reshape(geom.n_theta, len(ms))
    return A


def forward(f, geom, M=12, N_g=None):
    return spectra_to_detector(forward_spectra(f, geom, M, N_g), geom)


def backproject_spectra(G, geom, M=12, N_g=None):
    N_g = default_grid(geom.n) if N_g is None else N_g
    ls = freqs(geom.h_p)
    g = np.empty((len(ls), geom.n, geom.n), dtype=np.complex128)
    for li, l in enumerate(ls):
        X, Y = slab_positions(geom, l, N_g)
        g[li] = type1(G[:, li, :].reshape(-1), X, Y, geom.n, N_g, M)
    E = x3_phases(geom, +1.0)
    return np.einsum("zl,lyx->zyx", E, g, optimize=True).real


def adjoint(d, geom, M=12, N_g=None):
    return backproject_spectra(data_spectra(d, geom), geom, M, N_g)


def fbp(d, geom, kind=filters.SHEPP_LOGAN, M=12, N_g=None):
    G = filter_spectra(data_spectra(d, geom), geom, kind)
    return backproject_spectra(G, geom, M, N_g)
