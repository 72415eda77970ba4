"""Pins of O2, the exact discrete Fourier pair (CPU only)."""
import numpy as np
import pytest

from oracle import nudft, phantom
from oracle.geometry import Geometry, centred, detector_axes, freqs


def _geom(nz=12, n=14, n_theta=8, h=10, w=14, phi=np.deg2rad(30)):
    return Geometry(nz=nz, n=n, n_theta=n_theta, h=h, w=w, phi=phi)


def test_matches_bruteforce_definition():
    # eq:fftfwdsplit reorders the sum; the single-loop definition fixes it.
    g = Geometry(nz=3, n=4, n_theta=3, h=3, w=5, phi=0.4)
    f = np.random.default_rng(0).standard_normal((3, 4, 4))
    ref = nudft.forward_bruteforce(f, g)
    assert np.abs(nudft.forward(f, g) - ref).max() < 1e-13 * np.abs(ref).max()


def test_gaussian_blob_closed_form():
    # A nearly band-limited blob: the exact discrete L must reproduce the
    # closed-form line integrals of the continuous blob.
    for phi in [0.0, np.deg2rad(30)]:
        g = Geometry(nz=24, n=28, n_theta=10, h=24, w=28, phi=phi)
        c = np.array([1.3, -0.7, 0.4])
        f = phantom.blob_volume(g.nz, g.n, c, 2.0)
        ref = phantom.blob_projections(g.theta, g.phi, centred(g.w), centred(g.h), c, 2.0)
        d = nudft.forward(f, g)
        assert np.linalg.norm(d - ref) / np.linalg.norm(ref) < 1e-7


def _dirichlet(t, N):
    """(1/N) sum_{m=-N/2+1}^{N/2-1} exp(2 pi i m t / N) in closed form."""
    t = np.asarray(t, dtype=np.float64)
    s = np.sin(np.pi * t / N)
    out = np.empty_like(t)
    small = np.abs(s) < 1e-12
    out[~small] = np.sin(np.pi * t[~small] * (N - 1) / N) / (N * s[~small])
    # at integer multiples of N every term equals 1
    out[small] = (N - 1) / N
    return out


def test_single_voxel_is_dirichlet_kernel():
    # A unit voxel at x projects to a separable Dirichlet kernel centred
    # at (x.e_u, x.e_v): pins geometry, Nyquist handling and scaling.
    g = _geom()
    f = np.zeros((g.nz, g.n, g.n))
    iz, iy, ix = 8, 3, 10
    f[iz, iy, ix] = 1.0
    x = np.array([ix - g.n // 2, iy - g.n // 2, iz - g.nz // 2], dtype=float)
    e_u, e_v = detector_axes(g.theta, g.phi)
    pu, pv = e_u @ x, e_v @ x
    u, v = centred(g.w), centred(g.h)
    ref = _dirichlet(v[None, :, None] - pv[:, None, None], g.h_p) * _dirichlet(
        u[None, None, :] - pu[:, None, None], g.w_p
    )
    assert np.abs(nudft.forward(f, g) - ref).max() < 1e-13


def test_adjoint_identity():
    g = _geom()
    rng = np.random.default_rng(1)
    f = rng.standard_normal((g.nz, g.n, g.n))
    d = rng.standard_normal((g.n_theta, g.h, g.w))
    a = np.sum(nudft.forward(f, g) * d)
    b = np.sum(f * nudft.adjoint(d, g))
    assert abs(a - b) <= 1e-12 * np.linalg.norm(nudft.forward(f, g)) * np.linalg.norm(d)


def test_outputs_are_real():
    # Hermitian symmetry of the symmetric frequency ranges: the imaginary
    # part of both sums vanishes for real inputs.
    g = _geom()
    rng = np.random.default_rng(2)
    f = rng.standard_normal((g.nz, g.n, g.n))
    d = rng.standard_normal((g.n_theta, g.h, g.w))
    re, im = nudft.forward(f, g, imag=True)
    assert np.abs(im).max() < 1e-12 * np.abs(re).max()
    re, im = nudft.backproject_spectra(nudft.data_spectra(d, g), g, imag=True)
    assert np.abs(im).max() < 1e-12 * np.abs(re).max()


def test_mass_over_padded_period():
    # Summed over the whole padded period, each projection carries sum f.
    g = _geom()
    f = np.random.default_rng(3).standard_normal((g.nz, g.n, g.n))
    d = nudft.forward(f, g, rows=np.arange(-g.h_p // 2, g.h_p // 2),
                      cols=np.arange(-g.w_p // 2, g.w_p // 2))
    assert np.allclose(d.sum(axis=(1, 2)), f.sum(), rtol=0, atol=1e-11 * np.abs(f).sum())


def test_rotation_by_quarter_turn_shifts_angles():
    # f(-x2, x1, x3) (a quarter turn about x3) projects at theta like f at
    # theta + pi/2: exact when the phantom vanishes on the -n/2 row.
    g = _geom(n_theta=8)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((g.nz, g.n, g.n))
    f[:, 0, :] = 0
    f[:, :, 0] = 0
    fr = np.zeros_like(f)
    c = g.n // 2
    for iy in range(g.n):
        for ix in range(g.n):
            sx, sy = -(iy - c), ix - c  # source point (x1, x2) = (-x2', x1')
            if -c <= sx < g.n - c and -c <= sy < g.n - c:
                fr[:, iy, ix] = f[:, sy + c, sx + c]
    d = nudft.forward(f, g)
    dr = nudft.forward(fr, g)
    shift = g.n_theta // 4
    assert np.abs(dr - np.roll(d, -shift, axis=0)).max() < 1e-12 * np.abs(d).max()


def test_tomography_special_case_separates():
    # phi = 0: a single non-zero slice x3 = z0 gives data that factor as
    # K_h(v - z0) p(theta, u), the 2D transform of that slice.
    g = _geom(phi=0.0)
    f = np.zeros((g.nz, g.n, g.n))
    z0 = 7
    f[z0] = np.random.default_rng(5).standard_normal((g.n, g.n))
    d = nudft.forward(f, g)
    kv = _dirichlet(centred(g.h) - (z0 - g.nz // 2), g.h_p)
    p = d[:, np.argmax(np.abs(kv)), :] / kv[np.argmax(np.abs(kv))]
    assert np.abs(d - kv[None, :, None] * p[:, None, :]).max() < 1e-12 * np.abs(d).max()
    # and p is the 2D Fourier-route projection of the slice
    ms = freqs(g.w_p)
    x = centred(g.n)
    ref = np.zeros((g.n_theta, g.w))
    for t, th in enumerate(g.theta):
        ph = np.exp(-2j * np.pi * (ms[:, None, None] / g.w_p) *
                    (x[None, None, :] * np.cos(th) + x[None, :, None] * np.sin(th)))
        A = np.sum(ph * f[z0][None], axis=(1, 2))
        ref[t] = (np.exp(2j * np.pi * np.outer(centred(g.w), ms) / g.w_p) @ A).real / g.w_p
    assert np.abs(p - ref).max() < 1e-12 * np.abs(ref).max()


def test_data_spectra_match_library_fft():
    g = _geom()
    d = np.random.default_rng(6).standard_normal((g.n_theta, g.h, g.w))
    pad = np.zeros((g.n_theta, g.h_p, g.w_p))
    pad[np.ix_(np.arange(g.n_theta), centred(g.h) % g.h_p, centred(g.w) % g.w_p)] = d
    F = np.fft.fft2(pad) / (g.h_p * g.w_p)
    ls, ms = freqs(g.h_p), freqs(g.w_p)
    ref = F[:, (ls % g.h_p)[:, None], (ms % g.w_p)[None, :]]
    assert np.abs(nudft.data_spectra(d, g) - ref).max() < 1e-14


def test_backproject_columns_matches_full():
    g = _geom()
    d = np.random.default_rng(7).standard_normal((g.n_theta, g.h, g.w))
    G = nudft.data_spectra(d, g)
    full = nudft.backproject_spectra(G, g)
    ys, xs = np.array([0, 5, 13]), np.array([2, 9, 13])
    cols = nudft.backproject_columns(G, g, ys, xs)
    assert np.abs(cols - full[:, ys, xs]).max() < 1e-12 * np.abs(full).max()


def test_fft_spectra_match_explicit_sums():
    g = _geom()
    d = np.random.default_rng(8).standard_normal((g.n_theta, g.h, g.w))
    G = nudft.data_spectra(d, g)
    assert np.abs(nudft.data_spectra_fft(d, g) - G).max() < 1e-14
    assert np.abs(nudft.data_spectra_fft(d, g, half=True) - G[:, g.h_p // 2 - 1:, :]).max() < 1e-14
