"""Analytic phantoms with exact projections and Fourier transforms.

Oracle module (test infrastructure only).  Used to pin the geometry and
the operators against closed forms:

* the projection of eq:fwd of an object is its integral along the ray
  x = u e_u + v e_v + t b, b = e_u x e_v (the set selected by the two
  deltas);
* the Fourier-slice relation behind eq:fftfwd says the 2D Fourier
  transform of a projection at (k_u, k_v) equals the 3D Fourier transform
  of the object at xi(theta, k_u, k_v) of eq:uneqspace.

Ellipsoid: centre c, semi-axes a, rotation R (columns are the principal
axes), density rho; the set |diag(1/a) R^T (x - c)| <= 1.
  chord along p + t b:  2 sqrt(D) / (b^T A b),  A = R diag(a^-2) R^T,
  q = p - c,  D = (b^T A q)^2 - (b^T A b)(q^T A q - 1)  (0 if D < 0)
  3D transform (convention F f(xi) = int f exp(-2 pi i x.xi) dx):
  a1 a2 a3 exp(-2 pi i c.xi) B(|diag(a) R^T xi|),
  B(k) = (sin 2 pi k - 2 pi k cos 2 pi k) / (2 pi^2 k^3), B(0) = 4 pi / 3.

Gaussian blob exp(-|x - c|^2 / (2 s^2)):
  projection sqrt(2 pi) s exp(-((u - c.e_u)^2 + (v - c.e_v)^2) / (2 s^2))
  3D transform (2 pi s^2)^{3/2} exp(-2 pi i c.xi) exp(-2 pi^2 s^2 |xi|^2).
"""
from dataclasses import dataclass

import numpy as np

from .geometry import detector_axes, ray_direction


@dataclass
class Ellipsoid:
    centre: np.ndarray
    axes: np.ndarray
    rot: np.ndarray
    rho: float

    def quad(self):
        R = np.asarray(self.rot, dtype=np.float64)
        return R @ np.diag(1.0 / np.asarray(self.axes, dtype=np.float64) ** 2) @ R.T


def ellipsoid_chord(ell, p, b):
    """Length of the chord of `ell` cut by the lines p + t b (|b| = 1).

    p: (..., 3) points, b: (..., 3) unit directions (broadcast)."""
    A = ell.quad()
    q = np.asarray(p, dtype=np.float64) - np.asarray(ell.centre, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    Ab = b @ A
    bAb = np.sum(Ab * b, axis=-1)
    bAq = np.sum(Ab * q, axis=-1)
    qAq = np.sum((q @ A) * q, axis=-1)
    disc = bAq**2 - bAb * (qAq - 1.0)
    return 2.0 * np.sqrt(np.maximum(disc, 0.0)) / bAb


def detector_points(theta, phi, u, v):
    """Object-space points u e_u + v e_v for every (theta, v, u).

    Returns (points (T, V, U, 3), directions (T, 1, 1, 3))."""
    e_u, e_v = detector_axes(theta, phi)
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    pts = (
        u[None, None, :, None] * e_u[:, None, None, :]
        + v[None, :, None, None] * e_v[:, None, None, :]
    )
    b = ray_direction(theta, phi)[:, None, None, :]
    return pts, b


def ellipsoid_projections(ells, theta, phi, u, v):
    """Exact line integrals d[t, v, u] of a sum of ellipsoids (eq:fwd)."""
    pts, b = detector_points(theta, phi, u, v)
    d = np.zeros(pts.shape[:-1])
    for e in ells:
        d += e.rho * ellipsoid_chord(e, pts, b)
    return d


def unit_ball_ft(k):
    k = np.asarray(k, dtype=np.float64)
    out = np.full(k.shape, 4.0 * np.pi / 3.0)
    big = k > 1e-3
    kb = k[big]
    x = 2.0 * np.pi * kb
    out[big] = (np.sin(x) - x * np.cos(x)) / (2.0 * np.pi**2 * kb**3)
    small = ~big
    # series: 4 pi/3 (1 - (2 pi k)^2 / 10 + (2 pi k)^4 / 280)
    xs = 2.0 * np.pi * k[small]
    out[small] = 4.0 * np.pi / 3.0 * (1.0 - xs**2 / 10.0 + xs**4 / 280.0)
    return out


def ellipsoid_ft(ells, xi):
    """Exact 3D Fourier transform of a sum of ellipsoids at points xi (..., 3)."""
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros(xi.shape[:-1], dtype=np.complex128)
    for e in ells:
        a = np.asarray(e.axes, dtype=np.float64)
        k = np.linalg.norm((xi @ np.asarray(e.rot)) * a, axis=-1)
        phase = np.exp(-2j * np.pi * (xi @ np.asarray(e.centre, dtype=np.float64)))
        out += e.rho * np.prod(a) * phase * unit_ball_ft(k)
    return out


def ellipsoid_indicator(ells, pts):
    """Density of a sum of ellipsoids at points pts (..., 3)."""
    pts = np.asarray(pts, dtype=np.float64)
    out = np.zeros(pts.shape[:-1])
    for e in ells:
        q = pts - np.asarray(e.centre, dtype=np.float64)
        y = (q @ np.asarray(e.rot)) / np.asarray(e.axes, dtype=np.float64)
        out += e.rho * (np.sum(y * y, axis=-1) <= 1.0)
    return out


def blob_volume(nz, n, centre, s, voxel=1.0):
    """Gaussian blob sampled at the voxel centres of an nz x n x n grid."""
    x = (np.arange(n) - n // 2) * voxel
    z = (np.arange(nz) - nz // 2) * voxel
    c = np.asarray(centre, dtype=np.float64)
    r2 = (
        (z[:, None, None] - c[2]) ** 2
        + (x[None, :, None] - c[1]) ** 2
        + (x[None, None, :] - c[0]) ** 2
    )
    return np.exp(-r2 / (2.0 * s * s))


def blob_projections(theta, phi, u, v, centre, s):
    """Exact line integrals of a Gaussian blob at every (theta, v, u)."""
    e_u, e_v = detector_axes(theta, phi)
    c = np.asarray(centre, dtype=np.float64)
    cu = e_u @ c
    cv = e_v @ c
    du = np.asarray(u, dtype=np.float64)[None, None, :] - cu[:, None, None]
    dv = np.asarray(v, dtype=np.float64)[None, :, None] - cv[:, None, None]
    return np.sqrt(2.0 * np.pi) * s * np.exp(-(du**2 + dv**2) / (2.0 * s * s))


def blob_ft(xi, centre, s):
    xi = np.asarray(xi, dtype=np.float64)
    c = np.asarray(centre, dtype=np.float64)
    k2 = np.sum(xi * xi, axis=-1)
    return (
        (2.0 * np.pi * s * s) ** 1.5
        * np.exp(-2j * np.pi * (xi @ c))
        * np.exp(-2.0 * np.pi**2 * s * s * k2)
    )
