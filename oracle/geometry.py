"""Scan geometry and discrete grids (oracle, test infrastructure only).

Follows Section "Laminography reconstruction":

* eq:fwd -- a ray is fixed by two delta functions.  The first says
  x1 cos(theta) + x2 sin(theta) = u, the second says
  x1 sin(theta) sin(phi) - x2 cos(theta) sin(phi) + x3 cos(phi) = v.
  Hence the detector axes in object space are
  e_u = (cos t, sin t, 0) and e_v = (sin t sin p, -cos t sin p, cos p).
  phi = 0 is ordinary tomography (the paper says so right after the
  Beer-Lambert formula), so phi is read from the formulas, not from the
  prose definition of the tilt.
* eq:uneqspace -- the frequency of detector frequency (k_u, k_v) at angle
  theta is xi = k_u e_u + k_v e_v.

Discrete conventions (the paper states none; these are the readings used
by both sides of the parity tests, each written independently):

* volume vol[z][y][x], nz x n x n, voxel = 1, x1 = x - n//2,
  x2 = y - n//2, x3 = z - nz//2 (integer coordinates, so every
  exponential exp(-2 pi i x.xi) is 1-periodic in xi);
* detector d[j][r][c], h x w, u = c - w//2, v = r - h//2;
* theta_j = 2 pi j / n_theta (a full circle: laminography needs it);
* the detector is zero-padded to h_p x w_p, the smallest powers of two
  that are >= pad * (h, w); frequencies k_u = m / w_p, k_v = l / h_p with
  m in [-w_p/2+1, w_p/2-1], l in [-h_p/2+1, h_p/2-1] (the Nyquist bins are
  dropped so that every frequency has its mirror image).
"""
from dataclasses import dataclass

import numpy as np


def pow2_at_least(x):
    """Smallest power of two >= x (x >= 1)."""
    p = 1
    while p < x:
        p *= 2
    return p


def centred(n):
    """Integer coordinates of n samples with the origin at index n//2."""
    return np.arange(n) - n // 2


def freqs(N):
    """Frequency indices of an N-point grid without the Nyquist bin."""
    return np.arange(-N // 2 + 1, N // 2)


def default_angles(n_theta):
    """theta_j = 2 pi j / n_theta over the full circle."""
    return 2.0 * np.pi * np.arange(n_theta) / n_theta


@dataclass
class Geometry:
    nz: int
    n: int
    n_theta: int
    h: int
    w: int
    phi: float  # tilt, radians; 0 == tomography
    theta: np.ndarray = None
    pad_u: float = 2.0
    pad_v: float = 2.0

    def __post_init__(self):
        if self.theta is None:
            self.theta = default_angles(self.n_theta)
        self.theta = np.asarray(self.theta, dtype=np.float64)
        assert self.theta.shape == (self.n_theta,)

    @property
    def w_p(self):
        return pow2_at_least(int(np.ceil(self.pad_u * self.w)))

    @property
    def h_p(self):
        return pow2_at_least(int(np.ceil(self.pad_v * self.h)))


def detector_axes(theta, phi):
    """e_u(theta), e_v(theta) read off the two deltas of eq:fwd.

    Returns arrays of shape theta.shape + (3,)."""
    theta = np.asarray(theta, dtype=np.float64)
    ct, st = np.cos(theta), np.sin(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    e_u = np.stack([ct, st, np.zeros_like(ct)], axis=-1)
    e_v = np.stack([st * sp, -ct * sp, np.full_like(ct, cp)], axis=-1)
    return e_u, e_v


def ray_direction(theta, phi):
    """Unit vector along the ray: orthogonal to both detector axes."""
    e_u, e_v = detector_axes(theta, phi)
    return np.cross(e_u, e_v)


def xi(theta, ku, kv, phi):
    """eq:uneqspace: (xi1, xi2, xi3) for angle theta, detector freq (ku, kv).

    Arguments broadcast against each other."""
    theta = np.asarray(theta, dtype=np.float64)
    ct, st = np.cos(theta), np.sin(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    xi1 = ku * ct + kv * st * sp
    xi2 = ku * st - kv * ct * sp
    xi3 = kv * cp + 0.0 * ku * ct
    return xi1, xi2, xi3


def project_point(x, theta, phi):
    """Detector coordinates (u, v) hit by the ray through object point x."""
    e_u, e_v = detector_axes(theta, phi)
    x = np.asarray(x, dtype=np.float64)
    return e_u @ x, e_v @ x
