"""Pins of the oracle's geometry and analytic phantoms (CPU only)."""
import os

import numpy as np
import pytest

from oracle import geometry, phantom
from oracle.geometry import centred

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "geometry_points.txt")


def test_projected_points_match_hand_values():
    # eq:fwd: hand-computed (u, v) of a few object points.
    rows = np.loadtxt(GOLDEN)
    for th, ph, x1, x2, x3, u, v in rows:
        uu, vv = geometry.project_point([x1, x2, x3], np.deg2rad(th), np.deg2rad(ph))
        assert uu == pytest.approx(u, abs=1e-14)
        assert vv == pytest.approx(v, abs=1e-14)


def test_detector_axes_orthonormal():
    th = np.linspace(0, 2 * np.pi, 37)
    for ph in [0.0, 0.3, np.pi / 4, 1.2]:
        e_u, e_v = geometry.detector_axes(th, ph)
        b = geometry.ray_direction(th, ph)
        assert np.allclose(np.sum(e_u * e_v, -1), 0, atol=1e-15)
        assert np.allclose(np.linalg.norm(e_u, axis=-1), 1, atol=1e-15)
        assert np.allclose(np.linalg.norm(e_v, axis=-1), 1, atol=1e-15)
        assert np.allclose(np.linalg.norm(b, axis=-1), 1, atol=1e-15)
        assert np.allclose(np.sum(b * e_u, -1), 0, atol=1e-15)


def test_xi_is_combination_of_detector_axes():
    # eq:uneqspace equals k_u e_u + k_v e_v (the Fourier-slice relation).
    rng = np.random.default_rng(3)
    th = rng.uniform(0, 2 * np.pi, 50)
    ku = rng.uniform(-0.5, 0.5, 50)
    kv = rng.uniform(-0.5, 0.5, 50)
    ph = 0.44
    e_u, e_v = geometry.detector_axes(th, ph)
    ref = ku[:, None] * e_u + kv[:, None] * e_v
    got = np.stack(geometry.xi(th, ku, kv, ph), -1)
    assert np.allclose(got, ref, atol=1e-15)


def test_slab_zero_is_polar_grid():
    th = np.linspace(0, 2 * np.pi, 11)
    ku = np.linspace(-0.5, 0.5, 7)
    x1, x2, x3 = geometry.xi(th[:, None], ku[None, :], 0.0, 0.5)
    assert np.allclose(x1, ku[None, :] * np.cos(th)[:, None])
    assert np.allclose(x2, ku[None, :] * np.sin(th)[:, None])
    assert np.allclose(x3, 0)


def test_padding_sizes():
    g = geometry.Geometry(nz=64, n=64, n_theta=8, h=64, w=320, phi=0.3)
    assert g.w_p == 1024 and g.h_p == 128
    assert list(geometry.freqs(8)) == [-3, -2, -1, 0, 1, 2, 3]
    assert list(centred(5)) == [-2, -1, 0, 1, 2]


def _random_ellipsoid(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])
    return phantom.Ellipsoid(rng.uniform(-1, 1, 3), rng.uniform(1, 3, 3), R, 0.7)


def test_chord_matches_numerical_integration():
    rng = np.random.default_rng(5)
    e = _random_ellipsoid(rng)
    b = rng.standard_normal(3)
    b /= np.linalg.norm(b)
    t = np.linspace(-10, 10, 400001)
    dt = t[1] - t[0]
    for _ in range(5):
        p = e.centre + rng.uniform(-1, 1, 3)
        pts = p[None, :] + t[:, None] * b[None, :]
        num = np.sum(phantom.ellipsoid_indicator([e], pts)) * dt / e.rho
        ana = phantom.ellipsoid_chord(e, p, b)
        assert abs(num - ana) < 2e-4


def test_unit_ball_transform():
    from scipy.integrate import quad

    assert phantom.unit_ball_ft(np.array([0.0]))[0] == pytest.approx(4 * np.pi / 3)
    for k in [1e-4, 0.3, 0.9, 2.2]:
        # radial form of the 3D transform of the unit ball
        num = quad(lambda r: 4 * np.pi * r * r * np.sinc(2 * k * r), 0, 1, limit=200)[0]
        assert phantom.unit_ball_ft(np.array([k]))[0] == pytest.approx(num, rel=1e-7, abs=1e-10)


@pytest.mark.parametrize("ph", [0.0, np.deg2rad(30)])
def test_fourier_slice_identity_ellipsoid(ph):
    # eq:fftfwd in the continuum: 2D transform of an exact projection
    # equals the 3D transform at xi(theta, k_u, k_v).
    rng = np.random.default_rng(11)
    e = _random_ellipsoid(rng)
    step = 0.02
    u = np.arange(-6, 6, step)
    th = np.array([0.7, 2.9])
    d = phantom.ellipsoid_projections([e], th, ph, u, u)
    ks = [(0.05, 0.0), (0.1, -0.07), (-0.13, 0.2), (0.0, 0.3)]
    for ti in range(len(th)):
        for ku, kv in ks:
            ft2 = np.sum(d[ti] * np.exp(-2j * np.pi * (u[None, :] * ku + u[:, None] * kv))) * step**2
            x = np.stack(geometry.xi(th[ti], ku, kv, ph), -1)
            ft3 = phantom.ellipsoid_ft([e], x[None, :])[0]
            assert abs(ft2 - ft3) < 2e-3 * abs(phantom.ellipsoid_ft([e], np.zeros((1, 3)))[0])


def test_fourier_slice_identity_blob():
    c = np.array([0.4, -0.3, 0.2])
    s = 0.8
    step = 0.05
    u = np.arange(-6, 6, step)
    th = np.array([1.1])
    ph = 0.5
    d = phantom.blob_projections(th, ph, u, u, c, s)
    for ku, kv in [(0.1, 0.2), (-0.3, 0.05)]:
        ft2 = np.sum(d[0] * np.exp(-2j * np.pi * (u[None, :] * ku + u[:, None] * kv))) * step**2
        x = np.stack(geometry.xi(th[0], ku, kv, ph), -1)
        assert abs(ft2 - phantom.blob_ft(x[None, :], c, s)[0]) < 1e-10


def test_projection_mass_is_volume():
    rng = np.random.default_rng(2)
    e = _random_ellipsoid(rng)
    step = 0.02
    u = np.arange(-6, 6, step)
    d = phantom.ellipsoid_projections([e], np.array([0.3]), 0.4, u, u)
    vol = 4 / 3 * np.pi * np.prod(e.axes) * e.rho
    assert np.sum(d) * step**2 == pytest.approx(vol, rel=1e-4)
