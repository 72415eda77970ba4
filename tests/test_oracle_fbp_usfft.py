"""Pins of the FBP scale (eq:recon), O3 (USFFT) and O1 (direct pair)."""
import numpy as np
import pytest

from oracle import direct, filters, nudft, phantom, usfft
from oracle.geometry import Geometry, centred


def _windowed_cosine(g, xi0, s):
    x = centred(g.n)
    z = centred(g.nz)
    X3, X2, X1 = np.meshgrid(z, x, x, indexing="ij")
    env = np.exp(-(X1**2 + X2**2 + X3**2) / (2 * s * s))
    return env * np.cos(2 * np.pi * (xi0[0] * X1 + xi0[1] * X2 + xi0[2] * X3))


@pytest.mark.parametrize(
    "phi_deg, xi0, lo, hi",
    [
        (30, (0.15, 0.0, 0.05), 0.99, 1.01),  # outside the missing cone
        (30, (0.02, 0.0, 0.2), -0.02, 0.02),  # inside: |xi_perp| < |xi3| tan(phi)
        (0, (0.1, 0.1, 0.1), 0.999, 1.001),  # tomography: full coverage
    ],
)
def test_fbp_gain_outside_and_inside_missing_cone(phi_deg, xi0, lo, hi):
    # The weight (pi/n_theta) cos(phi) |k_u| comes from the Jacobian of
    # eq:uneqspace; a windowed plane wave outside the cone must come back
    # with gain 1, one inside the cone with gain ~0.
    g = Geometry(nz=32, n=32, n_theta=96, h=32, w=32, phi=np.deg2rad(phi_deg))
    f = _windowed_cosine(g, xi0, 4.0)
    r = nudft.fbp(nudft.forward(f, g), g, filters.RAMP)
    gain = np.sum(r * f) / np.sum(f * f)
    assert lo <= gain <= hi


def test_filter_windows():
    k = np.array([0.0, 0.25, 0.5])
    assert np.allclose(filters.window(k, filters.RAMP), 1)
    assert np.allclose(filters.window(k, filters.SHEPP_LOGAN), [1, np.sin(np.pi / 4) / (np.pi / 4), 2 / np.pi])
    assert np.allclose(filters.window(k, filters.PARZEN), [1, 0.25, 0])
    w = filters.fbp_weight(np.array([-3, 0, 5]), 16, 10, np.deg2rad(60), filters.RAMP)
    assert np.allclose(w, np.pi / 10 * 0.5 * np.array([3, 0, 5]) / 16)


def _small():
    return Geometry(nz=10, n=16, n_theta=12, h=10, w=16, phi=np.deg2rad(25))


def test_usfft_matches_exact_sums_at_high_accuracy():
    g = _small()
    rng = np.random.default_rng(0)
    f = rng.standard_normal((g.nz, g.n, g.n))
    d = rng.standard_normal((g.n_theta, g.h, g.w))
    A0 = nudft.forward_spectra(f, g)
    A = usfft.forward_spectra(f, g, M=12)
    assert np.linalg.norm(A - A0) / np.linalg.norm(A0) < 1e-10
    b0 = nudft.adjoint(d, g)
    b = usfft.adjoint(d, g, M=12)
    assert np.linalg.norm(b - b0) / np.linalg.norm(b0) < 1e-10


def test_usfft_error_falls_with_kernel_width():
    g = _small()
    f = np.random.default_rng(1).standard_normal((g.nz, g.n, g.n))
    A0 = nudft.forward_spectra(f, g)
    errs = [np.linalg.norm(usfft.forward_spectra(f, g, M=M) - A0) / np.linalg.norm(A0)
            for M in (2, 3, 4, 6)]
    assert all(a > 5 * b for a, b in zip(errs, errs[1:]))


def test_usfft_pair_is_exact_transpose():
    g = _small()
    rng = np.random.default_rng(2)
    f = rng.standard_normal((g.nz, g.n, g.n))
    d = rng.standard_normal((g.n_theta, g.h, g.w))
    a = np.sum(usfft.forward(f, g, M=3) * d)
    b = np.sum(f * usfft.adjoint(d, g, M=3))
    assert abs(a - b) < 1e-12 * abs(a)


def test_direct_adjoint_identity():
    g = Geometry(nz=14, n=18, n_theta=9, h=15, w=20, phi=np.deg2rad(30))
    rng = np.random.default_rng(3)
    f = rng.standard_normal((g.nz, g.n, g.n))
    d = rng.standard_normal((g.n_theta, g.h, g.w))
    Lf = direct.forward(f, g)
    a = np.sum(Lf * d)
    b = np.sum(f * direct.adjoint(d, g))
    assert abs(a - b) <= 1e-13 * np.linalg.norm(Lf) * np.linalg.norm(d)


def test_direct_mass_conservation():
    # Bilinear weights sum to one: a footprint inside the detector keeps sum f.
    g = Geometry(nz=8, n=8, n_theta=7, h=24, w=24, phi=np.deg2rad(30))
    f = np.random.default_rng(4).uniform(size=(g.nz, g.n, g.n))
    d = direct.forward(f, g)
    assert np.allclose(d.sum(axis=(1, 2)), f.sum(), rtol=1e-13)


def test_direct_converges_to_analytic_blob():
    # Linear interpolation error of a smooth blob falls like 1/s^2 as the
    # blob widens relative to the voxel: convergence to the closed form.
    errs = []
    for s in (2.0, 4.0):
        n = int(8 * s) + 8
        g = Geometry(nz=n, n=n, n_theta=6, h=n, w=n, phi=np.deg2rad(30))
        c = np.array([0.3, -0.2, 0.1])
        f = phantom.blob_volume(g.nz, g.n, c, s)
        ref = phantom.blob_projections(g.theta, g.phi, centred(g.w), centred(g.h), c, s)
        errs.append(np.linalg.norm(direct.forward(f, g) - ref) / np.linalg.norm(ref))
    assert errs[0] < 0.05
    assert errs[1] < errs[0] / 3


def test_direct_and_fourier_fbp_agree_on_smooth_object():
    # Two discretisations of eq:recon: for a smooth object both recover
    # the mid-frequency content; their gap is what the direct method's
    # linear interpolation loses.
    g = Geometry(nz=24, n=24, n_theta=64, h=24, w=24, phi=np.deg2rad(20))
    c = np.array([0.5, -0.5, 0.25])
    f = phantom.blob_volume(g.nz, g.n, c, 3.0)
    d = phantom.blob_projections(g.theta, g.phi, centred(g.w), centred(g.h), c, 3.0)
    rf = nudft.fbp(d, g, filters.SHEPP_LOGAN)
    rd = direct.fbp(d, g, filters.SHEPP_LOGAN)
    gap = np.linalg.norm(rf - rd) / np.linalg.norm(rf)
    assert gap < 0.1
    assert np.linalg.norm(rf - f) / np.linalg.norm(f) < 0.2
