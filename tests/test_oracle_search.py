"""Pins of O7 (axis and tilt search)."""
import numpy as np

from oracle import nudft, phantom, search
from oracle.geometry import Geometry, centred


def _geom(phi=np.deg2rad(25)):
    return Geometry(nz=8, n=12, n_theta=16, h=10, w=16, phi=phi)


def test_integer_axis_offset_equals_moving_detector_columns():
    g = _geom()
    rng = np.random.default_rng(0)
    d = rng.standard_normal((g.n_theta, g.h, g.w))
    d[..., :3] = 0.0  # zero margins: no column leaves the detector
    d[..., -3:] = 0.0
    for delta in (-2, 1, 3):
        moved = np.zeros_like(d)
        # axis at w/2 + delta: column c of the recording is column c - delta of a centred one
        if delta > 0:
            moved[..., : g.w - delta] = d[..., delta:]
        else:
            moved[..., -delta:] = d[..., : g.w + delta]
        a = search.fbp_shifted(d, g, delta)
        b = nudft.fbp(moved, g)
        assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()


def test_fractional_offset_recovers_shifted_sampling_of_a_smooth_phantom():
    # a Gaussian blob recorded with the axis at w/2 + 0.5 (samples at
    # u = c - w/2 - 0.5) is re-centred by the phase ramp to the blob recorded
    # with the axis at w/2, up to the interpolation error of a smooth row
    g = Geometry(nz=12, n=16, n_theta=24, h=16, w=24, phi=np.deg2rad(20))
    centre, s = (1.0, -0.5, 0.7), 2.5
    u0 = centred(g.w).astype(float)
    v = centred(g.h).astype(float)
    delta = 0.5
    rec = phantom.blob_projections(g.theta, g.phi, u0 - delta, v, centre, s)
    ref = phantom.blob_projections(g.theta, g.phi, u0, v, centre, s)
    a = search.fbp_shifted(rec, g, delta)
    b = nudft.fbp(ref, g)
    e = np.linalg.norm(a - b) / np.linalg.norm(b)
    unshifted = np.linalg.norm(nudft.fbp(rec, g) - b) / np.linalg.norm(b)
    assert e < 1e-3 and unshifted > 50 * e


def test_sweeps_are_fbp_slices():
    g = _geom()
    d = np.random.default_rng(1).standard_normal((g.n_theta, g.h, g.w))
    cs = search.center_sweep(d, g, [0.0, 0.25], z=3)
    assert np.abs(cs[0] - nudft.fbp(d, g)[3]).max() < 1e-12 * np.abs(cs[0]).max()
    ts = search.tilt_sweep(d, g, [np.deg2rad(20), np.deg2rad(30)], 0.0, z=5)
    g30 = Geometry(nz=g.nz, n=g.n, n_theta=g.n_theta, h=g.h, w=g.w, phi=np.deg2rad(30))
    assert np.abs(ts[1] - nudft.fbp(d, g30)[5]).max() < 1e-12 * np.abs(ts[1]).max()
