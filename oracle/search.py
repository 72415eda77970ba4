"""O7: rotation-axis and tilt search (oracle, test only).

The tilt of the wedge and the detector column of the rotation axis are only
approximately known; the paper finds both by reconstructing one slice for
a sweep of axis positions at a fixed tilt, then one slice for a sweep of
tilts at the chosen axis (Section "Mouse brain imaging": the search steps),
and judging the slices by eye.

Axis position.  With the axis at detector column w/2 + delta instead of
w/2, the recorded column c sees u = c - w/2 - delta.  In the Fourier route
the correction is exact for the trigonometric interpolant of the padded
rows: the row spectra are multiplied by exp(2 pi i m delta / w_p) before
backprojection (a translation by delta columns; fractional delta allowed).
Tilt.  Each tilt is a different geometry (xi of eq:uneqspace and the x3
phases change), i.e. a separate FBP.

Pinned in tests/test_oracle_search.py: an integer delta equals moving the
detector columns, a fractional delta recovers data sampled at the shifted
positions of a smooth analytic phantom, and sweeps reduce to FBPs.
"""
import numpy as np

from . import filters, nudft
from .geometry import Geometry, freqs


def axis_phase(geom, delta):
    """exp(2 pi i m delta / w_p) over the row frequencies m of the spectra."""
    ms = freqs(geom.w_p)
    return np.exp(2j * np.pi * ms * delta / geom.w_p)


def fbp_shifted(d, geom, delta, kind=filters.SHEPP_LOGAN):
    """FBP of data whose rotation axis sits at column w/2 + delta."""
    G = nudft.filter_spectra(nudft.data_spectra(d, geom), geom, kind)
    return nudft.backproject_spectra(G * axis_phase(geom, delta)[None, None, :], geom)


def center_sweep(d, geom, deltas, z, kind=filters.SHEPP_LOGAN):
    """Slice z of the FBP for every axis offset: (len(deltas), n, n)."""
    return np.stack([fbp_shifted(d, geom, dl, kind)[z] for dl in deltas])


def tilt_sweep(d, geom, tilts, delta, z, kind=filters.SHEPP_LOGAN):
    """Slice z of the FBP for every tilt (radians) at axis offset delta."""
    out = []
    for phi in tilts:
        g = Geometry(nz=geom.nz, n=geom.n, n_theta=geom.n_theta, h=geom.h, w=geom.w, phi=phi,
                     theta=geom.theta, pad_u=geom.pad_u, pad_v=geom.pad_v)
        out.append(fbp_shifted(d, g, delta, kind)[z])
    return np.stack(out)
