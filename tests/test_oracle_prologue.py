"""Pins of O6 (dark/flat correction and -log) against the recording model."""
import numpy as np

import synth
from oracle import nudft, prologue
from oracle.geometry import Geometry


def test_round_trip_of_the_recording_model_is_exact():
    # raw = exp(-d) (flat - dark) + dark, evaluated in float64 without
    # rounding to integers, must give d back to rounding error
    rng = np.random.default_rng(0)
    d = rng.uniform(0.0, 4.0, (5, 6, 7))
    dark = rng.uniform(50, 150, (6, 7))
    flat = rng.uniform(2e4, 5e4, (6, 7))
    raw = np.exp(-d) * (flat - dark) + dark
    out = prologue.flat_dark_log(raw, dark, flat, 1e-6)
    assert np.abs(out - d).max() < 1e-10


def test_hand_values_and_clamping():
    dark = np.array([[100.0, 100.0, 100.0, 100.0]])
    flat = np.array([[1100.0, 1100.0, 1100.0, 90.0]])
    raw = np.array([[[600.0, 1100.0, 50.0, 500.0]]])
    out = prologue.flat_dark_log(raw, dark, flat, 1e-3)[0, 0]
    assert np.isclose(out[0], np.log(2.0))          # half the open-beam signal
    assert out[1] == 0.0                            # open beam
    assert np.isclose(out[2], -np.log(1e-3))        # below the dark level: clamped
    assert np.isclose(out[3], -np.log(1e-3))        # dead pixel (flat <= dark)


def test_corrected_counts_reconstruct_like_the_line_integrals():
    # integer counts add rounding and photon noise of relative size
    # 1/sqrt(counts) ~ 1e-2 at most, so the FBP of the corrected counts must
    # stay that close to the FBP of the exact line integrals
    g = Geometry(nz=8, n=8, n_theta=12, h=8, w=10, phi=np.deg2rad(30))
    rng = np.random.default_rng(1)
    f = np.abs(rng.standard_normal((8, 8, 8))) * 0.05
    d = nudft.forward(f, g)
    raw, dark, flat = synth.raw_counts(np.maximum(d, 0), seed=2)
    dc = prologue.flat_dark_log(raw, dark, flat, 1e-6)
    assert np.abs(dc - d).max() < 0.05
    a = nudft.fbp(dc, g)
    b = nudft.fbp(d, g)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 0.1
