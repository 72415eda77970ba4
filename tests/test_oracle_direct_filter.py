"""Pins of the direct FBP's row filter (oracle.direct.filter_rows).

The filter of eq:recon acts along detector rows with the transfer function
W(m) = (pi / n_theta) cos(phi) |m / w_p| window(m / w_p) on rows
zero-padded to w_p and cropped back to w.  Pinned here by
* the impulse response of the ramp filter in closed form,
      sum_{|m| <= K} |m| exp(i m t) = 2 sum_{m=1..K} m cos(m t)
        = ((K + 1) cos(K t) - K cos((K + 1) t) - 1) / (1 - cos t),  t != 0,
        = K (K + 1)                                                t = 0,
  with K = w_p / 2 - 1 (the Nyquist bin is not part of the sum), placed at
  every detector column including both edges;
* a brute-force double sum over columns and frequencies for the windowed
  filters on a tiny detector.
"""
import numpy as np
import pytest

from oracle import direct, filters
from oracle.geometry import Geometry, freqs


def _ramp_sum(K, t):
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    zero = np.isclose(np.cos(t), 1.0, rtol=0.0, atol=1e-15)
    tt = t[~zero]
    out[~zero] = ((K + 1) * np.cos(K * tt) - K * np.cos((K + 1) * tt) - 1.0) / (1.0 - np.cos(tt))
    out[zero] = K * (K + 1)
    return out


def test_closed_form_sum_itself():
    # the identity against the plain sum, before it is used as a pin
    rng = np.random.default_rng(0)
    for K in (1, 2, 7, 31):
        t = np.concatenate([[0.0], rng.uniform(-np.pi, np.pi, 20)])
        ms = np.arange(-K, K + 1)
        plain = np.abs(ms)[None, :] * np.cos(np.outer(t, ms))
        # the closed form cancels near t = 0: absolute bar relative to K (K + 1)
        assert np.allclose(_ramp_sum(K, t), plain.sum(1), rtol=1e-12, atol=1e-9 * K * (K + 1))


@pytest.mark.parametrize("w, pad_u", [(20, 2.0), (17, 2.0), (9, 1.0), (24, 3.0)])
def test_ramp_impulse_response_closed_form(w, pad_u):
    g = Geometry(nz=4, n=8, n_theta=6, h=w, w=w, phi=np.deg2rad(25), pad_u=pad_u)
    w_p = g.w_p
    K = w_p // 2 - 1
    # row r of projection 0 carries a unit impulse at column r (every column
    # once, both edges included); projection j carries it at w - 1 - r
    d = np.zeros((g.n_theta, g.h, g.w))
    for r in range(w):
        d[0, r, r] = 1.0
        d[1, r, w - 1 - r] = 1.0
    out = direct.filter_rows(d, g, filters.RAMP)
    scale = np.pi * np.cos(g.phi) / (g.n_theta * w_p * w_p)
    cols = np.arange(w)
    for r in range(w):
        for j, c0 in ((0, r), (1, w - 1 - r)):
            want = scale * _ramp_sum(K, 2.0 * np.pi * (cols - c0) / w_p)
            assert np.allclose(out[j, r], want, rtol=1e-12, atol=1e-14), (j, r)
    assert np.abs(out[2:]).max() == 0.0


@pytest.mark.parametrize("kind", [filters.SHEPP_LOGAN, filters.PARZEN, filters.RAMP])
def test_windowed_filter_brute_force(kind):
    g = Geometry(nz=4, n=8, n_theta=3, h=2, w=7, phi=np.deg2rad(40))
    rng = np.random.default_rng(5)
    d = rng.standard_normal((g.n_theta, g.h, g.w))
    w_p = g.w_p
    ms = freqs(w_p)
    W = filters.fbp_weight(ms, w_p, g.n_theta, g.phi, kind)
    want = np.zeros_like(d)
    for j in range(g.n_theta):
        for r in range(g.h):
            for c in range(g.w):
                acc = 0.0
                for c2 in range(g.w):
                    for m, wm in zip(ms, W):
                        acc += d[j, r, c2] * wm * np.cos(2.0 * np.pi * m * (c - c2) / w_p)
                want[j, r, c] = acc / w_p
    got = direct.filter_rows(d, g, kind)
    assert np.allclose(got, want, rtol=1e-11, atol=1e-13)
