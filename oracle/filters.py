"""Filter operator W of eq:recon (oracle, test infrastructure only).

The paper describes W as a convolution in u whose transfer function is a
suitably scaled |sigma| cos(phi), optionally with a low-pass window
(Shepp-Logan, Parzen).  The scale used here comes from the change of
variables (theta, k_u, k_v) -> xi of eq:uneqspace: its Jacobian is
|k_u| cos(phi), and theta in [0, 2 pi) covers every reachable xi twice, so
a Riemann sum over n_theta angles weighs each sample by
(1/2)(2 pi / n_theta) |k_u| cos(phi) = (pi / n_theta) cos(phi) |k_u|.

Windows are functions of k = m / w_p in cycles per pixel, |k| <= 1/2:
  ramp         1
  shepp-logan  sin(pi k) / (pi k)                    (sinc, textbook form)
  parzen       the Parzen (de la Vallee Poussin) window on [-1/2, 1/2]
"""
import numpy as np

RAMP, SHEPP_LOGAN, PARZEN = 0, 1, 2


def window(k, kind):
    k = np.abs(np.asarray(k, dtype=np.float64))
    if kind == RAMP:
        return np.ones_like(k)
    if kind == SHEPP_LOGAN:
        return np.sinc(k)  # numpy's sinc is sin(pi k)/(pi k)
    if kind == PARZEN:
        t = 2.0 * k  # t in [0, 1]
        inner = 1.0 - 6.0 * t**2 * (1.0 - t)
        outer = 2.0 * (1.0 - t) ** 3
        return np.where(t <= 0.5, inner, np.where(t <= 1.0, outer, 0.0))
    raise ValueError(f"unknown filter {kind}")


def fbp_weight(m, w_p, n_theta, phi, kind):
    """W(m) = (pi / n_theta) cos(phi) |m / w_p| window(m / w_p)."""
    k = np.asarray(m, dtype=np.float64) / w_p
    return (np.pi / n_theta) * np.cos(phi) * np.abs(k) * window(k, kind)
