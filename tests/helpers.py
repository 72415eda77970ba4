"""Shared helpers of the GPU tests (inputs, tolerances, comparisons)."""
import numpy as np
import torch

import synth
from oracle import phantom
from oracle.geometry import Geometry, centred

# Relative L2 tolerances.  FP32 arithmetic with the default Gaussian
# half-width (M = 5, USFFT error ~1e-6) must match the exact discrete
# operators to 1e-4; FP16/BF16 storage with M = 3 to 1e-2.
TOL_F32 = 1e-4
TOL_LOWP = 1e-2


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev():
    return torch.device("cuda", 0)


def to_dev(x, dtype=torch.float32):
    return torch.tensor(np.asarray(x), dtype=dtype, device=dev())


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def ellipsoid_data(count, nz, n, n_theta, h, w, phi, noise, seed=0, noise_seed=1, theta=None):
    """Exact ellipsoid projections (oracle closed form) plus Gaussian noise."""
    ells = synth.random_ellipsoids(count, nz, n, seed=seed)
    objs = [phantom.Ellipsoid(c, a, r, p) for c, a, r, p in zip(*ells)]
    g = Geometry(nz=nz, n=n, n_theta=n_theta, h=h, w=w, phi=phi, theta=theta)
    d = phantom.ellipsoid_projections(objs, g.theta, phi, centred(w), centred(h))
    if noise:
        d = synth.add_noise(torch.from_numpy(d), noise, seed=noise_seed).numpy()
    return g, ells, d
