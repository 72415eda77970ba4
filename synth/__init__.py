"""Seeded synthetic inputs for tests and benchmarks.

Stand-ins for the paper's datasets (which are not available): random
ellipsoid phantoms, their exact projections, Gaussian noise and
log-normal speckle.  This module contains no part of the reconstruction
method; it is the only code shared by the oracle-side and the GPU-side
tests.

Recipe (all draws from numpy's PCG64 with the given seed):
  centres     U[-0.3, 0.3] * (n, n, nz)        (x1, x2, x3)
  semi-axes   U[0.05, 0.25] * (n, n, nz)
  rotation    uniform on SO(3) (unit quaternion from 4 normals)
  density     U[0, 1]; densities of overlapping ellipsoids add
  noise       i.i.d. N(0, (p * rms(d))^2), its own seed
  speckle     d * exp(a Z - a^2 / 2), Z ~ N(0, 1) per pixel (log-normal)
  raw counts  detector images of line integrals d under the recording model
              raw = exp(-d) (flat - dark) + dark: dark ~ dark_level (1 + 0.05 Z),
              flat ~ flat_level (1 + 0.05 Z) per pixel, Poisson-like noise
              sqrt(raw) Z, rounded and clipped to the integer type

Projections are exact chord lengths along the rays of the scan: the ray
hitting detector pixel (u, v) at angle theta is u e_u + v e_v + t b with
e_u = (cos t, sin t, 0), e_v = (sin t sin p, -cos t sin p, cos p),
b = e_u x e_v, u = c - w//2, v = r - h//2.
"""
import numpy as np
import torch


def random_ellipsoids(count, nz, n, seed=0):
    """Arrays (centres (E,3), axes (E,3), rots (E,3,3), rho (E,))."""
    rng = np.random.default_rng(seed)
    scale = np.array([n, n, nz], dtype=np.float64)
    centres = rng.uniform(-0.3, 0.3, size=(count, 3)) * scale
    axes = rng.uniform(0.05, 0.25, size=(count, 3)) * scale
    q = rng.standard_normal((count, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    rots = np.stack(
        [
            np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
            np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
            np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
        ],
        axis=1,
    )
    rho = rng.uniform(0.0, 1.0, size=count)
    return centres, axes, rots, rho


def angles(n_theta):
    return 2.0 * np.pi * np.arange(n_theta) / n_theta


def project_ellipsoids(ells, n_theta, h, w, phi, theta=None, device="cpu",
                       dtype=torch.float64, theta_chunk=16):
    """Exact projections d[t, r, c] of the ellipsoid sum, as a torch tensor."""
    centres, axes, rots, rho = ells
    theta = angles(n_theta) if theta is None else np.asarray(theta, dtype=np.float64)
    out = torch.zeros((n_theta, h, w), dtype=dtype, device=device)
    u = torch.arange(w, dtype=dtype, device=device) - (w // 2)
    v = torch.arange(h, dtype=dtype, device=device) - (h // 2)
    A = [torch.tensor(r @ np.diag(1.0 / a**2) @ r.T, dtype=dtype, device=device)
         for r, a in zip(rots, axes)]
    C = [torch.tensor(c, dtype=dtype, device=device) for c in centres]
    sp, cp = np.sin(phi), np.cos(phi)
    for t0 in range(0, n_theta, theta_chunk):
        th = torch.tensor(theta[t0:t0 + theta_chunk], dtype=dtype, device=device)
        ct, st = torch.cos(th), torch.sin(th)
        zero = torch.zeros_like(ct)
        e_u = torch.stack([ct, st, zero], -1)
        e_v = torch.stack([st * sp, -ct * sp, torch.full_like(ct, cp)], -1)
        b = torch.linalg.cross(e_u, e_v, dim=-1)  # (T, 3)
        p = u[None, None, :, None] * e_u[:, None, None, :] + v[None, :, None, None] * e_v[:, None, None, :]
        acc = torch.zeros(p.shape[:-1], dtype=dtype, device=device)
        for Ai, ci, ri in zip(A, C, rho):
            q = p - ci
            Ab = b @ Ai  # (T, 3)
            bAb = (Ab * b).sum(-1)[:, None, None]
            bAq = (q * Ab[:, None, None, :]).sum(-1)
            qAq = ((q @ Ai) * q).sum(-1)
            disc = torch.clamp(bAq * bAq - bAb * (qAq - 1.0), min=0.0)
            acc += float(ri) * 2.0 * torch.sqrt(disc) / bAb
        out[t0:t0 + theta_chunk] = acc
    return out


def voxelize_ellipsoids(ells, nz, n, device="cpu", dtype=torch.float64):
    """Ellipsoid densities sampled at voxel centres (vol[z][y][x])."""
    centres, axes, rots, rho = ells
    x = torch.arange(n, dtype=dtype, device=device) - (n // 2)
    z = torch.arange(nz, dtype=dtype, device=device) - (nz // 2)
    P = torch.stack(torch.meshgrid(z, x, x, indexing="ij")[::-1], -1)  # (nz,n,n,3) as (x1,x2,x3)
    vol = torch.zeros((nz, n, n), dtype=dtype, device=device)
    for c, a, r, ro in zip(centres, axes, rots, rho):
        q = P - torch.tensor(c, dtype=dtype, device=device)
        y = (q @ torch.tensor(r, dtype=dtype, device=device)) / torch.tensor(a, dtype=dtype, device=device)
        vol += float(ro) * ((y * y).sum(-1) <= 1.0).to(dtype)
    return vol


def add_noise(d, level, seed=1):
    """d + N(0, (level * rms(d))^2) i.i.d., numpy generator with `seed`."""
    rng = np.random.default_rng(seed)
    rms = float(torch.sqrt(torch.mean(d.double() ** 2)))
    z = torch.from_numpy(rng.standard_normal(tuple(d.shape))).to(d.device, d.dtype)
    return d + (level * rms) * z


def apply_speckle(d, amp, seed=1):
    """Log-normal multiplicative speckle with unit mean."""
    rng = np.random.default_rng(seed)
    z = torch.from_numpy(rng.standard_normal(tuple(d.shape)).astype(np.float32)).to(d.device)
    return d * torch.exp(amp * z - 0.5 * amp * amp).to(d.dtype)


def random_array(shape, seed, dtype=np.float64):
    """Standard-normal test array."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


def raw_counts(d, dark_level=100.0, flat_level=4.0e4, seed=5, dtype=np.uint16):
    """Seeded raw detector counts for line integrals d[n_theta][h][w]
    (numpy float64): returns (raw, dark, flat) with dark and flat as
    float32 [h][w] images and raw as the integer dtype."""
    d = np.asarray(d, dtype=np.float64)
    rng = np.random.default_rng(seed)
    h, w = d.shape[-2:]
    dark = dark_level * (1.0 + 0.05 * rng.standard_normal((h, w)))
    flat = flat_level * (1.0 + 0.05 * rng.standard_normal((h, w)))
    ideal = np.exp(-d) * (flat - dark) + dark
    noisy = ideal + np.sqrt(np.maximum(ideal, 0.0)) * rng.standard_normal(d.shape)
    top = np.iinfo(dtype).max
    raw = np.clip(np.rint(noisy), 0, top).astype(dtype)
    return raw, dark.astype(np.float32), flat.astype(np.float32)
