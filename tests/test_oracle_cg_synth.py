"""Pins of O4 (conjugate gradients) and of the synthetic input generator."""
import numpy as np
import pytest
import torch

import synth
from oracle import cg, nudft, phantom
from oracle.geometry import Geometry, centred


def test_cg_variants_agree_and_reach_lstsq():
    # Appendix A's CG (Dai-Yuan, exact line search) and textbook CGLS give
    # the same iterates on a quadratic; both reach numpy's least squares.
    rng = np.random.default_rng(0)
    A = rng.standard_normal((60, 25)) + 3 * np.eye(60, 25)
    b = rng.standard_normal(60)
    L = lambda x: A @ x
    Lt = lambda y: A.T @ y
    x0 = np.zeros(25)
    it_dy, it_cg = [], []
    cg.cg_daiyuan(L, Lt, b, x0, 10, callback=lambda k, x: it_dy.append(x.copy()))
    cg.cgls(L, Lt, b, x0, 10, callback=lambda k, x: it_cg.append(x.copy()))
    for a, c in zip(it_dy, it_cg):
        assert np.linalg.norm(a - c) <= 1e-9 * np.linalg.norm(c)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    x = cg.cgls(L, Lt, b, x0, 40)
    assert np.linalg.norm(x - xs) < 1e-10 * np.linalg.norm(xs)
    x = cg.cg_daiyuan(L, Lt, b, x0, 40)
    assert np.linalg.norm(x - xs) < 1e-8 * np.linalg.norm(xs)


def test_cg_on_laminography_residual_decreases():
    g = Geometry(nz=8, n=8, n_theta=12, h=8, w=8, phi=np.deg2rad(30))
    f = np.random.default_rng(1).standard_normal((g.nz, g.n, g.n))
    d = nudft.forward(f, g)
    res = []
    cg.cgls(lambda x: nudft.forward(x, g), lambda y: nudft.adjoint(y, g), d,
            np.zeros_like(f), 8,
            callback=lambda k, x: res.append(np.linalg.norm(nudft.forward(x, g) - d)))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res, res[1:]))
    assert res[-1] < 0.25 * res[0]


def test_synth_projections_match_oracle_closed_form():
    ells = synth.random_ellipsoids(5, 16, 20, seed=0)
    th = synth.angles(6)
    phi = np.deg2rad(25)
    d = synth.project_ellipsoids(ells, 6, 16, 20, phi).numpy()
    objs = [phantom.Ellipsoid(c, a, r, p) for c, a, r, p in zip(*ells)]
    ref = phantom.ellipsoid_projections(objs, th, phi, centred(20), centred(16))
    assert np.abs(d - ref).max() < 1e-10 * np.abs(ref).max()


def test_synth_voxels_match_oracle_indicator():
    ells = synth.random_ellipsoids(4, 10, 12, seed=3)
    vol = synth.voxelize_ellipsoids(ells, 10, 12).numpy()
    objs = [phantom.Ellipsoid(c, a, r, p) for c, a, r, p in zip(*ells)]
    x = centred(12)
    z = centred(10)
    Z, Y, X = np.meshgrid(z, x, x, indexing="ij")
    ref = phantom.ellipsoid_indicator(objs, np.stack([X, Y, Z], -1))
    assert np.array_equal(vol, ref)


def test_synth_is_seeded():
    a = synth.random_ellipsoids(3, 8, 8, seed=7)
    b = synth.random_ellipsoids(3, 8, 8, seed=7)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    d = torch.ones(4, 5, 6, dtype=torch.float64)
    assert torch.equal(synth.add_noise(d, 0.01, seed=1), synth.add_noise(d, 0.01, seed=1))
    r = synth.random_ellipsoids(50, 64, 64, seed=0)[2]
    assert np.allclose(np.einsum("eij,ekj->eik", r, r), np.eye(3)[None], atol=1e-12)
