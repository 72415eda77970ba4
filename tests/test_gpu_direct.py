"""Direct line-integral backprojection (L*_dir, FBP_dir) on the GPU against
oracle O1 (direct.c, FP64 voxel-driven bilinear pair)."""
import numpy as np
import pytest
import torch

import synth
from helpers import dev, ellipsoid_data, to_dev, to_np
from oracle import direct, filters
from oracle.geometry import Geometry
from paper_2401_11101_amd import Plan

pytestmark = pytest.mark.gpu

# Element-wise bar relative to the largest reference value: float32 sums of
# n_theta bilinear taps (coordinates formed in float64) and, for FBP, a
# float32 row FFT of length w_p.
TOL_DIR = 2e-6
TOL_DIR_FBP = 1e-5


def _maxrel(a, b):
    b = np.asarray(b, np.float64)
    return float(np.abs(np.asarray(a, np.float64) - b).max() / np.abs(b).max())


CASES = [
    # nz, n, n_theta, h, w, tilt (deg)
    (20, 24, 30, 20, 28, 30.0),
    (17, 33, 13, 19, 37, 25.0),
    (16, 64, 40, 16, 70, 0.0),
    (33, 20, 21, 40, 24, -40.0),
]


@pytest.mark.parametrize("case", CASES)
def test_direct_adjoint_matches_oracle(case):
    nz, n, nt, h, w, tilt = case
    print(f"direct adj {case}", flush=True)
    g, _, d = ellipsoid_data(8, nz, n, nt, h, w, np.deg2rad(tilt), 0.01, seed=3)
    d32 = d.astype(np.float32)
    plan = Plan(nz, n, nt, h, w, np.deg2rad(tilt))
    out = to_np(plan.direct_adj(to_dev(d32)))
    ref = direct.adjoint(d32.astype(np.float64), g)
    e = _maxrel(out, ref)
    print(f"  max rel {e:.2e}")
    assert e < TOL_DIR


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("filt", ["shepp-logan", "ramp"])
def test_direct_fbp_matches_oracle(case, filt):
    nz, n, nt, h, w, tilt = case
    print(f"direct fbp {case} {filt}", flush=True)
    g, _, d = ellipsoid_data(8, nz, n, nt, h, w, np.deg2rad(tilt), 0.01, seed=4)
    d32 = d.astype(np.float32)
    plan = Plan(nz, n, nt, h, w, np.deg2rad(tilt), filter=filt)
    out = to_np(plan.direct_fbp(to_dev(d32)))
    kind = {"shepp-logan": filters.SHEPP_LOGAN, "ramp": filters.RAMP}[filt]
    ref = direct.fbp(d32.astype(np.float64), g, kind=kind)
    e = _maxrel(out, ref)
    print(f"  max rel {e:.2e}")
    assert e < TOL_DIR_FBP


def test_direct_nonuniform_angles_and_narrow_data_types():
    nz, n, nt, h, w, tilt = 12, 40, 17, 14, 44, 20.0
    theta = np.sort(np.random.default_rng(5).uniform(0, 2 * np.pi, nt))
    g = Geometry(nz=nz, n=n, n_theta=nt, h=h, w=w, phi=np.deg2rad(tilt), theta=theta)
    rng = np.random.default_rng(6)
    counts = rng.integers(0, 256, (nt, h, w)).astype(np.uint8)
    ref = direct.adjoint(counts.astype(np.float64), g)
    for dt, torch_dt in [("u8", torch.uint8), ("f16", torch.float16), ("bf16", torch.bfloat16)]:
        plan = Plan(nz, n, nt, h, w, np.deg2rad(tilt), theta=theta, data_dtype=dt)
        # 0..255 integers are exact in every one of these types
        out = to_np(plan.direct_adj(torch.from_numpy(counts).to(dev()).to(torch_dt)))
        e = _maxrel(out, ref)
        print(f"  {dt}: max rel {e:.2e}")
        assert e < TOL_DIR
    plan = Plan(nz, n, nt, h, w, np.deg2rad(tilt), theta=theta, data_dtype="u16")
    out = to_np(plan.direct_adj(torch.from_numpy(counts.astype(np.uint16)).to(dev())))
    assert _maxrel(out, ref) < TOL_DIR
    plan = Plan(nz, n, nt, h, w, np.deg2rad(tilt), theta=theta, data_dtype="u8")
    out = to_np(plan.direct_fbp(torch.from_numpy(counts).to(dev())))
    assert _maxrel(out, direct.fbp(counts.astype(np.float64), g)) < TOL_DIR_FBP


def test_direct_fbp_full_size_sampled_slices():
    # the 256^3 / 400-projection / 256 x 256 workload at tilt 25 deg: whole
    # FBP_dir on the GPU, three z slices from the oracle
    nz = n = h = w = 256
    nt = 400
    tilt = np.deg2rad(25.0)
    print("direct fbp 256^3 sampled slices", flush=True)
    ells = synth.random_ellipsoids(50, nz, n, seed=0)
    d = synth.project_ellipsoids(ells, nt, h, w, tilt, device=dev(), dtype=torch.float64)
    d = synth.add_noise(d, 0.005, seed=1).float().contiguous()
    plan = Plan(nz, n, nt, h, w, tilt)
    vol = to_np(plan.direct_fbp(d))
    g = Geometry(nz=nz, n=n, n_theta=nt, h=h, w=w, phi=tilt)
    dn = to_np(d)
    for z0 in (0, 128, 255):
        ref = direct.fbp(dn, g, z_range=(z0, z0 + 1))[0]
        e = _maxrel(vol[z0], ref)
        print(f"  slice {z0}: max rel {e:.2e}")
        assert e < TOL_DIR_FBP


def test_direct_adjoint_table_scale_sampled_slice():
    # N = 1024: 1024 projections of 1024 x 1024, tilt 20 deg, 8-bit data
    # (the scale of the paper's timing table); one slice from the oracle
    N = 1024
    tilt = np.deg2rad(20.0)
    print("direct adj N=1024 sampled slice", flush=True)
    ells = synth.random_ellipsoids(20, N, N, seed=2)
    d = synth.project_ellipsoids(ells, N, N, N, tilt, device=dev(), dtype=torch.float32, theta_chunk=16)
    d8 = torch.clamp(d * (255.0 / float(d.max())), 0, 255).round().to(torch.uint8)
    del d
    plan = Plan(N, N, N, N, N, tilt, data_dtype="u8")
    vol = plan.direct_adj(d8)
    torch.cuda.synchronize()
    g = Geometry(nz=N, n=N, n_theta=N, h=N, w=N, phi=tilt)
    z0 = 600
    ref = direct.adjoint(d8.cpu().numpy().astype(np.float64), g, z_range=(z0, z0 + 1))[0]
    e = _maxrel(to_np(vol[z0]), ref)
    print(f"  slice {z0}: max rel {e:.2e}")
    assert e < 1e-5


def test_fourier_fbp_accepts_8bit_data_and_rejects_8bit_forward():
    nz, n, nt, h, w = 16, 24, 20, 16, 28
    rng = np.random.default_rng(7)
    counts = rng.integers(0, 256, (nt, h, w)).astype(np.uint8)
    p8 = Plan(nz, n, nt, h, w, np.deg2rad(30), data_dtype="u8")
    p32 = Plan(nz, n, nt, h, w, np.deg2rad(30))
    a = to_np(p8.fbp(torch.from_numpy(counts).to(dev())))
    b = to_np(p32.fbp(torch.from_numpy(counts.astype(np.float32)).to(dev())))
    assert np.array_equal(a, b)  # the same float values enter the same kernels
    from paper_2401_11101_amd import _abi
    with pytest.raises(_abi.LaminoError) as e:
        p8.fwd(torch.zeros(p8.shape_vol, device=dev()), out=torch.empty(p8.shape_data, dtype=torch.uint8,
                                                                          device=dev()))
    assert e.value.code == _abi.LAMINO_E_INVALID


def test_fourier_fbp_against_direct_fbp_triangle():
    # The 64^3 configuration (64 angles on [0, 2 pi), tilt 30 deg, detector
    # 64 x 64, 20 ellipsoids, 1% noise, Shepp-Logan).  The Fourier-route FBP
    # and the direct (bilinear) FBP are two discretisations of eq:recon; their
    # gap is a property of the discretisations, measured oracle against
    # oracle: g_O = |O2 - O1| / |O1| (O2 the exact Fourier sums, O1 the
    # direct FBP).  The GPU's Fourier FBP must show the same gap to the
    # direct FBP within its own distance to O2 (triangle inequality), and the
    # GPU's direct FBP must match O1.
    from oracle import nudft

    print("Fourier vs direct FBP, 64^3 configuration", flush=True)
    g, _, d = ellipsoid_data(20, 64, 64, 64, 64, 64, np.deg2rad(30), 0.01)
    d32 = d.astype(np.float32)
    d64 = d32.astype(np.float64)
    plan = Plan(64, 64, 64, 64, 64, g.phi)
    four = to_np(plan.fbp(to_dev(d32)))
    dirg = to_np(plan.direct_fbp(to_dev(d32)))
    o2 = nudft.fbp(d64, g, filters.SHEPP_LOGAN)
    o1 = direct.fbp(d64, g, filters.SHEPP_LOGAN)
    n1 = np.linalg.norm(o1)
    gap_oracle = np.linalg.norm(o2 - o1) / n1
    gap_gpu = np.linalg.norm(four - dirg) / np.linalg.norm(dirg)
    gap_gpu_o1 = np.linalg.norm(four - o1) / n1
    d_four = np.linalg.norm(four - o2) / n1
    d_dir = np.linalg.norm(dirg - o1) / n1
    print(f"  |O2 - O1|/|O1| {gap_oracle:.4e}; |GPU Fourier - GPU direct|/|GPU direct| {gap_gpu:.4e}; "
          f"|GPU Fourier - O1|/|O1| {gap_gpu_o1:.4e}")
    print(f"  |GPU Fourier - O2|/|O1| {d_four:.2e}; |GPU direct - O1|/|O1| {d_dir:.2e}")
    assert d_four < 1e-4 * np.linalg.norm(o2) / n1
    assert d_dir < TOL_DIR_FBP
    assert abs(gap_gpu_o1 - gap_oracle) <= d_four * (1 + 1e-9)
    assert abs(gap_gpu - gap_oracle) <= d_four + 2 * d_dir + 1e-12
