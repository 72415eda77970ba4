"""Rotation-axis offset, slice output and the axis / tilt sweeps on the GPU
against oracle O7 (exact Fourier sums)."""
import numpy as np
import pytest
import torch

import synth
from helpers import TOL_F32, dev, ellipsoid_data, rel, to_dev, to_np
from oracle import search as osearch
from paper_2401_11101_amd import Plan, search

pytestmark = pytest.mark.gpu

NZ, N, NT, H, W = 20, 24, 30, 20, 28
PHI = np.deg2rad(25)


def _data(seed=2):
    g, _, d = ellipsoid_data(10, NZ, N, NT, H, W, PHI, 0.01, seed=seed)
    return g, d.astype(np.float32)


def test_slices_without_offset_equal_the_fbp():
    g, d = _data()
    plan = Plan(NZ, N, NT, H, W, PHI)
    full = plan.fbp(to_dev(d))
    part = plan.fbp_slices(to_dev(d), 0.0, z_first=5, z_count=7)
    torch.cuda.synchronize()
    e = float((part - full[5:12]).abs().max() / full.abs().max())
    print(f"  slices vs fbp: max rel {e:.1e}")
    assert e < 1e-6
    allz = plan.fbp_slices(to_dev(d), 0.0)
    assert torch.equal(allz, full)


@pytest.mark.parametrize("shift", [0.5, -3.25, 6.0])
def test_axis_offset_matches_oracle(shift):
    print(f"axis offset {shift}", flush=True)
    g, d = _data()
    plan = Plan(NZ, N, NT, H, W, PHI)
    out = to_np(plan.fbp_slices(to_dev(d), shift))
    ref = osearch.fbp_shifted(d.astype(np.float64), g, shift)
    e = rel(out, ref)
    print(f"  rel-L2 {e:.2e}")
    assert e < TOL_F32


def test_center_and_tilt_sweeps_match_oracle():
    g, d = _data(3)
    shifts = [-1.5, 0.0, 2.25]
    plan = Plan(NZ, N, NT, H, W, PHI)
    cs = to_np(search.center_sweep(plan, to_dev(d), shifts, z=9))
    ref = osearch.center_sweep(d.astype(np.float64), g, shifts, 9)
    e = rel(cs, ref)
    print(f"  center sweep rel-L2 {e:.2e}")
    assert e < TOL_F32
    tilts = np.deg2rad([22.0, 25.0, 28.5])
    ts = to_np(search.tilt_sweep(NZ, N, NT, H, W, tilts, to_dev(d), z=9, center_shift=0.5))
    ref = osearch.tilt_sweep(d.astype(np.float64), g, tilts, 0.5, 9)
    e = rel(ts, ref)
    print(f"  tilt sweep rel-L2 {e:.2e}")
    assert e < TOL_F32


def test_full_size_integer_offset_equals_recentred_data():
    # 256^3 / 400 projections: data recorded with the axis 7 columns right of
    # centre (simulated by moving zero-margin columns) reconstruct, at the
    # right offset, to the slices of the centred data
    nz = n = h = w = 256
    nt = 400
    tilt = np.deg2rad(25.0)
    print("full-size axis offset", flush=True)
    ells = synth.random_ellipsoids(50, nz, n, seed=0)
    d = synth.project_ellipsoids(ells, nt, h, w, tilt, device=dev(), dtype=torch.float32)
    d[..., :12] = 0
    d[..., -12:] = 0
    delta = 7
    rec = torch.zeros_like(d)
    rec[..., delta:] = d[..., :-delta]  # column c of the recording is column c - delta of d
    plan = Plan(nz, n, nt, h, w, tilt)
    zs = [40, 128, 200]
    ref = plan.fbp(d.contiguous())
    for z in zs:
        a = plan.fbp_slices(rec, float(delta), z_first=z, z_count=1)[0]
        e = float((a - ref[z]).abs().max() / ref.abs().max())
        print(f"  slice {z}: max rel {e:.2e}")
        assert e < 1e-5
    sweep = search.center_sweep(plan, rec, [delta - 2.0, float(delta), delta + 2.0], z=128)
    err = [float((sweep[i] - ref[128]).norm() / ref[128].norm()) for i in range(3)]
    print("  sweep rel errors", err)
    assert err[1] < 1e-5 and min(err[0], err[2]) > 100 * err[1]


def test_slice_arguments_are_checked():
    from paper_2401_11101_amd import _abi
    _, d = _data()
    plan = Plan(NZ, N, NT, H, W, PHI)
    for kw in (dict(z_first=-1, z_count=1), dict(z_first=NZ - 2, z_count=3), dict(z_first=0, z_count=0)):
        with pytest.raises(Exception):
            plan.fbp_slices(to_dev(d), 0.0, out=torch.empty((max(kw["z_count"], 1), N, N), device=dev()),
                            **kw)
    room = (plan.info.w_p - W) / 2
    with pytest.raises(_abi.LaminoError):
        plan.fbp_slices(to_dev(d), room + 0.5)


def test_slices_with_chunked_plan_and_offset():
    # z chunks of 3, slab chunks of 2, theta chunks of 7: the slice range
    # starts inside a z chunk; the offset applies in every theta chunk
    g, d = _data(4)
    full = Plan(NZ, N, NT, H, W, PHI)
    chunked = Plan(NZ, N, NT, H, W, PHI, z_chunk=3, slab_chunk=2, theta_chunk=7)
    a = chunked.fbp_slices(to_dev(d), 1.75, z_first=4, z_count=9)
    b = full.fbp_slices(to_dev(d), 1.75)[4:13]
    torch.cuda.synchronize()
    e = float((a - b).abs().max() / b.abs().max())
    print(f"  chunked slices vs unchunked: max rel {e:.1e}")
    assert e < 1e-6
