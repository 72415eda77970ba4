"""Out-of-core execution: intermediates and inputs / outputs in host memory.

A plan whose device workspace would exceed opts.hbm_budget keeps the slab
planes g, and then also the spectra D, in pinned host memory and streams
double-buffered chunks between host and device on separate streams (the
chunked host-device pipeline of Section "GPU acceleration of
reconstruction").  lamino_fbp_host streams the projections in and the
volume out in chunks.  Every such run must equal the device-resident run bit
for bit: the same kernels see the same values, only the buffers differ.
"""
import functools

import numpy as np
import pytest
import torch

import synth
from helpers import TOL_LOWP, dev, to_np
from paper_2401_11101_amd import Plan, _abi

pytestmark = pytest.mark.gpu

SHAPE = (24, 40, 50, 24, 40)  # nz, n, n_theta, h, w: 1600 columns, 24 frequency slabs
TILT = np.deg2rad(28.0)


def _plans(storage, data_dtype):
    kw = dict(storage_dtype=storage, data_dtype=data_dtype)
    ref = Plan(*SHAPE, TILT, **kw)
    i = ref.info
    # budget of D + g: the slab planes must leave the device; half of D: both
    g_only = Plan(*SHAPE, TILT, hbm_budget=i.bytes_spectra + i.bytes_slabs, **kw)
    both = Plan(*SHAPE, TILT, hbm_budget=i.bytes_spectra // 2, **kw)
    assert (i.spill_spectra, i.spill_slabs) == (0, 0)
    assert g_only.info.spill_slabs == 1 and g_only.info.work_bytes <= i.bytes_spectra + i.bytes_slabs
    assert (both.info.spill_spectra, both.info.spill_slabs) == (1, 1)
    assert both.info.work_bytes <= i.bytes_spectra // 2
    # several projection, slab and column chunks
    assert both.info.theta_chunk < SHAPE[2] and both.info.slab_chunk < i.n_slab
    assert both.info.col_chunk < SHAPE[1] ** 2
    return ref, g_only, both


def _data(data_dtype, seed=3):
    g = torch.Generator(device="cpu").manual_seed(seed)
    d = torch.randn((SHAPE[2], SHAPE[3], SHAPE[4]), generator=g)
    return d.to({"f32": torch.float32, "f16": torch.float16}[data_dtype])


@pytest.mark.parametrize("storage, data_dtype", [("f32", "f32"), ("f16", "f16"), ("bf16", "f32")])
def test_spilled_plans_equal_resident(storage, data_dtype):
    print(f"out of core {storage} storage, {data_dtype} data", flush=True)
    ref, g_only, both = _plans(storage, data_dtype)
    d = _data(data_dtype).to(dev())
    want_fbp, want_adj = ref.fbp(d), ref.adj(d)
    want_sl = ref.fbp_slices(d, center_shift=1.5, z_first=5, z_count=7)
    for plan in (g_only, both):
        got_fbp, got_adj = plan.fbp(d), plan.adj(d)
        got_sl = plan.fbp_slices(d, center_shift=1.5, z_first=5, z_count=7)
        torch.cuda.synchronize()
        print(f"  spill D {plan.info.spill_spectra} g {plan.info.spill_slabs}: chunks theta "
              f"{plan.info.theta_chunk} slab {plan.info.slab_chunk} columns {plan.info.col_chunk}")
        assert torch.equal(got_fbp, want_fbp)
        assert torch.equal(got_adj, want_adj)
        assert torch.equal(got_sl, want_sl)


@pytest.mark.parametrize("storage, data_dtype", [("f32", "f32"), ("f16", "f16")])
def test_host_input_and_output_equal_device(storage, data_dtype):
    # data and volume in pinned host memory, streamed in chunks; z-chunks of 5
    # slices for a resident plan, column chunks for the spilled ones
    print(f"host I/O {storage} storage", flush=True)
    ref, g_only, both = _plans(storage, data_dtype)
    d = _data(data_dtype, seed=4)
    want = to_np(ref.fbp(d.to(dev())))
    zc = Plan(*SHAPE, TILT, storage_dtype=storage, data_dtype=data_dtype, z_chunk=5)
    assert zc.info.io_z == 5
    hd = d.pin_memory()
    for plan in (zc, ref, g_only, both):
        out = plan.fbp_host(hd)
        torch.cuda.synchronize()
        assert out.device.type == "cpu"
        assert np.array_equal(out.double().numpy(), want), (plan.info.spill_spectra, plan.info.spill_slabs)


def test_repeated_out_of_core_calls_and_forward_refused():
    ref, _, both = _plans("f32", "f32")
    d = _data("f32", seed=5).to(dev())
    a = both.fbp(d)
    b = both.fbp(d)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, ref.fbp(d))
    vol = torch.zeros(both.shape_vol, device=dev())
    with pytest.raises(_abi.LaminoError) as e:
        both.fwd(vol)
    assert e.value.code == _abi.LAMINO_E_UNSUPPORTED


@functools.lru_cache(maxsize=1)
def _large():
    # the large-chunk configuration at full size: detector 1024 wide x 512
    # rows, 1500 projections, tilt 20 deg, volume 512 x 1024 x 1024, data
    # fp16-stored from an ellipsoid phantom with log-normal speckle 0.1
    nz, n, nt, h, w = 512, 1024, 1500, 512, 1024
    ells = synth.random_ellipsoids(20, nz, n, seed=0)
    d = synth.project_ellipsoids(ells, nt, h, w, np.deg2rad(20.0), device=dev(), dtype=torch.float32,
                                 theta_chunk=8)
    return (nz, n, nt, h, w), synth.apply_speckle(d, 0.1, seed=1).half().contiguous()


def test_large_volume_z_chunks_host_output_and_fp32():
    shape, d16 = _large()
    nz, n, nt, h, w = shape
    tilt = np.deg2rad(20.0)
    print("large volume: z-chunks of 64 vs whole, host output, fp16 vs fp32", flush=True)
    p64 = Plan(*shape, tilt, data_dtype="f16", storage_dtype="f16", z_chunk=64)
    v64 = p64.fbp(d16)
    whole = Plan(*shape, tilt, data_dtype="f16", storage_dtype="f16")
    vw = whole.fbp(d16)
    torch.cuda.synchronize()
    assert torch.equal(v64, vw)
    del whole
    # the volume leaves the device in chunks of 64 slices (pinned host memory)
    assert p64.info.io_z == 64
    hv = p64.fbp_host(d16.cpu().pin_memory())
    torch.cuda.synchronize()
    assert torch.equal(hv, v64.cpu())
    del p64, hv
    torch.cuda.empty_cache()
    p32 = Plan(*shape, tilt, data_dtype="f16", storage_dtype="f32", z_chunk=64)
    v32 = p32.fbp(d16)
    torch.cuda.synchronize()
    e = float((v64.double() - v32.double()).norm() / v32.double().norm())
    print(f"  fp16 storage vs fp32 storage: rel-L2 {e:.2e}")
    assert e < TOL_LOWP
    assert bool(torch.isfinite(v64).all())
