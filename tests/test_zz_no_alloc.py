"""Allocation-free FBP (lamino_fbp_noalloc) against lamino_fbp, through the C ABI.

The entry point runs the same kernels with the plan's tables and workspace
in the library's device scratch array; its plans are never bound.  Two calls
in a row (the second with a smaller input) must each equal the bound entry
point's result, and the small one the exact FBP sums; a plan too large for
the array is refused on the host.
"""
import ctypes

import numpy as np
import pytest
import torch

from helpers import TOL_F32, TOL_LOWP, dev, rel, to_np
from oracle import filters, nudft
from oracle.geometry import Geometry
from paper_2401_11101_amd import Plan, _abi
from paper_2401_11101_amd.plan import _DTYPES

pytestmark = pytest.mark.gpu

P = ctypes.c_void_p


def _host_plan(nz, n, nt, h, w, tilt, storage="f32", data="f32", budget=0):
    g = _abi.lamino_geom()
    g.nz, g.n, g.n_theta, g.h, g.w, g.tilt = nz, n, nt, h, w, tilt
    o = _abi.lamino_opts_default()
    o.storage_dtype = _DTYPES[storage][0]
    o.data_dtype = _DTYPES[data][0]
    o.hbm_budget = budget
    return _abi.lamino_plan(g, o)


def _noalloc(h, data, shape_vol):
    out = torch.full(shape_vol, float("nan"), dtype=torch.float32, device=dev())
    stream = torch.cuda.current_stream()
    _abi.lamino_fbp_noalloc(h, P(data.data_ptr()), P(out.data_ptr()), P(stream.cuda_stream))
    return out


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_two_calls_match_the_bound_entry_point(storage):
    tilt = np.deg2rad(30.0)
    tdt = torch.float32 if storage == "f32" else torch.float16
    dtype = "f32" if storage == "f32" else "f16"
    shapes = [(64, 64, 64, 64, 64), (20, 24, 30, 16, 28)]  # the second call is smaller
    gen = torch.Generator(device="cpu").manual_seed(7)
    outs = []
    for shape in shapes:
        nz, n, nt, h, w = shape
        print(f"noalloc {storage} {shape}", flush=True)
        data = torch.randn((nt, h, w), generator=gen).to(tdt).to(dev())
        hp = _host_plan(*shape, tilt, storage=storage, data=dtype)
        info = _abi.lamino_plan_info(hp)
        assert info.table_bytes + info.work_bytes <= _abi.LAMINO_SCRATCH_BYTES
        got = _noalloc(hp, data, (nz, n, n))
        ref = Plan(*shape, tilt, storage_dtype=storage, data_dtype=dtype).fbp(data)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (shape, float((got - ref).abs().max()))
        outs.append((shape, data, got))
        _abi.lamino_plan_destroy(hp)
    # the smaller call against the exact FBP sums
    (nz, n, nt, h, w), data, got = outs[1]
    g = Geometry(nz=nz, n=n, n_theta=nt, h=h, w=w, phi=tilt)
    e = rel(to_np(got), nudft.fbp(to_np(data), g, filters.SHEPP_LOGAN))
    print(f"  small call vs exact FBP rel-L2 {e:.2e}")
    assert e < (TOL_F32 if storage == "f32" else TOL_LOWP)


def test_plan_above_the_scratch_limit_is_refused():
    hp = _host_plan(256, 256, 400, 256, 256, 0.4)
    data = torch.zeros((1,), device=dev())
    vol = torch.zeros((1,), device=dev())
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fbp_noalloc(hp, P(data.data_ptr()), P(vol.data_ptr()), None)
    assert e.value.code == _abi.LAMINO_E_BUDGET
    assert "scratch" in _abi.lamino_last_error()
    _abi.lamino_plan_destroy(hp)
    # the same geometry planned within the limit fits (smaller chunks)
    hp = _host_plan(64, 96, 60, 64, 96, 0.4, budget=_abi.LAMINO_SCRATCH_BYTES // 2)
    info = _abi.lamino_plan_info(hp)
    assert info.table_bytes + info.work_bytes <= _abi.LAMINO_SCRATCH_BYTES
    _abi.lamino_plan_destroy(hp)
