"""C-ABI checks that need no GPU: exports, host-side plan logic, index logic."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from oracle.geometry import Geometry
from paper_2401_11101_amd import _abi, build as _build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lamino.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH) or not os.path.exists(_build.SELFTEST):
        _build.build()
    return _abi.load_library()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lamino_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "lamino_plan" in names and "lamino_fbp" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_abi.EXPORTED) == names


def _geom(nz=16, n=20, n_theta=12, h=14, w=18, tilt=0.5):
    g = _abi.lamino_geom()
    g.nz, g.n, g.n_theta, g.h, g.w, g.tilt = nz, n, n_theta, h, w, tilt
    return g


def _plan_status(geom, opts=None):
    o = opts if opts is not None else _abi.lamino_opts_default()
    h = ctypes.c_void_p()
    st = _abi.load_library().lamino_plan(ctypes.byref(geom), ctypes.byref(o), ctypes.byref(h))
    if st == 0:
        _abi.lamino_plan_destroy(h)
    return st


def test_plan_sizes_match_conventions(lib):
    for (nz, n, nt, h, w) in [(16, 20, 12, 14, 18), (64, 64, 64, 64, 64), (256, 256, 720, 256, 320)]:
        plan = _abi.lamino_plan(_geom(nz, n, nt, h, w), _abi.lamino_opts_default())
        info = _abi.lamino_plan_info(plan)
        g = Geometry(nz=nz, n=n, n_theta=nt, h=h, w=w, phi=0.5)
        assert (info.h_p, info.w_p) == (g.h_p, g.w_p)
        assert info.n_slab == g.h_p // 2
        assert info.grid >= 2 * n and info.grid & (info.grid - 1) == 0
        assert info.kernel_m == 5
        R = info.grid / n
        assert info.beta == pytest.approx(math.pi * (R - 0.5) / (R * info.kernel_m))
        t, wb = _abi.lamino_plan_sizes(plan)
        assert t == info.table_bytes and wb == info.work_bytes and t % 256 == 0
        assert info.spectra_scale == 1.0
        _abi.lamino_plan_destroy(plan)


def test_float16_spectra_carry_a_power_of_two_scale(lib):
    for dt, want in [(_abi.LAMINO_F16, lambda hp, wp: hp * wp / 64), (_abi.LAMINO_BF16, lambda hp, wp: 1.0)]:
        o = _abi.lamino_opts_default()
        o.storage_dtype = dt
        plan = _abi.lamino_plan(_geom(32, 32, 20, 24, 40), o)
        info = _abi.lamino_plan_info(plan)
        s = info.spectra_scale
        assert s == want(info.h_p, info.w_p)
        assert math.frexp(s)[0] == 0.5  # an exact power of two
        _abi.lamino_plan_destroy(plan)


def test_plan_rejects_bad_geometry(lib):
    assert _plan_status(_geom(nz=0)) == _abi.LAMINO_E_INVALID
    assert _plan_status(_geom(n_theta=-3)) == _abi.LAMINO_E_INVALID
    assert _plan_status(_geom(tilt=math.pi / 2)) == _abi.LAMINO_E_INVALID
    assert _plan_status(_geom(tilt=float("nan"))) == _abi.LAMINO_E_INVALID
    assert _plan_status(_geom(w=5000)) == _abi.LAMINO_E_UNSUPPORTED
    assert _plan_status(_geom(n=5000)) == _abi.LAMINO_E_UNSUPPORTED
    o = _abi.lamino_opts_default()
    o.kernel_m = 1
    assert _plan_status(_geom(), o) == _abi.LAMINO_E_INVALID
    o = _abi.lamino_opts_default()
    o.storage_dtype = 7
    assert _plan_status(_geom(), o) == _abi.LAMINO_E_INVALID
    o = _abi.lamino_opts_default()
    o.hbm_budget = 1000
    assert _plan_status(_geom(), o) == _abi.LAMINO_E_BUDGET
    assert "budget" in _abi.lamino_last_error()
    assert _abi.lamino_strerror(_abi.LAMINO_E_BUDGET)


def test_budget_shrinks_chunks(lib):
    o = _abi.lamino_opts_default()
    full = _abi.lamino_plan(_geom(64, 128, 100, 64, 128), o)
    fi = _abi.lamino_plan_info(full)
    o.hbm_budget = fi.work_bytes - 1
    small = _abi.lamino_plan(_geom(64, 128, 100, 64, 128), o)
    si = _abi.lamino_plan_info(small)
    assert si.work_bytes <= o.hbm_budget
    assert si.slab_chunk < fi.slab_chunk or si.theta_chunk < fi.theta_chunk
    _abi.lamino_plan_destroy(full)
    _abi.lamino_plan_destroy(small)


def test_calls_before_bind_fail_cleanly(lib):
    plan = _abi.lamino_plan(_geom(), _abi.lamino_opts_default())
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fbp(plan, ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert e.value.code == _abi.LAMINO_E_UNBOUND
    _abi.lamino_plan_destroy(plan)


def test_host_index_logic_selftest(lib):
    out = subprocess.run([_build.SELFTEST], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    for part in ("fft ok", "cand ok", "ring ok", "xcd ok", "div24 ok"):
        assert part in out.stdout, part


def _a256(x):
    return (x + 255) // 256 * 256


def test_admm_state_layout(lib):
    # lambda [3][nz][n][n] at 0, shift at the next 256-byte boundary, then
    # w, g, eta, t (volumes), q (data), per-block partials of the volume
    # and data reductions (1024 blocks) and scalars.
    for (nz, n, nt, h, w) in [(16, 20, 12, 14, 18), (256, 256, 720, 256, 320), (33, 65, 7, 9, 11)]:
        plan = _abi.lamino_plan(_geom(nz, n, nt, h, w), _abi.lamino_opts_default())
        nv = nz * n * n
        tiles = -(-n // 64) * -(-n // 4) * -(-nz // 16)
        blocks = 8 * -(-tiles // 8)
        want = (2 * _a256(3 * nv * 4) + 4 * _a256(nv * 4) + _a256(nt * h * w * 4)
                + _a256(blocks * 16) + 1024 * 16 + 256)
        assert _abi.lamino_admm_tv_state_bytes(plan) == want
        _abi.lamino_plan_destroy(plan)


def test_tv_calls_validate_arguments_on_the_host(lib):
    P = ctypes.c_void_p
    cases = [
        (lambda: _abi.lamino_tv_grad(P(None), P(256), 4, 4, 4, None), _abi.LAMINO_E_INVALID),
        (lambda: _abi.lamino_tv_grad(P(256), P(512), 0, 4, 4, None), _abi.LAMINO_E_INVALID),
        (lambda: _abi.lamino_tv_div(P(256), P(512), 4, -1, 4, None), _abi.LAMINO_E_INVALID),
        (lambda: _abi.lamino_tv_term(P(256), P(None), P(None), float("nan"), P(512), 4, 4, 4, None),
         _abi.LAMINO_E_INVALID),
        (lambda: _abi.lamino_tv_shrink(P(256), P(512), P(768), P(None), 0.1, 0.0, 4, 4, 4, None),
         _abi.LAMINO_E_INVALID),
        (lambda: _abi.lamino_tv_shrink(P(256), P(512), P(768), P(None), -0.1, 1.0, 4, 4, 4, None),
         _abi.LAMINO_E_INVALID),
        (lambda: _abi.lamino_tv_shrink(P(256), P(512), P(None), P(None), 0.1, 1.0, 4, 4, 4, None),
         _abi.LAMINO_E_INVALID),
        (lambda: _abi.lamino_tv_grad(P(256), P(512), 1 << 30, 1 << 20, 1 << 20, None),
         _abi.LAMINO_E_UNSUPPORTED),
    ]
    for call, code in cases:
        with pytest.raises(_abi.LaminoError) as e:
            call()
        assert e.value.code == code
    plan = _abi.lamino_plan(_geom(), _abi.lamino_opts_default())
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_admm_tv(plan, P(256), P(512), 0.1, 1.0, 1, 1, 0, P(768), None)
    assert e.value.code == _abi.LAMINO_E_UNBOUND
    _abi.lamino_plan_destroy(plan)


def test_new_entry_points_validate_on_the_host(lib):
    P = ctypes.c_void_p
    plan = _abi.lamino_plan(_geom(), _abi.lamino_opts_default())
    # every call on an unbound plan fails before touching the device
    for call in (lambda: _abi.lamino_fbp_raw(plan, P(256), P(512), P(768), 1e-6, P(1024), None),
                 lambda: _abi.lamino_fbp_slices(plan, P(256), 0.0, 0, 1, P(512), None),
                 lambda: _abi.lamino_direct_adj(plan, P(256), P(512), None),
                 lambda: _abi.lamino_direct_fbp(plan, P(256), P(512), P(768), None)):
        with pytest.raises(_abi.LaminoError) as e:
            call()
        assert e.value.code == _abi.LAMINO_E_UNBOUND
    # the direct workspace holds the filtered rows, n_theta h w float32
    assert _abi.lamino_direct_work_bytes(plan) == _a256(12 * 14 * 18 * 4)
    _abi.lamino_plan_destroy(plan)


def test_integer_data_types_are_accepted_for_input(lib):
    for dt in (_abi.LAMINO_U8, _abi.LAMINO_U16):
        o = _abi.lamino_opts_default()
        o.data_dtype = dt
        plan = _abi.lamino_plan(_geom(), o)
        _abi.lamino_plan_destroy(plan)
    o = _abi.lamino_opts_default()
    o.data_dtype = 5
    assert _plan_status(_geom(), o) == _abi.LAMINO_E_INVALID
    o = _abi.lamino_opts_default()
    o.storage_dtype = _abi.LAMINO_U8  # integer types are not storage types
    assert _plan_status(_geom(), o) == _abi.LAMINO_E_INVALID


def test_table_image_and_attach_on_the_host(lib):
    # the table image is the plan's double-precision tables: identical for two
    # plans of the same geometry, different for another tilt; attach checks
    # its buffers and marks the plan bound without any HIP call
    P = ctypes.c_void_p
    a = _abi.lamino_plan(_geom(tilt=0.4), _abi.lamino_opts_default())
    b = _abi.lamino_plan(_geom(tilt=0.4), _abi.lamino_opts_default())
    c = _abi.lamino_plan(_geom(tilt=0.5), _abi.lamino_opts_default())
    tb = _abi.lamino_plan_sizes(a)[0]
    bufs = [ctypes.create_string_buffer(tb) for _ in range(3)]
    for plan, buf in zip((a, b, c), bufs):
        _abi.lamino_plan_table_image(plan, ctypes.cast(buf, P), tb)
    assert bufs[0].raw == bufs[1].raw and bufs[0].raw != bufs[2].raw
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_plan_table_image(a, ctypes.cast(bufs[0], P), tb - 1)
    assert e.value.code == _abi.LAMINO_E_INVALID
    for args in ((P(None), P(512)), (P(256), P(None)), (P(256), P(520))):
        with pytest.raises(_abi.LaminoError) as e:
            _abi.lamino_plan_attach(a, *args)
        assert e.value.code == _abi.LAMINO_E_INVALID
    # attached (not uploaded): a call now passes the host checks; only the
    # NULL data pointer is refused, before anything is enqueued
    _abi.lamino_plan_attach(a, P(256), P(512))
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fbp(a, P(None), P(768), None)
    assert e.value.code == _abi.LAMINO_E_INVALID
    for plan in (a, b, c):
        _abi.lamino_plan_destroy(plan)


def test_noalloc_fbp_validates_on_the_host(lib):
    # lamino_fbp_noalloc refuses NULL arguments and plans whose tables and
    # workspace exceed the library's scratch array before any HIP call
    P = ctypes.c_void_p
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fbp_noalloc(P(None), P(256), P(512), None)
    assert e.value.code == _abi.LAMINO_E_INVALID
    big = _abi.lamino_plan(_geom(256, 256, 400, 256, 256), _abi.lamino_opts_default())
    info = _abi.lamino_plan_info(big)
    assert info.work_bytes > _abi.LAMINO_SCRATCH_BYTES
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fbp_noalloc(big, P(256), P(512), None)
    assert e.value.code == _abi.LAMINO_E_BUDGET
    assert "scratch" in _abi.lamino_last_error()
    small = _abi.lamino_plan(_geom(), _abi.lamino_opts_default())
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fbp_noalloc(small, P(None), P(512), None)
    assert e.value.code == _abi.LAMINO_E_INVALID
    for plan in (big, small):
        _abi.lamino_plan_destroy(plan)
    text = open(HEADER).read()
    assert f"#define LAMINO_SCRATCH_BYTES (64u << 20)" in text
    assert _abi.LAMINO_SCRATCH_BYTES == 64 << 20


def test_out_of_core_plan_layout_and_host_checks(lib):
    # a budget below the device-resident workspace keeps g, then also D, in
    # host memory; calls check the host buffer and refuse the operations that
    # need the intermediates on the device, all before any HIP call
    P = ctypes.c_void_p
    shape = (24, 40, 50, 24, 40)
    ref = _abi.lamino_plan(_geom(*shape), _abi.lamino_opts_default())
    ri = _abi.lamino_plan_info(ref)
    assert (ri.spill_spectra, ri.spill_slabs, ri.host_bytes) == (0, 0, 0)
    o = _abi.lamino_opts_default()
    o.hbm_budget = ri.bytes_spectra // 2
    plan = _abi.lamino_plan(_geom(*shape), o)
    pi = _abi.lamino_plan_info(plan)
    assert (pi.spill_spectra, pi.spill_slabs) == (1, 1)
    assert pi.work_bytes <= o.hbm_budget
    assert pi.host_bytes == _a256(ri.bytes_spectra) + _a256(ri.bytes_slabs)
    hb, io = _abi.lamino_plan_host_sizes(plan)
    assert (hb, io) == (pi.host_bytes, pi.io_bytes) and io > 0
    _abi.lamino_plan_attach(plan, P(256), P(512))
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fbp(plan, P(256), P(512), None)
    assert e.value.code == _abi.LAMINO_E_UNBOUND
    for bad in (P(None), P(1000)):
        with pytest.raises(_abi.LaminoError) as e:
            _abi.lamino_plan_bind_host(plan, bad)
        assert e.value.code == _abi.LAMINO_E_INVALID
    host = ctypes.create_string_buffer(hb + 256)
    addr = ctypes.addressof(host)
    _abi.lamino_plan_bind_host(plan, P(addr + (-addr) % 256))
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fwd(plan, P(256), P(512), None)
    assert e.value.code == _abi.LAMINO_E_UNSUPPORTED
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_admm_tv(plan, P(256), P(512), 0.1, 1.0, 1, 1, 0, P(768), None)
    assert e.value.code == _abi.LAMINO_E_UNSUPPORTED
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fbp_noalloc(plan, P(256), P(512), None)
    assert e.value.code == _abi.LAMINO_E_UNSUPPORTED
    with pytest.raises(_abi.LaminoError) as e:
        _abi.lamino_fbp_host(plan, P(256), P(512), P(None), None)
    assert e.value.code == _abi.LAMINO_E_INVALID
    for h in (ref, plan):
        _abi.lamino_plan_destroy(h)
