"""Plan: torch-owned device buffers around one C-ABI plan.

PyTorch provides device memory and the stream; every step of the
operators runs in the library's HIP kernels.
"""
import ctypes

import numpy as np
import torch

from . import _abi

_DTYPES = {"f32": (_abi.LAMINO_F32, torch.float32), "f16": (_abi.LAMINO_F16, torch.float16),
           "bf16": (_abi.LAMINO_BF16, torch.bfloat16), "u8": (_abi.LAMINO_U8, torch.uint8),
           "u16": (_abi.LAMINO_U16, torch.uint16)}
_FILTERS = {"ramp": _abi.LAMINO_RAMP, "shepp-logan": _abi.LAMINO_SHEPP_LOGAN,
            "parzen": _abi.LAMINO_PARZEN}


def _stream_handle(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """Laminography operators for one geometry.

    Volumes are float32 tensors (nz, n, n); data are (n_theta, h, w)
    tensors of `data_dtype`.  Calls are asynchronous on the given stream
    (default: torch's current stream).  One plan serves one call at a time.
    """

    def __init__(self, nz, n, n_theta, h, w, tilt, theta=None, data_dtype="f32",
                 storage_dtype="f32", filter="shepp-logan", pad_u=2.0, pad_v=2.0, kernel_m=0,
                 z_chunk=0, slab_chunk=0, theta_chunk=0, hbm_budget=0, device=None, stream=None,
                 work=None):
        self.shape_vol = (nz, n, n)
        self.shape_data = (n_theta, h, w)
        self.data_dtype = data_dtype
        self.storage_dtype = storage_dtype
        self.torch_data_dtype = _DTYPES[data_dtype][1]
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._theta = None
        g = _abi.lamino_geom()
        g.nz, g.n, g.n_theta, g.h, g.w = nz, n, n_theta, h, w
        g.tilt = float(tilt)
        if theta is not None:
            self._theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
            if self._theta.shape != (n_theta,):
                raise ValueError("theta must have n_theta entries")
            g.theta = self._theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o = _abi.lamino_opts_default()
        o.data_dtype = _DTYPES[data_dtype][0]
        o.storage_dtype = _DTYPES[storage_dtype][0]
        o.filter = _FILTERS[filter]
        o.pad_u, o.pad_v = float(pad_u), float(pad_v)
        o.kernel_m = int(kernel_m)
        o.z_chunk, o.slab_chunk, o.theta_chunk = int(z_chunk), int(slab_chunk), int(theta_chunk)
        o.hbm_budget = int(hbm_budget)
        self._h = None
        self._h = _abi.lamino_plan(g, o)
        self.info = _abi.lamino_plan_info(self._h)
        tb, wb = _abi.lamino_plan_sizes(self._h)
        with torch.cuda.device(self.device):
            self.tables = torch.empty(max(tb, 256), dtype=torch.uint8, device=self.device)
            if work is None:
                work = torch.empty(max(wb, 256), dtype=torch.uint8, device=self.device)
            elif work.dtype != torch.uint8 or work.numel() < wb or work.device != self.device:
                raise ValueError(f"work must be a uint8 tensor of at least {wb} bytes on {self.device}")
            # plans of one shape may share a workspace when their calls do not overlap
            self.work = work
            _abi.lamino_plan_bind(self._h, ctypes.c_void_p(self.tables.data_ptr()),
                                  ctypes.c_void_p(self.work.data_ptr()), _stream_handle(stream))
        # out-of-core plan (workspace above hbm_budget): the spectra and / or
        # slab planes live in pinned host memory owned here
        self.host_spill = None
        host_bytes, _ = _abi.lamino_plan_host_sizes(self._h)
        if host_bytes:
            self.host_spill = torch.empty(host_bytes + 256, dtype=torch.uint8, pin_memory=True)
            off = (-self.host_spill.data_ptr()) % 256
            _abi.lamino_plan_bind_host(self._h, ctypes.c_void_p(self.host_spill.data_ptr() + off))
        self._io = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _abi is not None and _abi.lamino_plan_destroy is not None:
            try:
                _abi.lamino_plan_destroy(h)
            except Exception:  # interpreter shutdown: module state may be gone
                pass
            self._h = None

    # ---------------------------------------------------------------- checks
    def _check(self, t, shape, dtype, name):
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if tuple(t.shape) != shape or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {shape}, "
                             f"got {tuple(t.shape)} {t.dtype}")

    # ------------------------------------------------------------- operators
    def fbp(self, data, out=None, stream=None):
        """Filtered backprojection W L* d (float32 volume)."""
        self._check(data, self.shape_data, self.torch_data_dtype, "data")
        out = torch.empty(self.shape_vol, dtype=torch.float32, device=self.device) if out is None else out
        self._check(out, self.shape_vol, torch.float32, "out")
        _abi.lamino_fbp(self._h, ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                        _stream_handle(stream))
        return out

    def fbp_host(self, data, out=None, stream=None):
        """FBP with the data and the volume in (pinned) host memory: chunks
        stream through a device staging buffer while the kernels run.  The
        volume is complete when the stream has finished."""
        if not isinstance(data, torch.Tensor) or data.device.type != "cpu":
            raise ValueError("data must be a host tensor")
        if tuple(data.shape) != self.shape_data or data.dtype != self.torch_data_dtype or \
                not data.is_contiguous():
            raise ValueError(f"data must be a contiguous {self.torch_data_dtype} host tensor of "
                             f"shape {self.shape_data}")
        if out is None:
            out = torch.empty(self.shape_vol, dtype=torch.float32, pin_memory=True)
        elif out.device.type != "cpu" or tuple(out.shape) != self.shape_vol or \
                out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float32 host tensor of shape {self.shape_vol}")
        if self._io is None:
            _, io_bytes = _abi.lamino_plan_host_sizes(self._h)
            self._io = torch.empty(max(io_bytes, 256), dtype=torch.uint8, device=self.device)
        _abi.lamino_fbp_host(self._h, ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(self._io.data_ptr()), _stream_handle(stream))
        return out

    def fbp_raw(self, raw, dark, flat, min_ratio=1e-6, out=None, stream=None):
        """FBP of raw detector counts: -log of the dark/flat-corrected ratio
        (clamped below at min_ratio) is taken inside the first kernel."""
        self._check(raw, self.shape_data, self.torch_data_dtype, "raw")
        field = self.shape_data[1:]
        self._check(dark, field, torch.float32, "dark")
        self._check(flat, field, torch.float32, "flat")
        out = torch.empty(self.shape_vol, dtype=torch.float32, device=self.device) if out is None else out
        self._check(out, self.shape_vol, torch.float32, "out")
        _abi.lamino_fbp_raw(self._h, ctypes.c_void_p(raw.data_ptr()), ctypes.c_void_p(dark.data_ptr()),
                            ctypes.c_void_p(flat.data_ptr()), min_ratio, ctypes.c_void_p(out.data_ptr()),
                            _stream_handle(stream))
        return out

    def fbp_slices(self, data, center_shift=0.0, z_first=0, z_count=None, out=None, stream=None):
        """Slices z_first .. z_first + z_count - 1 of the FBP with the rotation
        axis at detector column w/2 + center_shift."""
        self._check(data, self.shape_data, self.torch_data_dtype, "data")
        z_count = self.shape_vol[0] - z_first if z_count is None else z_count
        shape = (z_count,) + self.shape_vol[1:]
        out = torch.empty(shape, dtype=torch.float32, device=self.device) if out is None else out
        self._check(out, shape, torch.float32, "out")
        _abi.lamino_fbp_slices(self._h, ctypes.c_void_p(data.data_ptr()), center_shift, z_first, z_count,
                               ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
        return out

    def adj(self, data, out=None, stream=None):
        """Adjoint L* d (float32 volume)."""
        self._check(data, self.shape_data, self.torch_data_dtype, "data")
        out = torch.empty(self.shape_vol, dtype=torch.float32, device=self.device) if out is None else out
        self._check(out, self.shape_vol, torch.float32, "out")
        _abi.lamino_adj(self._h, ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                        _stream_handle(stream))
        return out

    def fwd(self, vol, out=None, stream=None):
        """Forward projection L vol (data in data_dtype)."""
        self._check(vol, self.shape_vol, torch.float32, "vol")
        out = torch.empty(self.shape_data, dtype=self.torch_data_dtype, device=self.device) if out is None else out
        self._check(out, self.shape_data, self.torch_data_dtype, "out")
        _abi.lamino_fwd(self._h, ctypes.c_void_p(vol.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                        _stream_handle(stream))
        return out

    def direct_fbp(self, data, out=None, stream=None):
        """FBP by the direct line-integral discretisation (O(N^3 n_theta)):
        rows filtered with the same W(m), then bilinear backprojection."""
        self._check(data, self.shape_data, self.torch_data_dtype, "data")
        out = torch.empty(self.shape_vol, dtype=torch.float32, device=self.device) if out is None else out
        self._check(out, self.shape_vol, torch.float32, "out")
        if getattr(self, "_direct_work", None) is None:
            nbytes = _abi.lamino_direct_work_bytes(self._h)
            self._direct_work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        _abi.lamino_direct_fbp(self._h, ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(self._direct_work.data_ptr()), _stream_handle(stream))
        return out

    def direct_adj(self, data, out=None, stream=None):
        """Direct bilinear backprojection L*_dir d (no filter)."""
        self._check(data, self.shape_data, self.torch_data_dtype, "data")
        out = torch.empty(self.shape_vol, dtype=torch.float32, device=self.device) if out is None else out
        self._check(out, self.shape_vol, torch.float32, "out")
        _abi.lamino_direct_adj(self._h, ctypes.c_void_p(data.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               _stream_handle(stream))
        return out

    def profile(self, enable=True):
        """Record per-stage HIP events on the call stream for later calls."""
        _abi.lamino_plan_profile(self._h, enable)

    def stage_times(self, reset=False):
        """{stage: (ms, launches)} accumulated while profiling was on."""
        return _abi.lamino_plan_stage_times(self._h, reset)

    def spectra(self):
        """Stored spectra D[l][theta][k] after an FBP call (complex), with the
        storage scale (info.spectra_scale) divided out.  With float16 storage
        they also carry the call's power-of-two input factor."""
        i = self.info
        raw = self.work[i.off_spectra:i.off_spectra + i.bytes_spectra]
        n_theta, h, w = self.shape_data
        if self.storage_dtype == "f32":
            v = raw.view(torch.float32).view(i.n_slab, n_theta, i.w_p, 2)
        else:
            v = raw.view(_DTYPES[self.storage_dtype][1]).view(i.n_slab, n_theta, i.w_p, 2).float()
        return torch.view_as_complex(v.contiguous()) / i.spectra_scale
