"""Total-variation regularised reconstruction (Appendix A) on the HIP library.

`admm_tv` minimises 1/2 ||L mu - d||^2 + alpha ||grad mu||_1 with the
ADMM of Appendix A: each outer iteration runs a few Dai-Yuan conjugate
gradient steps on the tomography sub-problem (Eq:tomo, Eq:gradtomo,
Eq:DaiYuan2), then the soft threshold (Eq:reg) and the dual update
(Eq:lamd).  The whole loop is enqueued by one library call
(`lamino_admm_tv`); its scalars stay on the device.

`grad`, `div`, `tv_term` and `shrink` expose the library's finite-difference
and thresholding kernels on their own.  Volumes are float32 (nz, ny, nx)
tensors; gradient fields are float32 (3, nz, ny, nx), component x, y, z.
"""
import ctypes

import torch

from . import _abi
from .plan import _stream_handle


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _vol_check(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 tensor")


def _field_check(t, shape, name):
    _vol_check(t, name)
    if tuple(t.shape) != (3,) + tuple(shape):
        raise ValueError(f"{name} must have shape {(3,) + tuple(shape)}, got {tuple(t.shape)}")


def grad(vol, out=None, stream=None):
    """Forward differences (last difference along each axis 0)."""
    _vol_check(vol, "vol")
    nz, ny, nx = vol.shape
    out = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=vol.device) if out is None else out
    _field_check(out, vol.shape, "out")
    _abi.lamino_tv_grad(_ptr(vol), _ptr(out), nz, ny, nx, _stream_handle(stream))
    return out


def div(p, out=None, stream=None):
    """-grad^T p."""
    _vol_check(p, "p")
    _, nz, ny, nx = p.shape
    out = torch.empty((nz, ny, nx), dtype=torch.float32, device=p.device) if out is None else out
    _vol_check(out, "out")
    _abi.lamino_tv_div(_ptr(p), _ptr(out), nz, ny, nx, _stream_handle(stream))
    return out


def tv_term(vol, rho, shift=None, base=None, out=None, stream=None):
    """base - rho div(grad vol - shift) (base, shift default to zero)."""
    _vol_check(vol, "vol")
    nz, ny, nx = vol.shape
    if shift is not None:
        _field_check(shift, vol.shape, "shift")
    if base is not None:
        _vol_check(base, "base")
    out = torch.empty_like(vol) if out is None else out
    _vol_check(out, "out")
    _abi.lamino_tv_term(_ptr(vol), _ptr(shift), _ptr(base), rho, _ptr(out), nz, ny, nx,
                        _stream_handle(stream))
    return out


def shrink(vol, lam, shift, alpha, rho, psi=None, stream=None):
    """psi = shrink(grad vol + lam / rho, alpha / rho); lam += rho (grad vol - psi)
    in place; shift = psi - lam / rho.  Returns psi when it is given."""
    _vol_check(vol, "vol")
    nz, ny, nx = vol.shape
    _field_check(lam, vol.shape, "lam")
    _field_check(shift, vol.shape, "shift")
    if psi is not None:
        _field_check(psi, vol.shape, "psi")
    _abi.lamino_tv_shrink(_ptr(vol), _ptr(lam), _ptr(shift), _ptr(psi), alpha, rho, nz, ny, nx,
                          _stream_handle(stream))
    return psi


class AdmmTV:
    """ADMM state for one plan: lambda and shift = psi - lambda / rho live in
    a torch-owned device buffer between calls (so `run` can resume)."""

    def __init__(self, plan, alpha, rho):
        if plan.data_dtype != "f32":
            raise ValueError("ADMM needs a plan with float32 data")
        self.plan = plan
        self.alpha = float(alpha)
        self.rho = float(rho)
        nbytes = _abi.lamino_admm_tv_state_bytes(plan._h)
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=plan.device)
        nv = plan.shape_vol[0] * plan.shape_vol[1] * plan.shape_vol[2]
        off = (3 * nv * 4 + 255) // 256 * 256
        field = (3,) + tuple(plan.shape_vol)
        self.lam = self.state[: 3 * nv * 4].view(torch.float32).view(field)
        self.shift = self.state[off: off + 3 * nv * 4].view(torch.float32).view(field)
        self._started = False

    def run(self, data, vol, outer, inner, resume=None, stream=None):
        """Run `outer` ADMM iterations of `inner` CG steps each; vol (the initial
        guess) is updated in place.  resume defaults to True after the first call."""
        self.plan._check(data, self.plan.shape_data, torch.float32, "data")
        self.plan._check(vol, self.plan.shape_vol, torch.float32, "vol")
        if resume is None:
            resume = self._started
        _abi.lamino_admm_tv(self.plan._h, _ptr(data), _ptr(vol), self.alpha, self.rho, outer,
                            inner, resume, _ptr(self.state), _stream_handle(stream))
        self._started = True
        return vol


def admm_tv(plan, data, alpha, rho, outer, inner, x0=None, stream=None):
    """TV-regularised reconstruction; returns (vol, AdmmTV state)."""
    vol = (torch.zeros(plan.shape_vol, dtype=torch.float32, device=plan.device)
           if x0 is None else x0.clone())
    st = AdmmTV(plan, alpha, rho)
    st.run(data, vol, outer, inner, resume=False, stream=stream)
    return vol, st
