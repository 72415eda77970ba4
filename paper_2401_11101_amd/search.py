"""Rotation-axis and tilt search: one reconstructed slice per candidate.

The search strategy of the paper (Section "Mouse brain imaging") first
reconstructs one slice for a sweep of rotation-axis positions at an
approximate tilt, then one slice for a sweep of tilts at the chosen axis.
`center_sweep` runs `lamino_fbp_slices` once per axis offset on one plan;
`tilt_sweep` builds one plan per tilt, all bound to a single workspace
(their calls run one after another on one stream).  Each slice is a full
Fourier-route FBP up to the x3 transform, which forms only that slice.
"""
import torch

from .plan import Plan


def center_sweep(plan, data, shifts, z, stream=None):
    """(len(shifts), n, n) float32: slice z for the axis at column w/2 + shift."""
    out = torch.empty((len(shifts),) + plan.shape_vol[1:], dtype=torch.float32, device=plan.device)
    for i, sh in enumerate(shifts):
        plan.fbp_slices(data, center_shift=float(sh), z_first=z, z_count=1, out=out[i:i + 1],
                        stream=stream)
    return out


def tilt_sweep(nz, n, n_theta, h, w, tilts, data, z, center_shift=0.0, stream=None, **plan_kw):
    """(len(tilts), n, n) float32: slice z for every tilt (radians)."""
    out = None
    work = None
    for i, phi in enumerate(tilts):
        plan = Plan(nz, n, n_theta, h, w, phi, work=work, stream=stream, **plan_kw)
        work = plan.work
        if out is None:
            out = torch.empty((len(tilts), n, n), dtype=torch.float32, device=plan.device)
        plan.fbp_slices(data, center_shift=center_shift, z_first=z, z_count=1, out=out[i:i + 1],
                        stream=stream)
        # the tables of this plan must outlive its call: keep the plan until the stream has run it
        torch.cuda.current_stream(plan.device).synchronize() if stream is None else stream.synchronize()
        del plan
    return out
