"""Differentiable laminography operators and a least-squares CG solver.

`LaminoL` applies the forward projector L (eq:fwd, evaluated by the
library's Fourier route); its backward is the library's adjoint L*
(eq:adj), and `LaminoLstar` the other way round.  Because the library's
pair is an exact transpose, autograd gradients of any loss through these
Functions are exact up to rounding.

`cgls` minimises 1/2 ||L mu - d||^2 with conjugate gradients, the data
sub-problem that Appendix A solves inside its ADMM scheme: with an exact
line search and the Dai-Yuan direction this is the classical CGLS
recursion (one L and one L* per iteration).  Vector updates run as torch
element-wise operations on the device; inner products accumulate in
float64.
"""
import torch


class LaminoL(torch.autograd.Function):
    """d = L vol; backward: grad_vol = L* grad_d."""

    @staticmethod
    def forward(ctx, vol, plan):
        ctx.plan = plan
        return plan.fwd(vol.contiguous())

    @staticmethod
    def backward(ctx, grad_d):
        plan = ctx.plan
        g = grad_d.contiguous().to(plan.torch_data_dtype)
        return plan.adj(g), None


class LaminoLstar(torch.autograd.Function):
    """vol = L* d; backward: grad_d = L grad_vol."""

    @staticmethod
    def forward(ctx, data, plan):
        ctx.plan = plan
        ctx.dtype = data.dtype
        return plan.adj(data.contiguous())

    @staticmethod
    def backward(ctx, grad_vol):
        return ctx.plan.fwd(grad_vol.contiguous().float()).to(ctx.dtype), None


def _dot(a, b):
    return float(torch.sum(a.double() * b.double()))


def cgls(plan, data, iters=20, x0=None, callback=None):
    """Conjugate gradients for min 1/2 ||L x - d||^2 (x: float32 volume).

    callback(k, x, residual_norm) is called after every iteration."""
    L = lambda x: plan.fwd(x).float()
    Lt = lambda y: plan.adj(y.to(plan.torch_data_dtype).contiguous())
    d = data.float()
    x = torch.zeros(plan.shape_vol, dtype=torch.float32, device=plan.device) if x0 is None else x0.clone()
    r = d - L(x) if x0 is not None else d.clone()
    s = Lt(r)
    p = s.clone()
    gamma = _dot(s, s)
    for k in range(iters):
        q = L(p)
        qq = _dot(q, q)
        if qq == 0.0 or gamma == 0.0:
            break
        alpha = gamma / qq
        x.add_(p, alpha=alpha)
        r.add_(q, alpha=-alpha)
        s = Lt(r)
        gamma_new = _dot(s, s)
        p.mul_(gamma_new / gamma).add_(s)
        gamma = gamma_new
        if callback is not None:
            callback(k, x, float(torch.linalg.vector_norm(r.double())))
    return x
