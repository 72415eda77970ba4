"""O4: conjugate gradients for min 1/2 ||L mu - d||^2 (oracle, test only).

Appendix A solves its data sub-problem with conjugate gradients: the
gradient of F is L^T (L mu - d) (plus a TV term, absent here), the step
length comes from a line search and the direction update uses the
Dai-Yuan formula, starting from the negative gradient.  For this
quadratic F the line search is exact in closed form:
  gamma = -<grad F(mu), eta> / ||L eta||^2.

`cg_daiyuan` follows those steps.  `cgls` is the textbook CGLS recursion
(Hestenes-Stiefel applied to the normal equations, Bjorck's form).  In
exact arithmetic both produce the same iterates on this problem, which the
tests use as one pin; the other is numpy.linalg.lstsq on small dense
problems.
"""
import numpy as np


def _dot(a, b):
    return float(np.vdot(np.ravel(a), np.ravel(b)).real)


def cg_daiyuan(L, Lt, d, mu0, iters, callback=None):
    mu = np.array(mu0, dtype=np.float64, copy=True)
    grad = Lt(L(mu) - d)
    eta = -grad
    for k in range(iters):
        Leta = L(eta)
        denom = _dot(Leta, Leta)
        if denom == 0.0:
            break
        gamma = -_dot(grad, eta) / denom
        mu = mu + gamma * eta
        grad_new = Lt(L(mu) - d)
        y = _dot(grad_new - grad, eta)
        if y == 0.0:
            break
        beta = _dot(grad_new, grad_new) / y
        eta = -grad_new + beta * eta
        grad = grad_new
        if callback is not None:
            callback(k, mu)
    return mu


def cgls(L, Lt, d, mu0, iters, callback=None):
    x = np.array(mu0, dtype=np.float64, copy=True)
    r = d - L(x)
    s = Lt(r)
    p = s.copy()
    gamma = _dot(s, s)
    for k in range(iters):
        q = L(p)
        qq = _dot(q, q)
        if qq == 0.0 or gamma == 0.0:
            break
        alpha = gamma / qq
        x = x + alpha * p
        r = r - alpha * q
        s = Lt(r)
        gamma_new = _dot(s, s)
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        if callback is not None:
            callback(k, x)
    return x
