"""O5: TV-regularised reconstruction by ADMM (oracle, test infrastructure only).

Appendix A minimises 1/2 ||L mu - d||^2 + alpha ||grad mu||_1 (isotropic
total variation, eq:mainregproblem) by splitting psi = grad mu (Eq:minF),
forming the augmented Lagrangian with dual variable lambda and penalty rho
(Eq:alagr), and iterating three steps (Eq:tomo, Eq:reg, Eq:lamd):

  mu     <- argmin over mu of 1/2 ||L mu - d||^2 + rho/2 ||grad mu - psi + lambda/rho||^2
            (a few conjugate-gradient iterations from the current mu, with
            the gradient L^T (L mu - d) - rho div(grad mu - psi + lambda/rho)
            of Eq:gradtomo and Dai-Yuan directions, Eq:DaiYuan2)
  psi    <- soft-threshold of grad mu + lambda/rho at alpha/rho (per voxel,
            on the 3-vector: the closed-form minimiser of Eq:reg)
  lambda <- lambda + rho (grad mu - psi)

Readings (the paper gives the continuous operators only):
  * grad: forward differences along x, y, z with the last difference along
    each axis set to zero; div = -grad^T (the paper: div is the adjoint of
    -grad), i.e. backward differences with the matching boundary terms.
  * The printed soft-threshold carries factors 2 (2 lambda/rho, 2 alpha/rho)
    that do not follow from the Lagrangian as written; the minimiser of the
    Lagrangian as written uses lambda/rho and alpha/rho, which is taken here.
  * The line search of the quadratic sub-problem is exact:
    gamma = -<g, eta> / (||L eta||^2 + rho ||grad eta||^2).

Array layout: mu[z][y][x]; gradients g[c][z][y][x] with c = 0 (x), 1 (y), 2 (z).
Pinned in tests/test_oracle_tv.py against closed forms (ramp gradients, 1D
TV denoising of a step), the adjoint identity, brute-force proximal steps,
and least squares for alpha = 0.
"""
import numpy as np


def grad(mu):
    """Forward differences, zero last difference: (3, nz, ny, nx)."""
    mu = np.asarray(mu, dtype=np.float64)
    g = np.zeros((3,) + mu.shape)
    g[0, :, :, :-1] = mu[:, :, 1:] - mu[:, :, :-1]
    g[1, :, :-1, :] = mu[:, 1:, :] - mu[:, :-1, :]
    g[2, :-1, :, :] = mu[1:, :, :] - mu[:-1, :, :]
    return g


def div(p):
    """-grad^T p (backward differences with the matching boundary terms)."""
    p = np.asarray(p, dtype=np.float64)
    out = np.zeros(p.shape[1:])
    # component x: (grad^T q)_i = q_{i-1} [i >= 1] - q_i [i <= n-2]
    px, py, pz = p[0], p[1], p[2]
    out[:, :, :-1] += px[:, :, :-1]
    out[:, :, 1:] -= px[:, :, :-1]
    out[:, :-1, :] += py[:, :-1, :]
    out[:, 1:, :] -= py[:, :-1, :]
    out[:-1, :, :] += pz[:-1, :, :]
    out[1:, :, :] -= pz[:-1, :, :]
    return out


def shrink(v, t):
    """Isotropic soft threshold of the 3-vectors v[:, ...] at t >= 0."""
    v = np.asarray(v, dtype=np.float64)
    mag = np.sqrt(np.sum(v * v, axis=0))
    scale = np.where(mag > t, 1.0 - t / np.where(mag > 0, mag, 1.0), 0.0)
    return v * scale


def tv_norm(mu):
    g = grad(mu)
    return float(np.sum(np.sqrt(np.sum(g * g, axis=0))))


def objective(L, d, mu, alpha):
    r = L(mu) - d
    return 0.5 * float(np.vdot(r, r).real) + alpha * tv_norm(mu)


def _dot(a, b):
    return float(np.vdot(np.ravel(a), np.ravel(b)).real)


def tomo_subproblem(L, Lt, d, mu, psi, lam, rho, iters):
    """Eq:tomo by `iters` conjugate-gradient steps (Dai-Yuan, exact line search)."""
    mu = np.array(mu, dtype=np.float64, copy=True)
    shift = psi - lam / rho

    def gradF(x):
        return Lt(L(x) - d) - rho * div(grad(x) - shift)

    g = gradF(mu)
    eta = -g
    for _ in range(iters):
        Le = L(eta)
        ge = grad(eta)
        denom = _dot(Le, Le) + rho * _dot(ge, ge)
        if denom == 0.0:
            break
        gamma = -_dot(g, eta) / denom
        mu = mu + gamma * eta
        g_new = gradF(mu)
        y = _dot(g_new - g, eta)
        if y == 0.0:
            break
        eta = -g_new + (_dot(g_new, g_new) / y) * eta
        g = g_new
    return mu


def admm(L, Lt, d, mu0, alpha, rho, outer, inner, callback=None):
    """Appendix A's ADMM; returns (mu, psi, lambda)."""
    mu = np.array(mu0, dtype=np.float64, copy=True)
    psi = np.zeros((3,) + mu.shape)
    lam = np.zeros_like(psi)
    for k in range(outer):
        mu = tomo_subproblem(L, Lt, d, mu, psi, lam, rho, inner)
        g = grad(mu)
        psi = shrink(g + lam / rho, alpha / rho)
        lam = lam + rho * (g - psi)
        if callback is not None:
            callback(k, mu)
    return mu, psi, lam
