"""Pins of O5 (TV-regularised ADMM, Appendix A) against closed forms,
brute force and optimality conditions that do not go through its code."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import tv


def test_grad_of_affine_field_is_constant_with_zero_far_boundary():
    # mu = a x + b y + c z: forward differences are (a, b, c) exactly,
    # except on the last plane along each axis, where they are zero.
    nz, ny, nx = 4, 5, 6
    a, b, c = 0.5, -1.25, 2.0
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    g = tv.grad(a * x + b * y + c * z + 3.0)
    assert np.all(g[0, :, :, :-1] == a) and np.all(g[0, :, :, -1] == 0)
    assert np.all(g[1, :, :-1, :] == b) and np.all(g[1, :, -1, :] == 0)
    assert np.all(g[2, :-1, :, :] == c) and np.all(g[2, -1, :, :] == 0)


def test_grad_matches_hand_values():
    mu = np.zeros((2, 2, 3))
    mu[1, 1, 1] = 1.0
    g = tv.grad(mu)
    # only the neighbours before (1,1,1) along each axis see +1; the voxel
    # itself sees -1 towards its successor in x (x = 2 exists) and 0 along
    # y and z (last plane).
    assert g[0, 1, 1, 0] == 1.0 and g[0, 1, 1, 1] == -1.0
    assert g[1, 1, 0, 1] == 1.0 and g[1, 1, 1, 1] == 0.0
    assert g[2, 0, 1, 1] == 1.0 and g[2, 1, 1, 1] == 0.0
    assert np.count_nonzero(g) == 4


def test_div_is_minus_grad_transpose_by_matrix_columns():
    # Build both operators as dense matrices from unit vectors and check
    # D = -G^T entry by entry (div is written independently of grad).
    shape = (3, 4, 5)
    n = int(np.prod(shape))
    G = np.stack([tv.grad(np.eye(n)[k].reshape(shape)).ravel() for k in range(n)], 1)
    D = np.stack([tv.div(np.eye(3 * n)[k].reshape((3,) + shape)).ravel() for k in range(3 * n)], 1)
    assert np.array_equal(D, -G.T)


def test_div_of_interior_ramp_field():
    # p = (x, y, z) componentwise: backward differences give 1 + 1 + 1 in
    # the interior (every axis index in 1..n-2).
    nz, ny, nx = 5, 6, 7
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p = np.stack([x, y, z]).astype(float)
    d = tv.div(p)
    assert np.all(d[1:-1, 1:-1, 1:-1] == 3.0)


def test_shrink_is_the_proximal_minimiser_by_brute_force():
    # argmin_psi t |psi| + 1/2 |psi - v|^2 over 3-vectors, found numerically.
    rng = np.random.default_rng(4)
    for _ in range(20):
        v = rng.standard_normal(3) * rng.uniform(0.1, 3)
        t = rng.uniform(0.0, 2.0)
        f = lambda q: t * np.sqrt(q @ q + 1e-30) + 0.5 * np.sum((q - v) ** 2)
        best = minimize(f, v * 0.5, method="Nelder-Mead",
                        options=dict(xatol=1e-10, fatol=1e-14, maxiter=20000)).x
        s = tv.shrink(v.reshape(3, 1), t).ravel()
        assert f(s) <= f(best) + 1e-10
        assert np.linalg.norm(s - best) < 1e-4


def test_shrink_special_cases():
    v = np.array([[3.0, 0.1, 0.0], [4.0, 0.0, 0.0], [0.0, 0.0, 0.0]])  # (3, 3 voxels)
    s = tv.shrink(v, 1.0)
    assert np.allclose(s[:, 0], [2.4, 3.2, 0.0])  # |v| = 5 -> 4, same direction
    assert np.all(s[:, 1] == 0) and np.all(s[:, 2] == 0)
    assert np.array_equal(tv.shrink(v, 0.0), v)


def _dense_problem(shape, m, seed):
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    L = lambda x: A @ x.ravel()
    Lt = lambda y: (A.T @ y).reshape(shape)
    return A, L, Lt


def test_tomo_subproblem_reaches_the_normal_equation_solution():
    # With enough CG steps Eq:tomo is solved exactly: the minimiser of
    # 1/2|A mu - d|^2 + rho/2 |G mu - s|^2 solves
    # (A^T A + rho G^T G) mu = A^T d + rho G^T s, with s = psi - lambda/rho.
    shape = (2, 3, 4)
    n = 24
    A, L, Lt = _dense_problem(shape, 30, 0)
    rng = np.random.default_rng(1)
    d = rng.standard_normal(30)
    psi = rng.standard_normal((3,) + shape)
    lam = rng.standard_normal((3,) + shape)
    rho = 0.7
    G = np.stack([tv.grad(np.eye(n)[k].reshape(shape)).ravel() for k in range(n)], 1)
    s = (psi - lam / rho).ravel()
    x = np.linalg.solve(A.T @ A + rho * G.T @ G, A.T @ d + rho * G.T @ s)
    mu = tv.tomo_subproblem(L, Lt, d, np.zeros(shape), psi, lam, rho, 60)
    assert np.linalg.norm(mu.ravel() - x) < 1e-9 * np.linalg.norm(x)


def test_admm_without_regularisation_reaches_least_squares():
    # alpha = 0: psi = grad mu + lambda/rho and lambda stays zero, so the
    # iteration is a proximal-point method on the least-squares problem.
    shape = (2, 3, 4)
    A, L, Lt = _dense_problem(shape, 40, 2)
    d = np.random.default_rng(3).standard_normal(40)
    x = np.linalg.lstsq(A, d, rcond=None)[0]
    mu, psi, lam = tv.admm(L, Lt, d, np.zeros(shape), 0.0, 0.05, 100, 30)
    assert np.linalg.norm(mu.ravel() - x) < 1e-8 * np.linalg.norm(x)
    assert np.abs(lam).max() == 0.0


def test_admm_tv_denoises_a_step_to_its_closed_form():
    # L = identity on a 1D signal (nz = ny = 1): d = 0 on n1 samples, h on
    # n2.  The TV-denoised solution keeps the jump position and moves each
    # plateau towards the other by alpha / (its length):
    #   mu = alpha/n1 on the left, h - alpha/n2 on the right
    # (valid while alpha/n1 + alpha/n2 < h).
    n1, n2, h, alpha = 6, 10, 1.0, 0.5
    d = np.concatenate([np.zeros(n1), np.full(n2, h)]).reshape(1, 1, -1)
    ident = lambda x: x
    mu, _, _ = tv.admm(ident, ident, d, np.zeros_like(d), alpha, 1.0, 400, 20)
    want = np.concatenate([np.full(n1, alpha / n1), np.full(n2, h - alpha / n2)])
    assert np.abs(mu.ravel() - want).max() < 1e-6


def test_admm_fixed_point_satisfies_the_optimality_conditions():
    # At a minimiser of eq:mainregproblem there is a lambda with
    #   A^T (A mu - d) - div lambda = 0,
    #   |lambda_v| <= alpha everywhere and lambda_v = alpha g_v / |g_v|
    #   wherever g = grad mu is non-zero.
    # ADMM's dual variable must converge to such a certificate.
    shape = (3, 4, 4)
    A, L, Lt = _dense_problem(shape, 60, 5)
    rng = np.random.default_rng(6)
    truth = np.zeros(shape)
    truth[:, 1:3, 1:3] = 1.0
    d = L(truth) + 0.05 * rng.standard_normal(60)
    alpha = 0.05
    mu, psi, lam = tv.admm(L, Lt, d, np.zeros(shape), alpha, 2.0, 600, 10)
    stat = Lt(L(mu) - d) - tv.div(lam)
    assert np.abs(stat).max() < 1e-6
    mag = np.sqrt(np.sum(lam * lam, axis=0))
    assert mag.max() <= alpha * (1 + 1e-6)
    g = tv.grad(mu)
    gm = np.sqrt(np.sum(g * g, axis=0))
    on = gm > 1e-4
    assert np.any(on)
    assert np.abs(lam[:, on] - alpha * g[:, on] / gm[on]).max() < 1e-5
    assert np.abs(g - psi).max() < 1e-6


def test_admm_objective_beats_perturbations():
    # The ADMM result is a minimiser: random small perturbations never lower
    # the objective of eq:mainregproblem.
    shape = (2, 4, 4)
    A, L, Lt = _dense_problem(shape, 40, 7)
    d = np.random.default_rng(8).standard_normal(40)
    alpha = 0.1
    mu, _, _ = tv.admm(L, Lt, d, np.zeros(shape), alpha, 1.0, 600, 10)
    f0 = tv.objective(L, d, mu, alpha)
    rng = np.random.default_rng(9)
    for _ in range(50):
        e = rng.standard_normal(shape) * 1e-3
        assert tv.objective(L, d, mu + e, alpha) >= f0 - 1e-9


@pytest.mark.parametrize("outer", [1, 3])
def test_admm_first_step_by_hand(outer):
    # From zero state, step 1 solves the plain least-squares sub-problem
    # (psi = lambda = 0) and then applies shrink/dual update; compare with
    # the steps written out on a dense problem.
    shape = (2, 2, 3)
    n = 12
    A, L, Lt = _dense_problem(shape, 20, 10)
    d = np.random.default_rng(11).standard_normal(20)
    rho, alpha = 1.5, 0.2
    G = np.stack([tv.grad(np.eye(n)[k].reshape(shape)).ravel() for k in range(n)], 1)
    mu = np.zeros(n)
    psi = np.zeros(3 * n)
    lam = np.zeros(3 * n)
    for _ in range(outer):
        mu = np.linalg.solve(A.T @ A + rho * G.T @ G, A.T @ d + rho * G.T @ (psi - lam / rho))
        g = (G @ mu).reshape(3, n)
        v = g + lam.reshape(3, n) / rho
        mag = np.linalg.norm(v, axis=0)
        psi3 = np.where(mag > alpha / rho, 1 - (alpha / rho) / np.maximum(mag, 1e-300), 0) * v
        lam = lam + rho * (g.ravel() - psi3.ravel())
        psi = psi3.ravel()
    m2, p2, l2 = tv.admm(L, Lt, d, np.zeros(shape), alpha, rho, outer, 50)
    assert np.linalg.norm(m2.ravel() - mu) < 1e-9 * np.linalg.norm(mu)
    assert np.linalg.norm(p2.ravel() - psi) < 1e-8 * max(np.linalg.norm(psi), 1e-30) + 1e-12
    assert np.linalg.norm(l2.ravel() - lam) < 1e-8 * np.linalg.norm(lam) + 1e-12


def test_printed_factor_two_threshold_does_not_reach_the_minimiser():
    # The reading of the psi-step: the soft threshold printed with 2 lambda/rho
    # and 2 alpha/rho is not the minimiser of the Lagrangian as written.  Run
    # with it, the iteration stalls with a large constraint violation and a
    # higher objective, while the Lagrangian-consistent step (tv.admm)
    # satisfies the constraint to 1e-6 on the same problem.
    shape = (3, 4, 4)
    A, L, Lt = _dense_problem(shape, 60, 5)
    rng = np.random.default_rng(6)
    truth = np.zeros(shape)
    truth[:, 1:3, 1:3] = 1.0
    d = L(truth) + 0.05 * rng.standard_normal(60)
    alpha, rho = 0.05, 2.0
    mu_ok, psi_ok, _ = tv.admm(L, Lt, d, np.zeros(shape), alpha, rho, 600, 10)
    mu = np.zeros(shape)
    psi = np.zeros((3,) + shape)
    lam = np.zeros_like(psi)
    for _ in range(600):
        mu = tv.tomo_subproblem(L, Lt, d, mu, psi, lam, rho, 10)
        g = tv.grad(mu)
        psi = tv.shrink(g + 2 * lam / rho, 2 * alpha / rho)
        lam = lam + rho * (g - psi)
    assert np.abs(tv.grad(mu_ok) - psi_ok).max() < 1e-6
    assert np.abs(g - psi).max() > 1e-2
    assert tv.objective(L, d, mu, alpha) > tv.objective(L, d, mu_ok, alpha) + 1e-3
