"""Pins of the FGMRES oracle (CPU): the minimal-residual property against explicit
Krylov least-squares problems (plain, right-preconditioned with a fixed SSOR, flexible
with recorded directions), finite termination, monotone restarts, and FGMRES rescuing a
two-grid cycle that diverges on its own."""
import numpy as np
import pytest

from oracle import krylov, precond, problem, spectra, twogrid


def _problem(n=7, eps=0.05, theta=0.6, seed=0):
    coef = problem.q1_stencil(eps, theta)
    b = np.random.default_rng(seed).standard_normal((n, n))
    return coef, b, (lambda x: problem.apply_A(coef, x))


def _min_res(cols, b, A_on=None):
    """min_y ||b - sum_k y_k A(c_k)|| / ||b|| through an explicit least-squares solve."""
    Ac = np.stack([(A_on(c) if A_on else c).ravel() for c in cols], axis=1)
    y = np.linalg.lstsq(Ac, b.ravel(), rcond=None)[0]
    return np.linalg.norm(b.ravel() - Ac @ y) / np.linalg.norm(b)


def test_gmres_is_the_krylov_minimiser():
    coef, b, A = _problem()
    _, hist, _ = krylov.fgmres(A, b, restart=30, max_iter=12, tol=0.0)
    K = [b]
    for j in range(1, 12):
        K.append(A(K[-1]))
    for j in range(1, 13):
        # columns of A K_j span A times the Krylov space K_j(A, b)
        want = _min_res(K[:j], b, A_on=A)
        assert abs(hist[j - 1] - want) <= 1e-10 * max(1.0, want), (j, hist[j - 1], want)


def test_gmres_terminates_on_a_small_system():
    coef, b, A = _problem(n=5)
    x, hist, it = krylov.fgmres(A, b, restart=25, max_iter=25, tol=1e-12)
    assert hist[-1] <= 1e-12 and it <= 25
    Ad = np.stack([A(e.reshape(5, 5)).ravel() for e in np.eye(25)], axis=1)
    np.testing.assert_allclose(x.ravel(), np.linalg.solve(Ad, b.ravel()), rtol=1e-9, atol=1e-10)


def test_fixed_preconditioner_gives_right_preconditioned_gmres():
    coef, b, A = _problem(n=9, eps=1e-2)
    M = precond.ssor_binv(coef, 1.2)
    _, hist, _ = krylov.fgmres(A, b, precond=lambda j, v: M(v), restart=30, max_iter=10, tol=0.0)
    K = [b]
    for j in range(1, 10):
        K.append(A(M(K[-1])))
    for j in range(1, 11):
        want = _min_res([M(k) for k in K[:j]], b, A_on=A)
        assert abs(hist[j - 1] - want) <= 1e-10 * max(1.0, want), (j, hist[j - 1], want)


def test_flexible_minimises_over_its_own_directions():
    """With a preconditioner that changes every iteration, the residual is the minimum
    over the span of the directions z_j actually used."""
    coef, b, A = _problem(n=9, eps=0.2)
    Zs = []
    G = problem.gershgorin(coef)

    def M(j, v):
        # j + 1 Richardson steps with weight 1/G from zero: a different map every time
        z = np.zeros_like(v)
        for _ in range(j + 1):
            z = z + (v - A(z)) / G
        Zs.append(z)
        return z

    _, hist, _ = krylov.fgmres(A, b, precond=M, restart=30, max_iter=8, tol=0.0)
    for j in range(1, 9):
        want = _min_res(Zs[:j], b, A_on=A)
        assert abs(hist[j - 1] - want) <= 1e-10 * max(1.0, want), (j, hist[j - 1], want)


def test_restarted_residual_never_increases():
    coef, b, A = _problem(n=15, eps=1e-3)
    x, hist, it = krylov.fgmres(A, b, restart=5, max_iter=60, tol=1e-14)
    assert np.all(np.diff(hist) <= 1e-13)
    assert abs(np.linalg.norm(b - A(x)) / np.linalg.norm(b) - hist[-1]) <= 1e-9


def test_fgmres_rescues_a_diverging_two_grid_cycle():
    """A two-grid cycle whose coarse symbol is the exact inverse of the rediscretised coarse
    operator amplifies near-resonant modes at this wavenumber; as a preconditioner inside
    FGMRES(20) it still drives the residual below 1e-8."""
    n, kappa, m = 63, 31.0, 4
    nc = 31
    coef = problem.helmholtz_stencil(kappa, n)
    A = lambda x: problem.apply_A(coef, x)
    h = 1.0 / (n + 1)
    x_ = np.arange(1, n + 1) * h
    b = np.exp(-((x_[None, :] - 0.3) ** 2 + (x_[:, None] - 0.6) ** 2) / (2 * (2 * h) ** 2))
    G = problem.gershgorin(coef)
    omega = np.full(m, 0.6 / G)
    symbol = 1.0 / spectra.helmholtz_eigenvalues(kappa, nc)
    _, hist_tg = twogrid.run("richardson", coef, b, omega, symbol, 10, history=True)
    assert hist_tg[-1] > hist_tg[0], hist_tg
    pre = lambda j, v: twogrid.run("richardson", coef, v, omega, symbol, 1)
    x, hist, it = krylov.fgmres(A, b, precond=pre, restart=20, max_iter=100, tol=1e-8)
    assert hist[-1] <= 1e-8 and it < 100, (it, hist[-1])
    assert np.linalg.norm(b - A(x)) / np.linalg.norm(b) <= 2e-8
