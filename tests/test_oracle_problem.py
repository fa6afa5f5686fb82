"""Pins for the oracle's operator: stencil, symmetry, spectra (CPU only)."""
import numpy as np
import pytest

from oracle import problem, spectra

PARAMS = [(1.0, 0.0), (0.3, 1.1), (1e-4, 2.5), (1e-2, np.pi / 2), (0.7, np.pi)]


def q1_assembled_matrix(eps, theta, n):
    """Dense interior stiffness matrix built element by element with 2x2 Gauss quadrature
    on bilinear shape functions (an assembly route independent of the stencil formula)."""
    cs, sn = np.cos(theta), np.sin(theta)
    R = np.array([[cs, -sn], [sn, cs]])
    C = R @ np.diag([1.0, eps]) @ R.T
    g = 0.5 / np.sqrt(3.0)
    gauss = [0.5 - g, 0.5 + g]
    corners = [(0, 0), (1, 0), (0, 1), (1, 1)]

    def grad(k, xi, eta):
        cx, cy = corners[k]
        sx = xi if cx else (1.0 - xi)
        sy = eta if cy else (1.0 - eta)
        dx = (1.0 if cx else -1.0) * sy
        dy = (1.0 if cy else -1.0) * sx
        return np.array([dx, dy])

    Ke = np.zeros((4, 4))
    for xi in gauss:
        for eta in gauss:
            for p in range(4):
                for q in range(4):
                    Ke[p, q] += 0.25 * grad(p, xi, eta) @ C @ grad(q, xi, eta)
    M = n + 2
    Kg = np.zeros((M * M, M * M))
    for ej in range(M - 1):
        for ei in range(M - 1):
            nodes = [(ej + cy) * M + (ei + cx) for (cx, cy) in corners]
            for p in range(4):
                for q in range(4):
                    Kg[nodes[p], nodes[q]] += Ke[p, q]
    interior = [j * M + i for j in range(1, M - 1) for i in range(1, M - 1)]
    return Kg[np.ix_(interior, interior)]


def operator_matrix(coef, n):
    cols = []
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        cols.append(problem.apply_A(coef, e.reshape(n, n)).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("eps,theta", PARAMS)
def test_stencil_matches_element_assembly(eps, theta):
    for n in (3, 6):
        A_fe = q1_assembled_matrix(eps, theta, n)
        A_or = operator_matrix(problem.q1_stencil(eps, theta), n)
        assert np.max(np.abs(A_fe - A_or)) < 1e-14


@pytest.mark.parametrize("eps,theta", PARAMS)
def test_stencil_exact_on_quadratics(eps, theta):
    # -div(C grad q) for q = x^2, xy, y^2 is -2a, -2b, -2c; the Q1 row reproduces h^2 times it
    n = 15
    h = 1.0 / (n + 1)
    a, b, c = problem.diffusion_tensor(eps, theta)
    x = np.arange(1, n + 1) * h
    X, Y = np.meshgrid(x, x)          # X[j, i] = x_i, Y[j, i] = y_j
    coef = problem.q1_stencil(eps, theta)
    deep = (slice(2, -2), slice(2, -2))
    for q, want in ((X * X, -2 * a), (X * Y, -2 * b), (Y * Y, -2 * c), (np.ones_like(X), 0.0)):
        got = problem.apply_A(coef, q)[deep] / (h * h)
        assert np.max(np.abs(got - want)) < 1e-10


def test_isotropic_stencil_values():
    assert np.allclose(problem.q1_stencil(1.0, 0.0), [8 / 3, -1 / 3, -1 / 3, -1 / 3, -1 / 3], atol=1e-15)


@pytest.mark.parametrize("eps,theta", PARAMS)
def test_symmetry(eps, theta):
    rng = np.random.default_rng(7)
    coef = problem.q1_stencil(eps, theta)
    x, y = rng.standard_normal((2, 9, 9))
    lhs = np.sum(problem.apply_A(coef, x) * y)
    rhs = np.sum(x * problem.apply_A(coef, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) + 1e-13


@pytest.mark.parametrize("eps,theta", [(1.0, 0.0), (1e-3, 0.0), (0.2, np.pi / 2), (1e-6, np.pi)])
def test_q1_closed_form_spectrum(eps, theta):
    n = 15
    coef = problem.q1_stencil(eps, theta)
    lam = spectra.q1_eigenvalues(eps, theta, n)
    for p, q in ((1, 1), (3, 7), (15, 2), (15, 15)):
        phi = spectra.sine_mode(n, p, q)
        assert np.allclose(problem.apply_A(coef, phi), lam[q - 1, p - 1] * phi, atol=1e-13)
    dense = np.linalg.eigvalsh(q1_assembled_matrix(eps, theta, n))
    assert np.max(np.abs(np.sort(lam.ravel()) - dense)) < 1e-13


def test_q1_extremes_isotropic_n63():
    lmin, lmax = spectra.q1_extreme_eigenvalues(1.0, 0.0, 63)
    # eps = 1: lambda = (2/3)(4 - cx - cy - 2 cx cy); the largest value sits at (p, q) = (1, n),
    # cx = c, cy = -c, the smallest at p = q = 1, with c = cos(pi h)
    c = np.cos(np.pi / 64)
    assert abs(lmax - (8.0 + 4.0 * c * c) / 3.0) < 1e-14
    assert abs(lmin - (2.0 / 3.0) * (4.0 - 2.0 * c - 2.0 * c * c)) < 1e-15


def test_helmholtz_closed_form_spectrum():
    n, kappa = 31, 25.0
    coef = problem.helmholtz_stencil(kappa, n)
    lam = spectra.helmholtz_eigenvalues(kappa, n)
    for p, q in ((1, 1), (5, 9), (31, 30)):
        phi = spectra.sine_mode(n, p, q)
        got = problem.apply_A(coef, phi)
        assert np.allclose(got, lam[q - 1, p - 1] * phi, atol=1e-9 * np.max(np.abs(lam)))
    # 5-point Laplacian by hand at one interior node
    rng = np.random.default_rng(3)
    u = rng.standard_normal((n, n))
    h = 1.0 / (n + 1)
    j, i = 10, 20
    want = (4 * u[j, i] - u[j, i + 1] - u[j, i - 1] - u[j + 1, i] - u[j - 1, i]) / h**2 - kappa**2 * u[j, i]
    assert abs(problem.apply_A(coef, u)[j, i] - want) < 1e-9


def test_gershgorin_bounds_spectrum():
    for eps, theta in PARAMS:
        coef = problem.q1_stencil(eps, theta)
        lmax = np.linalg.eigvalsh(q1_assembled_matrix(eps, theta, 8)).max()
        assert lmax <= problem.gershgorin(coef) + 1e-12
