"""Closed-form spectra of the stencils, test infrastructure only.

When the mixed coefficient b of C vanishes (theta in {0, pi/2, pi}; §2.3), the
interior Q1 operator is diagonalised by the discrete sine modes
phi_pq[j, i] = sin(p pi x_i) sin(q pi y_j), x_i = i h, y_j = j h (i, j = 1..n,
h = 1/(n+1)), with cx = cos(p pi h), cy = cos(q pi h):
    lambda_pq = (2/3) [ a (1 - cx)(2 + cy) + c (1 - cy)(2 + cx) ].
For the 5-point Helmholtz operator of §3.2 (constant kappa):
    lambda_pq = (4/h^2) (sin^2(p pi h / 2) + sin^2(q pi h / 2)) - kappa^2.
Both follow from substituting phi_pq into the stencil rows and using
sin(t + s) + sin(t - s) = 2 sin t cos s.
"""
import numpy as np

from .problem import diffusion_tensor


def _modes(n):
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1)
    return h, np.cos(k * np.pi * h)


def q1_eigenvalues(eps, theta, n):
    """All n^2 eigenvalues as an array lam[q-1, p-1] (requires b = 0)."""
    a, b, c = diffusion_tensor(eps, theta)
    if abs(b) > 1e-14:
        raise ValueError("closed form needs a vanishing mixed term (theta in {0, pi/2, pi})")
    _, cs = _modes(n)
    cx = cs[None, :]
    cy = cs[:, None]
    return (2.0 / 3.0) * (a * (1.0 - cx) * (2.0 + cy) + c * (1.0 - cy) * (2.0 + cx))


def q1_extreme_eigenvalues(eps, theta, n):
    lam = q1_eigenvalues(eps, theta, n)
    return float(lam.min()), float(lam.max())


def helmholtz_eigenvalues(kappa, n):
    h, _ = _modes(n)
    k = np.arange(1, n + 1)
    s = np.sin(k * np.pi * h / 2.0) ** 2
    return (4.0 / (h * h)) * (s[None, :] + s[:, None]) - kappa * kappa


def sine_mode(n, p, q):
    """phi_pq sampled on the interior nodes, as u[j, i]."""
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    return np.sin(q * np.pi * x)[:, None] * np.sin(p * np.pi * x)[None, :]
