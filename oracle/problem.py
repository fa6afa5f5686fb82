"""Problem and discretisation (test infrastructure only; see ``oracle/__init__``).

Anisotropic diffusion (paper §2.3, eq. anisotropy-poisson):
    -div(C grad u) = f on (0,1)^2, u = 0 on the boundary,
    C = R(theta) diag(1, eps) R(theta)^T with R(theta) = [[cos, -sin], [sin, cos]].
Discretised with bilinear (Q1) elements on a uniform grid; boundary nodes are
eliminated (homogeneous Dirichlet), which leaves an interior-only SPD system.
The paper does not print the stencil.  For a constant C the element integrals
are exact, and the assembled interior row is the 9-point stencil below (no h
factor: the 2D Q1 stiffness is scale free).

Helmholtz (paper §3.2, eq. Helmholtz-Sponge-stencil), constant wavenumber kappa,
no sponge: centre (4 - kappa^2 h^2)/h^2, the four edge neighbours -1/h^2.

Grid convention: ``n`` interior nodes per direction, h = 1/(n+1); arrays are
``u[j, i]`` with i the x index (fastest) and y increasing with j.
"""
import numpy as np

# stencil offsets (dx, dy) and the coefficient slot each one uses
#   slot 0: centre, 1: (+-1, 0), 2: (0, +-1), 3: (1,1),(-1,-1), 4: (-1,1),(1,-1)
OFFSETS = (
    ((0, 0), 0),
    ((1, 0), 1), ((-1, 0), 1),
    ((0, 1), 2), ((0, -1), 2),
    ((1, 1), 3), ((-1, -1), 3),
    ((-1, 1), 4), ((1, -1), 4),
)


def diffusion_tensor(eps, theta):
    """C = R diag(1, eps) R^T as (a, b, c) = (C11, C12, C22).  §2.3."""
    cs, sn = np.cos(theta), np.sin(theta)
    a = cs * cs + eps * sn * sn
    b = (1.0 - eps) * sn * cs
    c = sn * sn + eps * cs * cs
    return a, b, c


def q1_stencil(eps, theta):
    """Five distinct coefficients of the interior Q1 stencil row.  §2.3.

    Returns (centre, x-edge, y-edge, (1,1)/(-1,-1) corner, (-1,1)/(1,-1) corner).
    """
    a, b, c = diffusion_tensor(eps, theta)
    return np.array([
        4.0 * (a + c) / 3.0,
        -2.0 * a / 3.0 + c / 3.0,
        a / 3.0 - 2.0 * c / 3.0,
        -(a + c) / 6.0 - b / 2.0,
        -(a + c) / 6.0 + b / 2.0,
    ])


def helmholtz_stencil(kappa, n):
    """5-point FD Helmholtz coefficients in the same five slots.  §3.2."""
    h = 1.0 / (n + 1)
    return np.array([(4.0 - kappa * kappa * h * h) / (h * h), -1.0 / (h * h), -1.0 / (h * h), 0.0, 0.0])


def gershgorin(coef):
    """Gershgorin bound on the spectrum: |centre| + sum of |off-diagonal| entries."""
    return abs(coef[0]) + 2.0 * (abs(coef[1]) + abs(coef[2]) + abs(coef[3]) + abs(coef[4]))


def apply_A(coef, x):
    """y = A x for one instance with zero Dirichlet values outside the n x n interior."""
    n1, n0 = x.shape
    xp = np.zeros((n1 + 2, n0 + 2))
    xp[1:-1, 1:-1] = x
    y = np.zeros_like(x, dtype=np.float64)
    for (dx, dy), slot in OFFSETS:
        y += coef[slot] * xp[1 + dy:1 + dy + n1, 1 + dx:1 + dx + n0]
    return y


def residual(coef, f, u):
    """r = f - A u."""
    return f - apply_A(coef, u)


def relres(coef, f, u):
    """Relative residual ||f - A u|| / ||f|| (the paper's stopping quantity, §2.3)."""
    return np.linalg.norm(residual(coef, f, u)) / np.linalg.norm(f)
