"""Iterative refinement around a long-step inner solve, test infrastructure only.

Not in the paper: the paper stops a single iteration at a relative residual of
1e-6 (§2.3).  To reach 1e-10 with low-precision sweeps the inner iteration is
wrapped in classical iterative refinement:

  round j:  r_j = b - A x_j,  rho_j = ||r_j|| / ||b||;  stop when rho_j <= tol;
            solve A d = r_j approximately with the chosen Table-1 scheme from
            d = 0, v = 0 (the momentum restarts every round), running whole outer
            iterations until ||r_j - A d|| / ||r_j|| <= tol_inner or the cap;
            x_{j+1} = x_j + d.

This oracle runs the inner solve in FP64 as well.
"""
import numpy as np

from .problem import apply_A
from . import iterate


def refined_solve(method, coef, b, omega, tol, tol_inner=1e-4, max_outer=100000, max_rounds=50,
                  alpha=None, alpha_t=None):
    """Returns (x, rounds, rho_history, inner_outer_iterations)."""
    x = np.zeros_like(b, dtype=np.float64)
    bn = np.linalg.norm(b)
    rhos, inner = [], []
    for _ in range(max_rounds + 1):
        r = b - apply_A(coef, x)
        rho = np.linalg.norm(r) / bn
        rhos.append(rho)
        if rho <= tol or not np.isfinite(rho) or len(inner) == max_rounds:
            break
        d, k, _ = iterate.solve_to_tol(method, coef, r, omega, tol_inner, max_outer,
                                       alpha=alpha, alpha_t=alpha_t)
        inner.append(k)
        x = x + d
    return x, len(inner), np.array(rhos), inner
