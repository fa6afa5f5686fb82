"""Two-grid iteration for the Helmholtz problem, test infrastructure only.

The multilevel solvers of §3 alternate a smoothing iteration (eq. dl-him-b) with a
spectral correction u += H (f - A u) (eq. dl-him-h), H = F T Lambda~ T* F^{-1}:
a transform to a basis that (approximately) diagonalises A, a pointwise symbol
Lambda~ standing in for the inverse eigenvalues, and the transform back.  §3.2 puts a
Table-1 scheme in the smoother's place.  This module is the two-grid form of that
cycle on the constant-coefficient Dirichlet problem:

  smoothing:   m inner steps of a Table-1 scheme from (u_k, v = 0), weights
               omega_1 .. omega_m in order;
  correction:  r = f - A u^{k+1/2};  u_{k+1} = u^{k+1/2} + P S (Lambda~ * (S R r S)) S

with R full weighting onto the coarse grid, P bilinear interpolation back, and S the
orthonormal DST-I matrix of the coarse grid (the exact eigenvector basis of every
constant-coefficient 5-point Dirichlet operator there, so T = I).  Lambda~ is an input
of shape [nc, nc], indexed [q, p] like the grid (row = y mode).

Grid: n = 2 nc + 1 interior points per direction; coarse point (I, J) sits on fine
point (2I + 1, 2J + 1) (0-based); Dirichlet zeros outside both grids.

The transfer operators are written as dense 1D matrices applied along both axes:
restrict(r) = R1 r R1^T and prolong(e) = P1 e P1^T.
"""
import numpy as np

from . import iterate
from .adjoint import NAGEX, _factors, reverse
from .problem import apply_A


def _coarse_size(n):
    if n < 3 or n % 2 == 0:
        raise ValueError("the fine grid needs an odd n >= 3")
    return (n - 1) // 2


def restriction_1d(n):
    """Full weighting (1/4)[1 2 1] centred on fine point 2J + 1, as an nc x n matrix."""
    nc = _coarse_size(n)
    R1 = np.zeros((nc, n))
    for J in range(nc):
        R1[J, 2 * J] = 0.25
        R1[J, 2 * J + 1] = 0.5
        R1[J, 2 * J + 2] = 0.25
    return R1


def prolongation_1d(n):
    """Linear interpolation from the coarse grid (zero outside) as an n x nc matrix."""
    nc = _coarse_size(n)
    P1 = np.zeros((n, nc))
    for j in range(n):
        if j % 2 == 1:
            P1[j, (j - 1) // 2] = 1.0
        else:
            for J in (j // 2 - 1, j // 2):
                if 0 <= J < nc:
                    P1[j, J] = 0.5
    return P1


def restrict(r):
    R1 = restriction_1d(r.shape[0])
    return R1 @ r @ R1.T


def restrict_T(c, n):
    """Transpose of restrict: fine-grid vector from a coarse one."""
    R1 = restriction_1d(n)
    return R1.T @ c @ R1


def prolong(e):
    P1 = prolongation_1d(2 * e.shape[0] + 1)
    return P1 @ e @ P1.T


def prolong_T(x):
    P1 = prolongation_1d(x.shape[0])
    return P1.T @ x @ P1


def dst_matrix(nc):
    """Orthonormal DST-I: S[j, k] = sqrt(2/(nc+1)) sin(pi (j+1)(k+1)/(nc+1)); S = S^T = S^-1."""
    j = np.arange(1, nc + 1)
    return np.sqrt(2.0 / (nc + 1)) * np.sin(np.pi * np.outer(j, j) / (nc + 1))


def transform(x):
    """2D sine transform S x S of a coarse field x[J, I] -> coefficients [q, p]."""
    S = dst_matrix(x.shape[0])
    return S @ x @ S


def coarse_correction(r, symbol):
    """P S (symbol * (S R r S)) S for a fine-grid residual r."""
    return prolong(transform(symbol * transform(restrict(r))))


def cycle(method, coef, f, u, omega, symbol, alpha=None, alpha_t=None, binv=None):
    """One two-grid cycle from u_k; returns u_{k+1}."""
    m = len(omega)
    uh, _ = iterate.run(method, coef, f, omega, m, alpha=alpha, alpha_t=alpha_t, u0=u, binv=binv)
    return uh + coarse_correction(f - apply_A(coef, uh), symbol)


def run(method, coef, f, omega, symbol, K, alpha=None, alpha_t=None, u0=None, binv=None, history=False):
    """K cycles from u0 (default 0); returns u_K [, relres after every cycle]."""
    u = np.zeros_like(f, dtype=np.float64) if u0 is None else np.array(u0, dtype=np.float64)
    fn = np.linalg.norm(f)
    hist = []
    for _ in range(K):
        u = cycle(method, coef, f, u, omega, symbol, alpha=alpha, alpha_t=alpha_t, binv=binv)
        if history:
            hist.append(np.linalg.norm(f - apply_A(coef, u)) / fn)
    return (u, np.array(hist)) if history else u


def loss_and_grads(method, coef, f, omega, symbol, K, alpha=None, alpha_t=None, dinv=1.0, u0=None, g_uK=None):
    """Reverse mode through K cycles.

    Returns (L, d_omega[m], d_alpha[m], d_alpha_t[m], d_symbol[nc, nc], d_f) for
    L = ||f - A u_K||^2 / ||f||^2, or L = <g_uK, u_K> when a seed is given.  The
    smoother's gradients follow oracle.adjoint (NAG: d_alpha + d_alpha_t is the
    gradient of its single factor).  Through one correction
    u' = u_h + P C R (f - A u_h), C = S diag(symbol) S, with adjoint ub of u':
        c_bar = P^T ub;   d_symbol += (S c_bar S) * (S R r S);
        y_bar = C c_bar;  r_bar = R^T y_bar;   f_bar += r_bar;   ub_h = ub - A r_bar.
    The smoothing restarts from v = 0, so the adjoint of that v is dropped."""
    omega = np.asarray(omega, dtype=np.float64)
    m = len(omega)
    a, at = _factors(method, alpha, alpha_t, m)
    n = f.shape[0]
    u = np.zeros_like(f, dtype=np.float64) if u0 is None else np.array(u0, dtype=np.float64)
    # forward: per cycle the smoothing states and the smoothed iterate
    segments = []
    for _ in range(K):
        us = [u]
        vs = [np.zeros_like(u)]
        for s in range(m):
            ut = us[-1] + at[s] * vs[-1]
            v = a[s] * vs[-1] + omega[s] * dinv * (f - apply_A(coef, ut))
            vs.append(v)
            us.append(us[-1] + v)
        uh = us[-1]
        r = f - apply_A(coef, uh)
        segments.append((us, vs, r))
        u = uh + coarse_correction(r, symbol)
    fn2 = float(np.sum(f * f))
    if g_uK is None:
        rK = f - apply_A(coef, u)
        L = float(np.sum(rK * rK)) / fn2
        ub = -2.0 * apply_A(coef, rK) / fn2
        fb = 2.0 * rK / fn2 - 2.0 * L * f / fn2
    else:
        L = float(np.sum(g_uK * u))
        ub = np.array(g_uK, dtype=np.float64)
        fb = np.zeros_like(f, dtype=np.float64)
    d_omega = np.zeros(m)
    d_alpha = np.zeros(m)
    d_alpha_t = np.zeros(m)
    d_symbol = np.zeros_like(symbol, dtype=np.float64)
    for us, vs, r in reversed(segments):
        c_bar = prolong_T(ub)
        g_hat = transform(c_bar)
        d_symbol += g_hat * transform(restrict(r))
        y_bar = transform(symbol * g_hat)
        r_bar = restrict_T(y_bar, n)
        fb = fb + r_bar
        ub = ub - apply_A(coef, r_bar)
        ub, _, dw, da, dat, dfb = reverse(NAGEX, coef, f, omega, us, vs, ub, np.zeros_like(ub), alpha=a,
                                          alpha_t=at, dinv=dinv)
        d_omega += dw
        d_alpha += da
        d_alpha_t += dat
        fb = fb + dfb
    return L, d_omega, d_alpha, d_alpha_t, d_symbol, fb
