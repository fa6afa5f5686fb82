"""Long-step iterations of Table 1 (tb:optimization-iterative-method), test infrastructure only.

Every scheme runs in the paper's three-vector form: inner steps i = 1..m make one
outer iteration, the weights are used in the order omega_1 first (eq.
Chebyshev(m)T: T_m = (I - omega_m A) ... (I - omega_1 A)), and u, v carry over
from one outer iteration to the next (u^0_{k+1} = u^m_k, v^0_{k+1} = v^m_k).

Readings where the paper is silent: the initial momentum is v_0 = 0 (u_0 = 0 is
stated in §2.3); the residual history is taken at u (not at the look-ahead point)
after every outer iteration; "iterations" in the paper's tables count outer
iterations.

An optional preconditioner ``binv`` (a callable r -> B^{-1} r) gives the
preconditioned variants of §2.1 (eq. momentum-m-Binv); ``None`` means B^{-1} = I.
"""
import numpy as np

from .problem import apply_A

RICHARDSON, MOM, NAG, NAGEX = "richardson", "mom", "nag", "nagex"


def _inner_step(method, coef, f, u, v, w, a, at, binv):
    """One inner step i of the chosen Table-1 scheme; returns (u^i, v^i)."""
    pre = (lambda r: r) if binv is None else binv
    if method == RICHARDSON:
        # v^i = w_i (f - A u^{i-1});  u^i = u^{i-1} + v^i
        v_new = w * pre(f - apply_A(coef, u))
    elif method == MOM:
        # v^i = a_i v^{i-1} + w_i (f - A u^{i-1});  u^i = u^{i-1} + v^i
        v_new = a * v + w * pre(f - apply_A(coef, u))
    elif method == NAG:
        # look-ahead u~ = u^{i-1} + a_i v^{i-1};  v^i = a_i v^{i-1} + w_i (f - A u~)
        u_look = u + a * v
        v_new = a * v + w * pre(f - apply_A(coef, u_look))
    elif method == NAGEX:
        # look-ahead with its own factor a~_i; momentum with a_i
        u_look = u + at * v
        v_new = a * v + w * pre(f - apply_A(coef, u_look))
    else:
        raise ValueError(method)
    return u + v_new, v_new


def run(method, coef, f, omega, K, alpha=None, alpha_t=None, u0=None, v0=None, binv=None,
        history=False):
    """Run K inner steps (step s uses weight index (s mod m)); returns (u, v[, hist]).

    ``hist`` holds ||f - A u|| / ||f|| after every completed outer iteration.
    """
    m = len(omega)
    u = np.zeros_like(f, dtype=np.float64) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros_like(f, dtype=np.float64) if v0 is None else np.array(v0, dtype=np.float64)
    alpha = np.zeros(m) if alpha is None else np.asarray(alpha, dtype=np.float64)
    alpha_t = alpha if alpha_t is None else np.asarray(alpha_t, dtype=np.float64)
    fn = np.linalg.norm(f)
    hist = []
    for s in range(K):
        i = s % m
        u, v = _inner_step(method, coef, f, u, v, omega[i], alpha[i], alpha_t[i], binv)
        if history and i == m - 1:
            hist.append(np.linalg.norm(f - apply_A(coef, u)) / fn)
    if history:
        return u, v, np.array(hist)
    return u, v


def solve_to_tol(method, coef, f, omega, tol, max_outer, alpha=None, alpha_t=None, binv=None,
                 u0=None):
    """Evaluation procedure of §2.2: iterate whole outer iterations until relres < tol.

    Returns (u, outer_iterations, history); outer_iterations = max_outer + 1 when
    the cap was reached without convergence.
    """
    m = len(omega)
    u = np.zeros_like(f, dtype=np.float64) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros_like(f, dtype=np.float64)
    fn = np.linalg.norm(f)
    hist = []
    for k in range(1, max_outer + 1):
        u, v = run(method, coef, f, omega, m, alpha=alpha, alpha_t=alpha_t, u0=u, v0=v, binv=binv)
        rho = np.linalg.norm(f - apply_A(coef, u)) / fn
        hist.append(rho)
        if not np.isfinite(rho):
            break
        if rho < tol:
            return u, k, np.array(hist)
    return u, max_outer + 1, np.array(hist)
