"""Reverse-mode derivative of a K-step NAG-Richardson(m) unroll, test infrastructure only.

Training (§2.2, Algorithm 1, loss L2 of eq. loss-fun-relative-res) back-propagates
through K inner steps of a Table-1 scheme.  This oracle differentiates the
NAG-Richardson(m) row literally; Richardson(m) is the case alpha = 0.

Forward step s (weight index i = s mod m), from the state (u, v) before the step:
    u~ = u + alpha_i v;  r_s = f - A u~;  v' = alpha_i v + omega_i r_s;  u' = u + v'.
Reverse step, given the adjoints (ub, vb) of (u', v') and g = vb + ub:
    omega_bar_i += <g, r_s>,  rb = omega_i g,  f_bar += rb,  ut_bar = -A rb
    (A is symmetric, so A^T = A),
    alpha_bar_i += <g + ut_bar, v>,  ub <- ub + ut_bar,  vb <- alpha_i (g + ut_bar).
Terminal values for the squared relative residual L = ||f - A u_K||^2 / ||f||^2:
    ub_K = -2 A r_K / ||f||^2,  vb_K = 0,  f_bar = 2 r_K / ||f||^2 - 2 L f / ||f||^2.
A user-supplied seed g_uK replaces ub_K and the f_bar terminal term.

Forward states are simply all stored here; the GPU path recomputes them from
checkpoints, which gives the same values.
"""
import numpy as np

from .problem import apply_A


def unroll_states(coef, f, omega, alpha, K, u0=None, v0=None):
    """States (u_s, v_s) for s = 0..K of the NAG-Richardson(m) unroll."""
    m = len(omega)
    u = np.zeros_like(f, dtype=np.float64) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros_like(f, dtype=np.float64) if v0 is None else np.array(v0, dtype=np.float64)
    us, vs = [u], [v]
    for s in range(K):
        i = s % m
        ut = u + alpha[i] * v
        r = f - apply_A(coef, ut)
        v = alpha[i] * v + omega[i] * r
        u = u + v
        us.append(u)
        vs.append(v)
    return us, vs


def loss_and_grads(coef, f, omega, alpha, K, g_uK=None, u0=None, v0=None):
    """Returns (L, d_omega[m], d_alpha[m], d_f).  With g_uK given, L is <g_uK, u_K>."""
    omega = np.asarray(omega, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    m = len(omega)
    us, vs = unroll_states(coef, f, omega, alpha, K, u0, v0)
    fn2 = float(np.sum(f * f))
    if g_uK is None:
        rK = f - apply_A(coef, us[K])
        L = float(np.sum(rK * rK)) / fn2
        ub = -2.0 * apply_A(coef, rK) / fn2
        fb = 2.0 * rK / fn2 - 2.0 * L * f / fn2
    else:
        L = float(np.sum(g_uK * us[K]))
        ub = np.array(g_uK, dtype=np.float64)
        fb = np.zeros_like(f, dtype=np.float64)
    vb = np.zeros_like(f, dtype=np.float64)
    d_omega = np.zeros(m)
    d_alpha = np.zeros(m)
    for s in range(K, 0, -1):
        i = (s - 1) % m
        u, v = us[s - 1], vs[s - 1]
        r = f - apply_A(coef, u + alpha[i] * v)
        g = vb + ub
        d_omega[i] += float(np.sum(g * r))
        rb = omega[i] * g
        fb = fb + rb
        ut_bar = -apply_A(coef, rb)
        d_alpha[i] += float(np.sum((g + ut_bar) * v))
        ub = ub + ut_bar
        vb = alpha[i] * (g + ut_bar)
    return L, d_omega, d_alpha, fb
