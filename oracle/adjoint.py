"""Reverse-mode derivative of a K-step unroll of the Table-1 schemes, test infrastructure only.

Training (§2.2, Algorithm 1, loss L2 of eq. loss-fun-relative-res) back-propagates
through K inner steps of a Table-1 scheme.  This oracle differentiates the
NAGex-Richardson(m) row literally; the other rows are its special cases:
NAG (look-ahead factor equal to the momentum factor), MOM (no look-ahead) and
Richardson (no momentum).  A preconditioner (§2.1, eq. momentum-m-Binv) enters as
B^{-1} applied to the residual: a constant-diagonal weighted Jacobi scale dinv = 1/D,
or any symmetric B^{-1} passed as a callable `binv` (SSOR is symmetric when A is).

Forward step s (weight index i = s mod m), from the state (u, v) before the step:
    u~ = u + at_i v;  r_s = f - A u~;  v' = a_i v + omega_i B^{-1} r_s;  u' = u + v'.
Reverse step, given the adjoints (ub, vb) of (u', v') and g = vb + ub:
    omega_bar_i += <g, B^{-1} r_s>,  rb = omega_i B^{-1} g,  f_bar += rb,  ut_bar = -A rb
    (A and B^{-1} are symmetric),
    alpha_bar_i += <g, v>,  alpha_t_bar_i += <ut_bar, v>,
    ub <- ub + ut_bar,  vb <- a_i g + at_i ut_bar.
For NAG the two momentum gradients add up: alpha_bar_i = <g + ut_bar, v>.
Terminal values for the squared relative residual L = ||f - A u_K||^2 / ||f||^2:
    ub_K = -2 A r_K / ||f||^2,  vb_K = 0,  f_bar = 2 r_K / ||f||^2 - 2 L f / ||f||^2.
A user-supplied seed g_uK replaces ub_K and the f_bar terminal term.

Forward states are simply all stored here; the GPU path recomputes them from
checkpoints, which gives the same values.
"""
import numpy as np

from .problem import apply_A

RICHARDSON, MOM, NAG, NAGEX = "richardson", "mom", "nag", "nagex"


def _factors(method, alpha, alpha_t, m):
    z = np.zeros(m)
    if method == RICHARDSON:
        return z, z
    a = np.asarray(alpha, dtype=np.float64)
    if method == MOM:
        return a, z
    if method == NAG:
        return a, a
    if method == NAGEX:
        return a, np.asarray(alpha_t, dtype=np.float64)
    raise ValueError(method)


def _precond(dinv, binv):
    return (lambda r: dinv * r) if binv is None else binv


def unroll_states(coef, f, omega, alpha, K, u0=None, v0=None, method=NAG, alpha_t=None, dinv=1.0, binv=None):
    """States (u_s, v_s) for s = 0..K of the unroll."""
    m = len(omega)
    a, at = _factors(method, alpha, alpha_t, m)
    pre = _precond(dinv, binv)
    u = np.zeros_like(f, dtype=np.float64) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros_like(f, dtype=np.float64) if v0 is None else np.array(v0, dtype=np.float64)
    us, vs = [u], [v]
    for s in range(K):
        i = s % m
        ut = u + at[i] * v
        r = f - apply_A(coef, ut)
        v = a[i] * v + omega[i] * pre(r)
        u = u + v
        us.append(u)
        vs.append(v)
    return us, vs


def reverse(method, coef, f, omega, us, vs, ub, vb, alpha=None, alpha_t=None, dinv=1.0, binv=None):
    """Reverse sweep over a stored unroll (us[0..K], vs[0..K]) from the adjoints (ub, vb)
    of (u_K, v_K).  Returns (ub_0, vb_0, d_omega, d_alpha, d_alpha_t, f_bar increment)."""
    omega = np.asarray(omega, dtype=np.float64)
    m = len(omega)
    a, at = _factors(method, alpha, alpha_t, m)
    pre = _precond(dinv, binv)
    K = len(us) - 1
    ub = np.array(ub, dtype=np.float64)
    vb = np.array(vb, dtype=np.float64)
    fb = np.zeros_like(ub)
    d_omega = np.zeros(m)
    d_alpha = np.zeros(m)
    d_alpha_t = np.zeros(m)
    for s in range(K, 0, -1):
        i = (s - 1) % m
        u, v = us[s - 1], vs[s - 1]
        r = f - apply_A(coef, u + at[i] * v)
        g = vb + ub
        d_omega[i] += float(np.sum(g * pre(r)))
        rb = omega[i] * pre(g)
        fb = fb + rb
        ut_bar = -apply_A(coef, rb)
        d_alpha[i] += float(np.sum(g * v))
        d_alpha_t[i] += float(np.sum(ut_bar * v))
        ub = ub + ut_bar
        vb = a[i] * g + at[i] * ut_bar
    return ub, vb, d_omega, d_alpha, d_alpha_t, fb


def loss_and_grads_general(method, coef, f, omega, K, alpha=None, alpha_t=None, dinv=1.0, g_uK=None, binv=None):
    """Returns (L, d_omega[m], d_alpha[m], d_alpha_t[m], d_f).

    With g_uK given, L is <g_uK, u_K>.  d_alpha is the gradient through the momentum
    term and d_alpha_t through the look-ahead; for NAG the gradient with respect to
    its single factor is d_alpha + d_alpha_t."""
    omega = np.asarray(omega, dtype=np.float64)
    m = len(omega)
    a, at = _factors(method, alpha, alpha_t, m)
    us, vs = unroll_states(coef, f, omega, a, K, method=NAGEX, alpha_t=at, dinv=dinv, binv=binv)
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
    _, _, d_omega, d_alpha, d_alpha_t, dfb = reverse(NAGEX, coef, f, omega, us, vs, ub, vb, alpha=a,
                                                     alpha_t=at, dinv=dinv, binv=binv)
    return L, d_omega, d_alpha, d_alpha_t, fb + dfb


def loss_and_grads(coef, f, omega, alpha, K, g_uK=None, u0=None, v0=None):
    """NAG-Richardson(m): returns (L, d_omega[m], d_alpha[m], d_f)."""
    if u0 is not None or v0 is not None:
        raise NotImplementedError("the unroll starts from u = v = 0")
    L, dw, da, dat, df = loss_and_grads_general(NAG, coef, f, omega, K, alpha=alpha, g_uK=g_uK)
    return L, dw, da + dat, df
