"""Pins for the oracle's iterations, weights and refinement (CPU only)."""
import json
import os

import numpy as np
import pytest
import scipy.fft

from oracle import iterate, problem, refine, spectra, weights
from tests.test_oracle_problem import q1_assembled_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cheb_T(m, x):
    """Chebyshev polynomial of the first kind through its trigonometric/hyperbolic closed form."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(m * np.arccos(x[inside]))
    big = ~inside
    out[big] = np.sign(x[big]) ** m * np.cosh(m * np.arccosh(np.abs(x[big])))
    return out


@pytest.mark.parametrize("m", [1, 3, 8, 16])
def test_chebyshev_residual_polynomial(m):
    # prod (1 - w_i lam) = T_m((lmax + lmin - 2 lam)/(lmax - lmin)) / T_m(sigma)
    lmin, lmax = 0.0048, 3.9968
    w = weights.chebyshev_weights(lmin, lmax, m)
    lam = np.linspace(lmin, lmax, 997)
    sigma = (lmax + lmin) / (lmax - lmin)
    want = cheb_T(m, (lmax + lmin - 2 * lam) / (lmax - lmin)) / cheb_T(m, np.array([sigma]))[0]
    assert np.max(np.abs(weights.cycle_polynomial(w, lam) - want)) < 1e-9
    # nodes 1/w_i are the mapped Chebyshev roots and lie inside the spectrum interval
    assert np.all((1 / w > lmin) & (1 / w < lmax))


@pytest.mark.parametrize("m", [4, 8, 16])
def test_semi_iteration_weights_equioscillate_on_the_assumed_interval(m):
    # with lmin := lmax / 30 the cycle polynomial is the Chebyshev minimax polynomial on
    # [lmax / 30, lmax]: it takes the values (-1)^k / T_m(31 / 29) at the m + 1 mapped
    # extrema x_k = cos(k pi / m) and never exceeds that magnitude in between
    lmax = 3.9968
    lmin = lmax / 30.0
    w = weights.semi_iteration_weights(lmax, m)
    bound = 1.0 / cheb_T(m, np.array([31.0 / 29.0]))[0]
    k = np.arange(m + 1)
    lam_k = (lmax + lmin - np.cos(k * np.pi / m) * (lmax - lmin)) / 2.0
    assert np.allclose(weights.cycle_polynomial(w, lam_k), bound * (-1.0) ** k, rtol=1e-10, atol=0.0)
    lam = np.linspace(lmin, lmax, 4001)
    assert np.max(np.abs(weights.cycle_polynomial(w, lam))) <= bound * (1 + 1e-10)
    # outside the assumed interval, below lmin, the polynomial exceeds the bound
    assert weights.cycle_polynomial(w, np.array([lmin / 4]))[0] > bound


def test_lowest_mode_decays_at_chebyshev_rate():
    # f = phi_11 (lowest mode): every cycle multiplies the residual by exactly 1/T_8(sigma)
    n, m = 63, 8
    coef = problem.q1_stencil(1.0, 0.0)
    lmin, lmax = spectra.q1_extreme_eigenvalues(1.0, 0.0, n)
    w = weights.chebyshev_weights(lmin, lmax, m)
    f = spectra.sine_mode(n, 1, 1)
    _, _, hist = iterate.run(iterate.RICHARDSON, coef, f, w, 10 * m, history=True)
    sigma = (lmax + lmin) / (lmax - lmin)
    rate = 1.0 / np.cosh(m * np.arccosh(sigma))
    assert np.allclose(hist, rate ** np.arange(1, 11), rtol=1e-9)


def test_single_isotropic_run_matches_spectral_closed_form():
    # eps = 1, n = 63, f ~ N(0, I) seed 0, Richardson(8) with exact Chebyshev weights:
    # r_K = sum_pq fhat_pq P(lambda_pq)^(K/m) phi_pq, evaluated with the orthonormal DST-I
    n, m = 63, 8
    coef = problem.q1_stencil(1.0, 0.0)
    f = np.random.default_rng(0).standard_normal((n, n))
    lam = spectra.q1_eigenvalues(1.0, 0.0, n)
    w = weights.chebyshev_weights(lam.min(), lam.max(), m)
    fhat = scipy.fft.dstn(f, type=1, norm="ortho")
    P = weights.cycle_polynomial(w, lam)
    _, _, hist = iterate.run(iterate.RICHARDSON, coef, f, w, 50 * m, history=True)
    for k in (1, 10, 50):
        want = np.linalg.norm(fhat * P ** k) / np.linalg.norm(f)
        assert abs(hist[k - 1] - want) <= 1e-9 * want


def test_table2_chebyshev_row_counts():
    """Paper Table 2, 'Chebyshev iteration (m=3)': outer iterations to relres < 1e-6."""
    with open(os.path.join(GOLDEN, "table2_chebyshev_row.json")) as fh:
        g = json.load(fh)
    n, m = 64, 3
    f = np.random.default_rng(0).standard_normal((n, n))
    for eps, paper in zip(g["eps"], g["outer_iterations"]):
        coef = problem.q1_stencil(eps, 0.0)
        lmin, lmax = spectra.q1_extreme_eigenvalues(eps, 0.0, n)
        w = weights.chebyshev_weights(lmin, lmax, m)
        _, k, _ = iterate.solve_to_tol(iterate.RICHARDSON, coef, f, w, 1e-6, 2 * paper)
        # a different draw of f moves the count by a few percent (the paper's f is unseeded)
        assert abs(k - paper) <= 0.03 * paper, (eps, k, paper)


def _small(seed=1, n=7, eps=0.05, theta=0.7):
    rng = np.random.default_rng(seed)
    return problem.q1_stencil(eps, theta), rng.standard_normal((n, n)), rng


def test_degenerate_schemes():
    coef, f, rng = _small()
    m, K = 4, 12
    w = rng.uniform(0.1, 0.35, m)
    a = rng.uniform(0.2, 0.9, m)
    at = rng.uniform(0.2, 0.9, m)
    z = np.zeros(m)
    u_r, _ = iterate.run(iterate.RICHARDSON, coef, f, w, K)
    for meth in (iterate.MOM, iterate.NAG):
        u, _ = iterate.run(meth, coef, f, w, K, alpha=z)
        assert np.allclose(u, u_r, rtol=0, atol=1e-13)
    # NAGex with alpha~ = alpha is NAG; with alpha~ = 0 the look-ahead vanishes, which is MOM
    u_nag, v_nag = iterate.run(iterate.NAG, coef, f, w, K, alpha=a)
    u_ex, v_ex = iterate.run(iterate.NAGEX, coef, f, w, K, alpha=a, alpha_t=a)
    assert np.array_equal(u_nag, u_ex) and np.array_equal(v_nag, v_ex)
    u_mom, _ = iterate.run(iterate.MOM, coef, f, w, K, alpha=a)
    u_ex0, _ = iterate.run(iterate.NAGEX, coef, f, w, K, alpha=a, alpha_t=z)
    assert np.allclose(u_mom, u_ex0, atol=1e-13)
    # NAG differs from MOM once alpha != 0
    assert np.max(np.abs(u_nag - u_mom)) > 1e-3
    # a NAGex run with a different look-ahead differs from NAG
    u_ex2, _ = iterate.run(iterate.NAGEX, coef, f, w, K, alpha=a, alpha_t=at)
    assert np.max(np.abs(u_ex2 - u_nag)) > 1e-3


def test_richardson_m_matrix_form():
    # one outer iteration equals T_m u + g with T_m = (I - w_m A)...(I - w_1 A) and
    # g = (w_m + sum_{j<m} prod_{i>j} (I - w_i A) w_j) f   (eq. Chebyshev(m)T, Chebyshev(m)f)
    eps, theta, n = 0.05, 0.7, 6
    coef = problem.q1_stencil(eps, theta)
    A = q1_assembled_matrix(eps, theta, n)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(n * n)
    u0 = rng.standard_normal(n * n)
    m = 5
    w = rng.uniform(0.1, 0.6, m)
    I = np.eye(n * n)
    T = I.copy()
    for i in range(m):
        T = (I - w[i] * A) @ T
    G = w[m - 1] * I
    for j in range(m - 1):
        P = I.copy()
        for i in range(j + 1, m):
            P = (I - w[i] * A) @ P
        G = G + w[j] * P
    want = T @ u0 + G @ f
    got, _ = iterate.run(iterate.RICHARDSON, coef, f.reshape(n, n), w, m, u0=u0.reshape(n, n))
    assert np.allclose(got.ravel(), want, atol=1e-12)


def test_m1_is_classical_richardson():
    # eq. richard: u_k = (I - w A) u_{k-1} + w f  (k steps from zero = sum_j (I - wA)^j w f)
    eps, theta, n = 0.3, 0.2, 5
    A = q1_assembled_matrix(eps, theta, n)
    f = np.random.default_rng(2).standard_normal(n * n)
    w, K = 0.31, 17
    M = np.eye(n * n) - w * A
    want = sum(np.linalg.matrix_power(M, j) @ (w * f) for j in range(K))
    got, _ = iterate.run(iterate.RICHARDSON, problem.q1_stencil(eps, theta), f.reshape(n, n), [w], K)
    assert np.allclose(got.ravel(), want, atol=1e-12)


def test_cycle_invariance():
    coef, f, rng = _small(seed=3)
    lam = np.linalg.eigvalsh(q1_assembled_matrix(0.05, 0.7, 7))
    w = weights.chebyshev_weights(lam.min(), lam.max(), 6)
    u1, _ = iterate.run(iterate.RICHARDSON, coef, f, w, 6 * 4)
    u2, _ = iterate.run(iterate.RICHARDSON, coef, f, rng.permutation(w), 6 * 4)
    u3, _ = iterate.run(iterate.RICHARDSON, coef, f, weights.leja_order(w), 6 * 4)
    assert np.allclose(u1, u2, rtol=1e-11, atol=1e-11)
    assert np.allclose(u1, u3, rtol=1e-11, atol=1e-11)
    assert sorted(weights.leja_order(w)) == sorted(w)


@pytest.mark.parametrize("alpha,omega_scale", [(0.5, 0.9), (0.95, 1.0), (0.99, 0.3), (0.0, 0.7)])
def test_nag_on_an_eigenmode_matches_two_root_closed_form(alpha, omega_scale):
    # f = phi (eigenvalue lam), constant weights: u_s = c_s phi with e_s = c_s - 1/lam obeying
    # e_{s+1} = (1 + a)(1 - q) e_s - a (1 - q) e_{s-1}, q = w lam; e_0 = -1/lam, e_1 = (1 - q) e_0.
    n = 15
    eps, theta = 1e-2, 0.0
    coef = problem.q1_stencil(eps, theta)
    lam_all = spectra.q1_eigenvalues(eps, theta, n)
    p, q_ = 2, 3
    lam = lam_all[q_ - 1, p - 1]
    phi = spectra.sine_mode(n, p, q_)
    w = omega_scale / lam_all.max()
    K = 40
    u, _ = iterate.run(iterate.NAG, coef, phi, [w], K, alpha=[alpha])
    c = np.sum(u * phi) / np.sum(phi * phi)
    qq = w * lam
    roots = np.roots([1.0, -(1 + alpha) * (1 - qq), alpha * (1 - qq)]).astype(complex)
    e0 = -1.0 / lam
    e1 = (1 - qq) * e0
    if abs(roots[0] - roots[1]) < 1e-12:
        z = roots[0]
        B = (e1 - e0 * z) / z
        eK = (e0 + B * K) * z ** K
    else:
        z1, z2 = roots
        A2 = (e1 - e0 * z1) / (z2 - z1)
        A1 = e0 - A2
        eK = A1 * z1 ** K + A2 * z2 ** K
    assert abs(c - (1.0 / lam + eK.real)) < 1e-10 * abs(1.0 / lam)
    assert abs(eK.imag) < 1e-12 / lam


def test_refinement_equals_plain_for_richardson_m():
    coef, f, _ = _small(seed=4)
    lam = np.linalg.eigvalsh(q1_assembled_matrix(0.05, 0.7, 7))
    m = 4
    w = weights.chebyshev_weights(lam.min(), lam.max(), m)
    x, rounds, rhos, inner = refine.refined_solve(iterate.RICHARDSON, coef, f, w, tol=1e-11,
                                                  tol_inner=1e-3)
    assert rounds >= 2 and rhos[-1] <= 1e-11
    u, _ = iterate.run(iterate.RICHARDSON, coef, f, w, m * sum(inner))
    assert np.max(np.abs(x - u)) <= 1e-12 * np.max(np.abs(u))


def test_refined_solve_matches_direct_solve():
    eps, theta, n = 1e-3, 1.3, 7
    coef = problem.q1_stencil(eps, theta)
    A = q1_assembled_matrix(eps, theta, n)
    lam = np.linalg.eigvalsh(A)
    b = np.random.default_rng(11).standard_normal((n, n))
    xs = np.linalg.solve(A, b.ravel()).reshape(n, n)
    kappa = lam.max() / lam.min()
    w = weights.chebyshev_weights(lam.min(), lam.max(), 8)
    runs = [(iterate.RICHARDSON, w, None),
            (iterate.NAG, np.full(4, 1.0 / lam.max()), np.full(4, 0.9))]
    for meth, om, al in runs:
        x, rounds, rhos, _ = refine.refined_solve(meth, coef, b, om, tol=1e-13, alpha=al)
        assert rhos[-1] <= 1e-13
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-13


def test_amplification_diagnostic():
    n, m = 63, 8
    lmin, lmax = spectra.q1_extreme_eigenvalues(1.0, 0.0, n)
    w = weights.chebyshev_weights(lmin, lmax, m)
    nat = weights.amplification(w, lmin, lmax)
    lej = weights.amplification(weights.leja_order(w), lmin, lmax)
    # the last factor alone reaches |1 - w_m lmax| for ascending weights
    assert nat >= abs(1 - w[-1] * lmax) - 1e-12
    assert lej < nat
    assert weights.amplification([0.5 / lmax], lmin, lmax) == 1.0


def test_amplification_closed_form_two_weights():
    # m = 2: the tail after step 1 is |1 - w2 lam|, linear in lam, so its maximum over
    # [lmin, lmax] sits at an end; after step 2 the tail is empty (factor 1).  With w2 = 0.5
    # on [1, 10] that is |1 - 5| = 4.  The whole product (1 - 0.3 lam)(1 - 0.5 lam) reaches
    # 8 at lam = 10, so a tail that wrongly starts at step j instead of j + 1 reads 8.
    assert abs(weights.amplification([0.3, 0.5], 1.0, 10.0) - 4.0) < 1e-12


def test_amplification_closed_form_three_weights():
    # m = 3, w = (0.5, 1.0, 0.1) on [0.2, 9]:
    #   tail after step 1: q(lam) = (1 - lam)(1 - 0.1 lam), vertex at lam = 1.1 / 0.2 = 5.5
    #     where |q| = 4.5 * 0.45 = 2.025; at the ends 0.784 and 0.8;
    #   tail after step 2: |1 - 0.1 lam| <= 0.98;  after step 3: 1.
    # The full product (one step too many) reaches 3.5 * 8 * 0.1 = 2.8 at lam = 9.
    got = weights.amplification([0.5, 1.0, 0.1], 0.2, 9.0)
    assert abs(got - 2.025) < 1e-7


def test_leja_order_hand_computed():
    # nodes 1/w = {1, 2, 4, 8}: start at 8; then the farthest from 8 is 1 (distance 7);
    # then products |x - 8||x - 1|: 2 -> 6, 4 -> 12, so 4; then 2.
    got = weights.leja_order([0.5, 0.125, 1.0, 0.25])
    assert np.array_equal(1.0 / np.asarray(got), [8.0, 1.0, 4.0, 2.0])
    # nodes {0.5, 1.5, 2, 7, 9}: 9; 0.5 (8.5); products with {9, 0.5}: 1.5 -> 7.5,
    # 2 -> 10.5, 7 -> 13, so 7; with {9, 0.5, 7}: 1.5 -> 41.25, 2 -> 52.5, so 2; then 1.5.
    nodes = np.array([2.0, 9.0, 0.5, 1.5, 7.0])
    got = weights.leja_order(1.0 / nodes)
    assert np.allclose(1.0 / np.asarray(got), [9.0, 0.5, 7.0, 2.0, 1.5], rtol=0, atol=1e-12)
