"""Pins of the two-grid oracle (CPU): transfer operators against exactness and sine-mode
closed forms, the sine transform against scipy and the coarse spectrum, the correction
against a dense coarse solve, the cycle against its dense error propagator, and the
adjoint against finite differences and autograd of an independent torch version."""
import numpy as np
import pytest
import scipy.fft
import torch

from oracle import problem, spectra, twogrid
from oracle.weights import chebyshev_weights


def _grid(n):
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    return x, h


def _dense(coef, n):
    A = np.zeros((n * n, n * n))
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        A[:, k] = problem.apply_A(coef, e.reshape(n, n)).ravel()
    return A


@pytest.mark.parametrize("n", [7, 15, 31])
def test_restriction_reproduces_bilinear_functions(n):
    x, _ = _grid(n)
    X, Y = np.meshgrid(x, x)  # X[j, i] = x_i, Y[j, i] = y_j
    g = lambda X, Y: 0.3 + 1.7 * X - 0.4 * Y + 2.5 * X * Y
    xc = x[1::2]
    Xc, Yc = np.meshgrid(xc, xc)
    np.testing.assert_allclose(twogrid.restrict(g(X, Y)), g(Xc, Yc), rtol=0, atol=1e-14)


@pytest.mark.parametrize("n,p,q", [(15, 1, 1), (15, 3, 5), (31, 7, 2), (31, 15, 15)])
def test_restriction_on_sine_modes(n, p, q):
    """Full weighting maps the fine mode (p, q) to cos^2(p pi h/2) cos^2(q pi h/2) times
    the coarse mode (p, q)."""
    nc = (n - 1) // 2
    _, h = _grid(n)
    fine = spectra.sine_mode(n, p, q)
    coarse = spectra.sine_mode(nc, p, q)
    fac = np.cos(p * np.pi * h / 2) ** 2 * np.cos(q * np.pi * h / 2) ** 2
    np.testing.assert_allclose(twogrid.restrict(fine), fac * coarse, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [7, 15, 31])
def test_prolongation_interpolates_xy_exactly(n):
    """x*y vanishes on x = 0 and y = 0, so linear interpolation reproduces it on every
    fine point whose coarse neighbours lie inside the grid or on those two edges."""
    x, _ = _grid(n)
    xc = x[1::2]
    Xc, Yc = np.meshgrid(xc, xc)
    X, Y = np.meshgrid(x, x)
    e = twogrid.prolong(Xc * Yc)
    np.testing.assert_allclose(e[: n - 1, : n - 1], (X * Y)[: n - 1, : n - 1], rtol=0, atol=1e-14)
    # the coarse points themselves are copied
    np.testing.assert_array_equal(e[1::2, 1::2], Xc * Yc)


def test_prolongation_is_four_times_restriction_transpose():
    rng = np.random.default_rng(0)
    n = 15
    c = rng.standard_normal((7, 7))
    np.testing.assert_allclose(twogrid.prolong(c), 4.0 * twogrid.restrict_T(c, n), rtol=0, atol=1e-15)


def test_transposes_are_adjoints():
    rng = np.random.default_rng(1)
    n = 31
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((15, 15))
    assert abs(np.sum(twogrid.restrict(x) * y) - np.sum(x * twogrid.restrict_T(y, n))) < 1e-12
    assert abs(np.sum(twogrid.prolong(y) * x) - np.sum(y * twogrid.prolong_T(x))) < 1e-12


@pytest.mark.parametrize("nc", [3, 7, 15, 255])
def test_dst_matrix_matches_scipy_and_is_involutory(nc):
    rng = np.random.default_rng(nc)
    x = rng.standard_normal((nc, nc))
    want = scipy.fft.dstn(x, type=1, norm="ortho")
    np.testing.assert_allclose(twogrid.transform(x), want, rtol=0, atol=1e-12)
    S = twogrid.dst_matrix(nc)
    np.testing.assert_allclose(S @ S, np.eye(nc), rtol=0, atol=1e-12)


@pytest.mark.parametrize("kappa", [0.0, 7.0])
def test_sine_transform_diagonalises_coarse_helmholtz(kappa):
    nc = 15
    rng = np.random.default_rng(2)
    x = rng.standard_normal((nc, nc))
    coef = problem.helmholtz_stencil(kappa, nc)
    lam = spectra.helmholtz_eigenvalues(kappa, nc)
    np.testing.assert_allclose(twogrid.transform(problem.apply_A(coef, x)), lam * twogrid.transform(x),
                               rtol=1e-12, atol=1e-9)


def test_correction_with_inverse_symbol_is_a_coarse_solve():
    n, kappa = 31, 9.0
    nc = 15
    rng = np.random.default_rng(3)
    r = rng.standard_normal((n, n))
    symbol = 1.0 / spectra.helmholtz_eigenvalues(kappa, nc)
    Ac = _dense(problem.helmholtz_stencil(kappa, nc), nc)
    ec = np.linalg.solve(Ac, twogrid.restrict(r).ravel()).reshape(nc, nc)
    np.testing.assert_allclose(twogrid.coarse_correction(r, symbol), twogrid.prolong(ec), rtol=1e-11, atol=1e-13)


def test_cycle_matches_dense_error_propagator():
    """u_{k+1} - u* = (I - P Ac^{-1} R A) prod_i (I - omega_i A) (u_k - u*) for Richardson
    smoothing and the exact coarse inverse, with every matrix assembled densely."""
    n, kappa = 15, 5.0
    nc = 7
    coef = problem.helmholtz_stencil(kappa, n)
    A = _dense(coef, n)
    Ac = _dense(problem.helmholtz_stencil(kappa, nc), nc)
    Rd = np.kron(twogrid.restriction_1d(n), twogrid.restriction_1d(n))
    Pd = np.kron(twogrid.prolongation_1d(n), twogrid.prolongation_1d(n))
    rng = np.random.default_rng(4)
    f = rng.standard_normal((n, n))
    u0 = rng.standard_normal((n, n))
    omega = rng.uniform(0.3, 1.0, 3) / problem.gershgorin(coef)
    symbol = 1.0 / spectra.helmholtz_eigenvalues(kappa, nc)
    ustar = np.linalg.solve(A, f.ravel())
    Sm = np.eye(n * n)
    for w in omega:
        Sm = (np.eye(n * n) - w * A) @ Sm
    E = (np.eye(n * n) - Pd @ np.linalg.solve(Ac, Rd @ A)) @ Sm
    u1 = twogrid.cycle("richardson", coef, f, u0, omega, symbol)
    np.testing.assert_allclose(u1.ravel() - ustar, E @ (u0.ravel() - ustar), rtol=1e-10, atol=1e-10)


def test_poisson_two_grid_contracts():
    """Two-grid for the Laplacian with a Chebyshev smoother on the upper quarter of the
    spectrum and the exact coarse inverse reduces the residual by > 10x per cycle."""
    n = 63
    coef = problem.helmholtz_stencil(0.0, n)
    lmax = problem.gershgorin(coef)
    omega = chebyshev_weights(lmax / 4, lmax, 4)
    symbol = 1.0 / spectra.helmholtz_eigenvalues(0.0, 31)
    f = np.random.default_rng(5).standard_normal((n, n))
    _, hist = twogrid.run("richardson", coef, f, omega, symbol, 6, history=True)
    assert np.all(hist[1:] / hist[:-1] < 0.1), hist


def _case(method, jacobi, seed=6):
    n, kappa, m = 15, 6.0, 3
    nc = 7
    coef = problem.helmholtz_stencil(kappa, n)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n))
    scale = coef[0] if jacobi else 1.0
    omega = rng.uniform(0.3, 0.9, m) / problem.gershgorin(coef) * scale
    alpha = rng.uniform(0.1, 0.5, m)
    alpha_t = rng.uniform(0.1, 0.5, m)
    lam = spectra.helmholtz_eigenvalues(kappa, nc)
    symbol = (1.0 / lam) * rng.uniform(0.8, 1.2, lam.shape)
    dinv = 1.0 / coef[0] if jacobi else 1.0
    return coef, f, omega, alpha, alpha_t, symbol, dinv


@pytest.mark.parametrize("method,jacobi", [("nag", False), ("nagex", True), ("mom", False), ("richardson", True)])
def test_twogrid_adjoint_finite_differences(method, jacobi):
    coef, f, omega, alpha, alpha_t, symbol, dinv = _case(method, jacobi)
    K = 2
    L, dw, da, dat, dsym, df = twogrid.loss_and_grads(method, coef, f, omega, symbol, K, alpha=alpha,
                                                      alpha_t=alpha_t, dinv=dinv)
    binv = (lambda r: r * dinv) if jacobi else None

    def loss(omega=omega, alpha=alpha, alpha_t=alpha_t, symbol=symbol, f=f):
        u = twogrid.run(method, coef, f, omega, symbol, K, alpha=alpha, alpha_t=alpha_t, binv=binv)
        r = f - problem.apply_A(coef, u)
        return np.sum(r * r) / np.sum(f * f)

    assert abs(loss() - L) <= 1e-12 * L
    d = 1e-6

    def cd(fun, x0, idx):
        xp = x0.copy()
        xm = x0.copy()
        xp[idx] += d * max(1.0, abs(x0[idx]))
        xm[idx] -= d * max(1.0, abs(x0[idx]))
        return (fun(xp) - fun(xm)) / (xp[idx] - xm[idx])

    for i in range(len(omega)):
        w_scale = 1e-4 * np.max(np.abs(dw)) + 1e-12
        assert abs(cd(lambda w: loss(omega=w), omega, i) - dw[i]) <= w_scale
    if method != "richardson":
        for i in range(len(alpha)):
            if method == "nag":
                got = cd(lambda a: loss(alpha=a, alpha_t=a), alpha, i)
                want = da[i] + dat[i]
            else:
                got = cd(lambda a: loss(alpha=a), alpha, i)
                want = da[i]
            assert abs(got - want) <= 1e-4 * np.max(np.abs(da)) + 1e-10
        if method == "nagex":
            for i in range(len(alpha_t)):
                assert abs(cd(lambda a: loss(alpha_t=a), alpha_t, i) - dat[i]) <= 1e-4 * np.max(np.abs(dat)) + 1e-10
    for idx in [(0, 0), (3, 5), (6, 6), (2, 1)]:
        got = cd(lambda s: loss(symbol=s), symbol, idx)
        assert abs(got - dsym[idx]) <= 1e-4 * np.max(np.abs(dsym)) + 1e-12, idx
    for idx in [(0, 0), (7, 7), (14, 3)]:
        got = cd(lambda g: loss(f=g), f, idx)
        assert abs(got - df[idx]) <= 1e-4 * np.max(np.abs(df)) + 1e-12, idx


def _torch_cycle_loss(coef, f, omega, alpha, alpha_t, symbol, K, n):
    """Independent torch version: stencils as conv2d, full weighting as a stride-2
    conv2d, interpolation as a stride-2 transposed conv2d, the sine transform through
    the FFT of the odd extension."""
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float64)
    c = coef
    k = torch.zeros(1, 1, 3, 3, dtype=torch.float64)
    k[0, 0, 1, 1] = c[0]
    k[0, 0, 1, 0] = k[0, 0, 1, 2] = c[1]
    k[0, 0, 0, 1] = k[0, 0, 2, 1] = c[2]
    k[0, 0, 0, 0] = k[0, 0, 2, 2] = c[3]
    k[0, 0, 0, 2] = k[0, 0, 2, 0] = c[4]
    A = lambda x: torch.nn.functional.conv2d(x[None, None], k, padding=1)[0, 0]
    fw = t([[1, 2, 1], [2, 4, 2], [1, 2, 1]])[None, None] / 16.0
    R = lambda x: torch.nn.functional.conv2d(x[None, None], fw, stride=2)[0, 0]
    P = lambda e: torch.nn.functional.conv_transpose2d(e[None, None], 4.0 * fw, stride=2)[0, 0]
    nc = (n - 1) // 2

    def dst(x, dim):
        x = x.movedim(dim, -1)
        z = torch.zeros(x.shape[:-1] + (1,), dtype=x.dtype)
        ext = torch.cat([z, x, z, -x.flip(-1)], dim=-1)
        y = -torch.fft.fft(ext.to(torch.complex128)).imag[..., 1:nc + 1] * np.sqrt(2.0 / (nc + 1)) / 2.0
        return y.movedim(-1, dim)

    T = lambda x: dst(dst(x, 0), 1)
    ft = f
    u = torch.zeros_like(ft)
    for _ in range(K):
        v = torch.zeros_like(u)
        for s in range(len(omega)):
            ut = u + alpha_t[s] * v
            v = alpha[s] * v + omega[s] * (ft - A(ut))
            u = u + v
        r = ft - A(u)
        u = u + P(T(symbol * T(R(r))))
    r = ft - A(u)
    return torch.sum(r * r) / torch.sum(ft * ft)


def test_twogrid_adjoint_matches_torch_autograd():
    coef, f, omega, alpha, alpha_t, symbol, _ = _case("nagex", False, seed=8)
    K, n = 3, 15
    L, dw, da, dat, dsym, df = twogrid.loss_and_grads("nagex", coef, f, omega, symbol, K, alpha=alpha,
                                                      alpha_t=alpha_t)
    tw = torch.tensor(omega, requires_grad=True)
    ta = torch.tensor(alpha, requires_grad=True)
    tat = torch.tensor(alpha_t, requires_grad=True)
    ts = torch.tensor(symbol, requires_grad=True)
    tf = torch.tensor(f, requires_grad=True)
    Lt = _torch_cycle_loss(coef, tf, tw, ta, tat, ts, K, n)
    Lt.backward()
    assert abs(Lt.item() - L) <= 1e-12 * L
    for got, want in ((dw, tw.grad), (da, ta.grad), (dat, tat.grad), (dsym, ts.grad), (df, tf.grad)):
        np.testing.assert_allclose(got, want.numpy(), rtol=1e-9, atol=1e-12 * np.max(np.abs(want.numpy())))
