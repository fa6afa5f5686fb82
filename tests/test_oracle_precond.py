"""Pins of the SSOR preconditioner oracle (CPU): assembly against the stencil, the colour
ordering's decoupling, one preconditioned Richardson step against the classical pointwise
SSOR sweeps, B B^{-1} = I by multiplication, symmetry, positivity and the (0, 1] spectrum
of B^{-1} A, and the preconditioned adjoint against finite differences and torch autograd."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import adjoint, iterate, precond, problem


def _q1(eps, theta):
    return problem.q1_stencil(eps, theta)


CASES = [(_q1(1.0, 0.0), 7), (_q1(1e-3, 0.7), 9), (_q1(0.05, 2.2), 8), (problem.helmholtz_stencil(3.0, 7), 7)]


@pytest.mark.parametrize("coef,n", CASES)
def test_assembly_matches_stencil_and_colours_decouple(coef, n):
    A = precond.assemble(coef, n)
    x = np.random.default_rng(0).standard_normal((n, n))
    np.testing.assert_allclose((A @ x.ravel()).reshape(n, n), problem.apply_A(coef, x), rtol=1e-13, atol=1e-13)
    c = precond.colours(n).ravel()
    Ac = A.tocoo()
    off = Ac.row != Ac.col
    assert np.all(c[Ac.row[off]] != c[Ac.col[off]])
    perm = precond.colour_order(n)
    assert sorted(perm.tolist()) == list(range(n * n))
    assert np.all(np.diff(c[perm]) >= 0)


def _pointwise_ssor(coef, n, f, u, a):
    """One classical SSOR iteration written point by point: an SOR sweep over the colours
    in increasing order, then one in decreasing order, each point relaxed with the
    newest neighbour values."""
    u = u.copy()
    col = precond.colours(n)
    d = coef[0]
    nbrs = [((dx, dy), slot) for (dx, dy), slot in problem.OFFSETS if (dx, dy) != (0, 0)]

    def relax_point(j, i):
        s = f[j, i]
        for (dx, dy), slot in nbrs:
            jj, ii = j + dy, i + dx
            if 0 <= jj < n and 0 <= ii < n:
                s -= coef[slot] * u[jj, ii]
        u[j, i] = (1.0 - a) * u[j, i] + a * s / d

    for order in ((0, 1, 2, 3), (3, 2, 1, 0)):
        for k in order:
            for j in range(n):
                for i in range(n):
                    if col[j, i] == k:
                        relax_point(j, i)
    return u


@pytest.mark.parametrize("coef,n", CASES)
@pytest.mark.parametrize("a", [0.7, 1.0, 1.6])
def test_ssor_step_equals_pointwise_sweeps(coef, n, a):
    rng = np.random.default_rng(1)
    f = rng.standard_normal((n, n))
    u = rng.standard_normal((n, n))
    want = _pointwise_ssor(coef, n, f, u, a)
    got = u + precond.ssor_apply(coef, f - problem.apply_A(coef, u), a)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("coef,n", CASES[:3])
@pytest.mark.parametrize("a", [0.5, 1.0, 1.8])
def test_ssor_inverse_symmetric_positive_spectrum(coef, n, a):
    rng = np.random.default_rng(2)
    D, L, U, perm = precond.split(coef, n)
    Dinv = sp.diags(1.0 / D.diagonal())
    B = ((D - a * L) @ Dinv @ (D - a * U)) / (a * (2.0 - a))
    r = rng.standard_normal((n, n))
    z = precond.ssor_apply(coef, r, a)
    np.testing.assert_allclose(B @ z.ravel()[perm], r.ravel()[perm], rtol=1e-11, atol=1e-11)
    x, y = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    assert abs(np.sum(x * precond.ssor_apply(coef, y, a)) - np.sum(precond.ssor_apply(coef, x, a) * y)) < 1e-11
    assert np.sum(x * precond.ssor_apply(coef, x, a)) > 0
    # SSOR: B - A is positive semidefinite, so the spectrum of B^{-1} A lies in (0, 1]
    Ad = precond.assemble(coef, n).toarray()
    M = np.stack([precond.ssor_apply(coef, Ad[:, k].reshape(n, n), a).ravel() for k in range(n * n)], axis=1)
    lam = np.linalg.eigvals(M)
    assert np.max(np.abs(lam.imag)) < 1e-9
    assert lam.real.min() > 0 and lam.real.max() <= 1.0 + 1e-10


def test_preconditioned_nagex_converges_faster():
    """SSOR-preconditioned NAGex(3) reaches 1e-6 within 40 outer iterations on an
    anisotropic problem where plain NAGex(3) with Gershgorin-scaled weights is still
    above 1e-4 (the ordering of Table 2's last two rows)."""
    n = 31
    coef = _q1(1e-2, 0.3)
    f = np.random.default_rng(3).standard_normal((n, n))
    binv = precond.ssor_binv(coef, 1.0)
    _, _, h_ssor = iterate.run("nagex", coef, f, np.full(3, 1.2), 3 * 40, alpha=np.full(3, 0.8),
                               alpha_t=np.full(3, 0.8), binv=binv, history=True)
    G = problem.gershgorin(coef)
    _, _, h_plain = iterate.run("nagex", coef, f, np.full(3, 1.0 / G), 3 * 40, alpha=np.full(3, 0.9),
                                alpha_t=np.full(3, 0.9), history=True)
    assert h_ssor[-1] < 1e-6 and h_plain[-1] > 1e-4, (h_ssor[-1], h_plain[-1])


def _case(method, seed=4):
    n = 7
    coef = _q1(0.02, 1.1)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n))
    m = 3
    omega = rng.uniform(0.5, 1.2, m)
    alpha = rng.uniform(0.1, 0.5, m)
    alpha_t = rng.uniform(0.1, 0.5, m)
    return coef, n, f, omega, alpha, alpha_t


@pytest.mark.parametrize("method", ["nagex", "nag", "mom", "richardson"])
def test_ssor_adjoint_finite_differences(method):
    coef, n, f, omega, alpha, alpha_t = _case(method)
    a, K = 1.3, 6
    binv = precond.ssor_binv(coef, a)
    L, dw, da, dat, df = adjoint.loss_and_grads_general(method, coef, f, omega, K, alpha=alpha, alpha_t=alpha_t,
                                                        binv=binv)

    def loss(omega=omega, alpha=alpha, alpha_t=alpha_t, f=f):
        kw = {} if method == "richardson" else dict(alpha=alpha, alpha_t=alpha_t)
        u, _ = iterate.run(method, coef, f, omega, K, binv=binv, **kw)
        r = f - problem.apply_A(coef, u)
        return np.sum(r * r) / np.sum(f * f)

    assert abs(loss() - L) <= 1e-12 * L
    d = 1e-6

    def cd(fun, x0, idx):
        xp, xm = x0.copy(), x0.copy()
        xp[idx] += d
        xm[idx] -= d
        return (fun(xp) - fun(xm)) / (2 * d)

    for i in range(3):
        assert abs(cd(lambda w: loss(omega=w), omega, i) - dw[i]) <= 1e-5 * np.max(np.abs(dw))
        if method == "nag":
            assert abs(cd(lambda x: loss(alpha=x, alpha_t=x), alpha, i) - (da[i] + dat[i])) <= 1e-5 * np.max(np.abs(da))
        elif method in ("mom", "nagex"):
            assert abs(cd(lambda x: loss(alpha=x), alpha, i) - da[i]) <= 1e-5 * np.max(np.abs(da))
        if method == "nagex":
            assert abs(cd(lambda x: loss(alpha_t=x), alpha_t, i) - dat[i]) <= 1e-5 * np.max(np.abs(dat))
    for idx in [(0, 0), (3, 4), (6, 6)]:
        assert abs(cd(lambda g: loss(f=g), f, idx) - df[idx]) <= 1e-5 * np.max(np.abs(df))


def test_ssor_adjoint_matches_torch_autograd():
    """Independent torch version: dense A from the stencil by conv2d of unit vectors,
    SSOR through torch.linalg.solve_triangular in the colour order."""
    coef, n, f, omega, alpha, alpha_t = _case("nagex", seed=5)
    a, K = 0.9, 6
    L, dw, da, dat, df = adjoint.loss_and_grads_general("nagex", coef, f, omega, K, alpha=alpha, alpha_t=alpha_t,
                                                        binv=precond.ssor_binv(coef, a))
    N = n * n
    k = torch.zeros(1, 1, 3, 3, dtype=torch.float64)
    for (dx, dy), slot in problem.OFFSETS:
        k[0, 0, 1 + dy, 1 + dx] = coef[slot]
    eye = torch.eye(N, dtype=torch.float64).reshape(N, 1, n, n)
    A = torch.nn.functional.conv2d(eye, k, padding=1).reshape(N, N).T  # column k = A e_k
    col = torch.tensor([(i % 2) + 2 * (j % 2) for j in range(n) for i in range(n)])
    perm = torch.cat([torch.nonzero(col == c).flatten() for c in range(4)])
    Ap = A[perm][:, perm]
    Dm = torch.diag(torch.diagonal(Ap))
    Lm, Um = -torch.tril(Ap, -1), -torch.triu(Ap, 1)
    inv_perm = torch.argsort(perm)

    def binv(r):
        rp = r[perm].unsqueeze(1)
        y = torch.linalg.solve_triangular(Dm - a * Lm, rp, upper=False)
        w = torch.linalg.solve_triangular(Dm - a * Um, Dm @ y, upper=True)
        return (a * (2 - a) * w).squeeze(1)[inv_perm]

    tw = torch.tensor(omega, requires_grad=True)
    ta = torch.tensor(alpha, requires_grad=True)
    tat = torch.tensor(alpha_t, requires_grad=True)
    tf = torch.tensor(f.ravel(), requires_grad=True)
    u = torch.zeros(N, dtype=torch.float64)
    v = torch.zeros(N, dtype=torch.float64)
    for s in range(K):
        i = s % 3
        ut = u + tat[i] * v
        v = ta[i] * v + tw[i] * binv(tf - A @ ut)
        u = u + v
    r = tf - A @ u
    Lt = torch.sum(r * r) / torch.sum(tf * tf)
    Lt.backward()
    assert abs(Lt.item() - L) <= 1e-12 * L
    for got, want in ((dw, tw.grad), (da, ta.grad), (dat, tat.grad), (df.ravel(), tf.grad)):
        np.testing.assert_allclose(got, want.numpy(), rtol=1e-9, atol=1e-12 * np.max(np.abs(want.numpy())))
