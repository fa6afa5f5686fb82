"""Pins for the oracle's adjoint of the unrolled NAG-Richardson(m) and its meta network (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import adjoint, iterate, meta, problem
from synthetic import meta_params


def _setup(seed=0, n=7, m=4, eps=0.02, theta=0.9):
    rng = np.random.default_rng(seed)
    coef = problem.q1_stencil(eps, theta)
    f = rng.standard_normal((n, n))
    G = problem.gershgorin(coef)
    omega = rng.uniform(0.3, 1.0, m) / G
    alpha = rng.uniform(0.3, 0.9, m)
    return coef, f, omega, alpha, rng


def _loss(coef, f, omega, alpha, K):
    u, _ = iterate.run(iterate.NAG, coef, f, omega, K, alpha=alpha)
    r = f - problem.apply_A(coef, u)
    return float(np.sum(r * r) / np.sum(f * f))


def test_adjoint_matches_central_differences():
    coef, f, omega, alpha, rng = _setup()
    K, d = 12, 1e-6
    L, dw, da, df = adjoint.loss_and_grads(coef, f, omega, alpha, K)
    assert abs(L - _loss(coef, f, omega, alpha, K)) < 1e-15
    for i in range(len(omega)):
        e = np.zeros_like(omega)
        e[i] = d
        fd_w = (_loss(coef, f, omega + e, alpha, K) - _loss(coef, f, omega - e, alpha, K)) / (2 * d)
        fd_a = (_loss(coef, f, omega, alpha + e, K) - _loss(coef, f, omega, alpha - e, K)) / (2 * d)
        assert abs(fd_w - dw[i]) <= 1e-6 * max(abs(dw[i]), 1e-3 * np.max(np.abs(dw)))
        assert abs(fd_a - da[i]) <= 1e-6 * max(abs(da[i]), 1e-3 * np.max(np.abs(da)))
    for (j, i) in ((0, 0), (3, 4), (6, 2)):
        e = np.zeros_like(f)
        e[j, i] = d
        fd = (_loss(coef, f + e, omega, alpha, K) - _loss(coef, f - e, omega, alpha, K)) / (2 * d)
        assert abs(fd - df[j, i]) <= 1e-6 * np.max(np.abs(df))


def _torch_unroll(coef, f, omega, alpha, K, seed_g=None):
    """NAG-Richardson(m) written with torch.conv2d (3x3 kernel, zero padding) and autograd."""
    w = torch.tensor(omega, dtype=torch.float64, requires_grad=True)
    a = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
    ft = torch.tensor(f, dtype=torch.float64, requires_grad=True)
    c0, cx, cy, cpp, cpm = coef
    # kernel[dy + 1, dx + 1] multiplies u[j + dy, i + dx]
    ker = torch.tensor([[cpp, cy, cpm], [cx, c0, cx], [cpm, cy, cpp]], dtype=torch.float64)
    ker = ker.view(1, 1, 3, 3)

    def A(x):
        return torch.nn.functional.conv2d(x.view(1, 1, *x.shape), ker, padding=1).view(*x.shape)

    m = len(omega)
    u = torch.zeros_like(ft)
    v = torch.zeros_like(ft)
    for s in range(K):
        i = s % m
        ut = u + a[i] * v
        v = a[i] * v + w[i] * (ft - A(ut))
        u = u + v
    if seed_g is None:
        r = ft - A(u)
        L = (r * r).sum() / (ft * ft).sum()
    else:
        L = (torch.tensor(seed_g) * u).sum()
    L.backward()
    return L.item(), w.grad.numpy(), a.grad.numpy(), ft.grad.numpy()


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_matches_torch_autograd(seed):
    coef, f, omega, alpha, rng = _setup(seed=seed, n=9, m=4)
    K = 16
    L, dw, da, df = adjoint.loss_and_grads(coef, f, omega, alpha, K)
    Lt, dwt, dat, dft = _torch_unroll(coef, f, omega, alpha, K)
    assert abs(L - Lt) <= 1e-13 * abs(Lt)
    assert np.allclose(dw, dwt, rtol=1e-11, atol=1e-13)
    assert np.allclose(da, dat, rtol=1e-11, atol=1e-13)
    assert np.allclose(df, dft, rtol=1e-10, atol=1e-13)
    # a user-supplied seed for dL/du_K
    g = rng.standard_normal(f.shape)
    L2, dw2, da2, df2 = adjoint.loss_and_grads(coef, f, omega, alpha, K, g_uK=g)
    Lt2, dwt2, dat2, dft2 = _torch_unroll(coef, f, omega, alpha, K, seed_g=g)
    assert abs(L2 - Lt2) <= 1e-12 * abs(Lt2)
    assert np.allclose(dw2, dwt2, rtol=1e-11) and np.allclose(da2, dat2, rtol=1e-11)
    assert np.allclose(df2, dft2, rtol=1e-10, atol=1e-13)


def _torch_meta(params, m):
    H = meta.H
    net = torch.nn.Sequential(torch.nn.Linear(2, H), torch.nn.Tanh(), torch.nn.Linear(H, H),
                              torch.nn.Tanh(), torch.nn.Linear(H, m + 1)).double()
    k = 0
    for layer in (net[0], net[2], net[4]):
        for t in (layer.weight, layer.bias):
            t.data = torch.tensor(params[k:k + t.numel()], dtype=torch.float64).view_as(t)
            k += t.numel()
    assert k == len(params)
    return net


def test_meta_network_matches_torch():
    m = 16
    params = meta_params(m=m, seed=0)
    assert len(params) == meta.n_params(m) == 5457
    rng = np.random.default_rng(9)
    B = 12
    leps = rng.uniform(-4, 0, B)
    theta = rng.uniform(0, np.pi, B)
    gersh = rng.uniform(2.0, 4.0, B)
    om, al, cache = meta.forward(params, m, leps, theta, gersh)
    net = _torch_meta(params, m)
    x = torch.tensor(np.stack([leps, theta], 1))
    z = net(x)
    om_t = torch.exp(z[:, :m]) / torch.tensor(gersh)[:, None]
    beta_t = torch.sigmoid(z[:, m])
    assert np.allclose(om, om_t.detach().numpy(), rtol=1e-13)
    assert np.allclose(al, np.repeat(beta_t.detach().numpy()[:, None], m, 1), rtol=1e-13)
    # backward of a random linear functional of (omega, alpha)
    gw = rng.standard_normal((B, m))
    ga = rng.standard_normal((B, m))
    grads = meta.backward(params, m, cache, gw, ga)
    obj = (om_t * torch.tensor(gw)).sum() + (beta_t[:, None] * torch.tensor(ga)).sum()
    obj.backward()
    gt = np.concatenate([p.grad.numpy().ravel() for p in net.parameters()])
    assert np.allclose(grads, gt, rtol=1e-11, atol=1e-15)


def test_meta_head_at_initialisation_is_contractive():
    # head reading: omega_i = exp(z_i)/G keeps omega * lambda_max <= ~1 and beta ~ 0.99 at init
    params = meta_params(m=16, seed=0)
    eps = np.array([1e-4, 1e-2, 1.0])
    theta = np.array([0.3, 1.7, 3.0])
    G = np.array([problem.gershgorin(problem.q1_stencil(e, t)) for e, t in zip(eps, theta)])
    om, al, _ = meta.forward(params, 16, np.log10(eps), theta, G)
    assert np.all(om * G[:, None] < 1.2) and np.all(om * G[:, None] > 0.8)
    assert np.all(np.abs(al - 0.99) < 0.01)


def _torch_unroll_general(coef, f, omega, alpha, alpha_t, K, dinv):
    """The NAGex recurrence with a Jacobi scale, written with torch.conv2d and autograd."""
    w = torch.tensor(omega, dtype=torch.float64, requires_grad=True)
    a = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
    at = torch.tensor(alpha_t, dtype=torch.float64, requires_grad=True)
    ft = torch.tensor(f, dtype=torch.float64, requires_grad=True)
    c0, cx, cy, cpp, cpm = coef
    ker = torch.tensor([[cpp, cy, cpm], [cx, c0, cx], [cpm, cy, cpp]], dtype=torch.float64).view(1, 1, 3, 3)

    def A(x):
        return torch.nn.functional.conv2d(x.view(1, 1, *x.shape), ker, padding=1).view(*x.shape)

    m = len(omega)
    u = torch.zeros_like(ft)
    v = torch.zeros_like(ft)
    for s in range(K):
        i = s % m
        r = ft - A(u + at[i] * v)
        v = a[i] * v + w[i] * dinv * r
        u = u + v
    r = ft - A(u)
    L = (r * r).sum() / (ft * ft).sum()
    L.backward()
    return L.item(), w.grad.numpy(), a.grad.numpy(), at.grad.numpy(), ft.grad.numpy()


@pytest.mark.parametrize("method", [adjoint.RICHARDSON, adjoint.MOM, adjoint.NAG, adjoint.NAGEX])
@pytest.mark.parametrize("dinv", [1.0, 0.37])
def test_general_adjoint_matches_torch_autograd(method, dinv):
    coef, f, omega, alpha, rng = _setup(seed=4, n=8, m=3)
    alpha_t = rng.uniform(0.1, 0.9, 3)
    omega = omega / dinv if dinv != 1.0 else omega
    K = 12
    L, dw, da, dat, df = adjoint.loss_and_grads_general(method, coef, f, omega, K, alpha=alpha,
                                                          alpha_t=alpha_t, dinv=dinv)
    z = np.zeros(3)
    a_eff = {adjoint.RICHARDSON: z, adjoint.MOM: alpha, adjoint.NAG: alpha, adjoint.NAGEX: alpha}[method]
    at_eff = {adjoint.RICHARDSON: z, adjoint.MOM: z, adjoint.NAG: alpha, adjoint.NAGEX: alpha_t}[method]
    Lt, dwt, dat_, datt, dft = _torch_unroll_general(coef, f, omega, a_eff, at_eff, K, dinv)
    assert abs(L - Lt) <= 1e-13 * abs(Lt)
    assert np.allclose(dw, dwt, rtol=1e-10, atol=1e-14)
    assert np.allclose(df, dft, rtol=1e-10, atol=1e-14)
    if method == adjoint.NAG:
        # one factor drives both the momentum and the look-ahead
        assert np.allclose(da + dat, dat_ + datt, rtol=1e-10, atol=1e-14)
    elif method != adjoint.RICHARDSON:
        assert np.allclose(da, dat_, rtol=1e-10, atol=1e-14)
        if method == adjoint.NAGEX:
            assert np.allclose(dat, datt, rtol=1e-10, atol=1e-14)


def test_general_adjoint_central_differences_nagex():
    coef, f, omega, alpha, rng = _setup(seed=6, n=7, m=3)
    alpha_t = rng.uniform(0.1, 0.9, 3)
    dinv, K, d = 0.5, 9, 1e-6
    omega = omega / dinv

    def loss(w, a, at):
        us, _ = adjoint.unroll_states(coef, f, w, a, K, method=adjoint.NAGEX, alpha_t=at, dinv=dinv)
        r = f - problem.apply_A(coef, us[K])
        return float(np.sum(r * r) / np.sum(f * f))

    L, dw, da, dat, _ = adjoint.loss_and_grads_general(adjoint.NAGEX, coef, f, omega, K, alpha=alpha,
                                                        alpha_t=alpha_t, dinv=dinv)
    for i in range(3):
        e = np.zeros(3)
        e[i] = d
        for grad, fd in ((dw, (loss(omega + e, alpha, alpha_t) - loss(omega - e, alpha, alpha_t)) / (2 * d)),
                         (da, (loss(omega, alpha + e, alpha_t) - loss(omega, alpha - e, alpha_t)) / (2 * d)),
                         (dat, (loss(omega, alpha, alpha_t + e) - loss(omega, alpha, alpha_t - e)) / (2 * d))):
            assert abs(fd - grad[i]) <= 1e-6 * max(abs(grad[i]), 1e-3 * np.max(np.abs(grad)))


def test_oracle_jacobi_unroll_matches_iterate_preconditioner():
    # the adjoint's forward with dinv equals the Table-1 scheme with B^{-1} = dinv I
    coef, f, omega, alpha, rng = _setup(seed=8, n=6, m=4)
    alpha_t = rng.uniform(0.1, 0.9, 4)
    dinv = 1.0 / coef[0]
    us, vs = adjoint.unroll_states(coef, f, omega, alpha, 10, method=adjoint.NAGEX, alpha_t=alpha_t, dinv=dinv)
    u, v = iterate.run(iterate.NAGEX, coef, f, omega, 10, alpha=alpha, alpha_t=alpha_t, binv=lambda r: dinv * r)
    assert np.allclose(us[10], u, atol=1e-13) and np.allclose(vs[10], v, atol=1e-13)
