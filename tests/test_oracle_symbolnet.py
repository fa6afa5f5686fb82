"""Pins of the two-grid symbol network oracle (oracle/symbolnet.py), CPU only:
  - its convolutions, activations and symbol against an independent torch FP64 version
    built on torch.nn.functional.conv2d (zero padding 1);
  - its parameter gradient against torch autograd of that version and against central
    differences;
  - its eigenvalue feature against the dense spectrum of the assembled Helmholtz matrix
    (the modes p, q <= nc of a 7 x 7 grid);
  - with the last layer zero the symbol is the regularised inverse eigenvalue, which for
    |lam| >> 1 multiplies lam to 1 within 1 / lam^2."""
import numpy as np
import pytest
import torch

from oracle import problem, symbolnet as sn
from synthetic import symbolnet_params


def _torch_forward(theta, kappa, n):
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a) for a in sn.unpack(theta)]
    X = torch.tensor(sn.features(kappa, n))[None]
    F = torch.nn.functional
    a1 = torch.tanh(F.conv2d(X, W1, b1, padding=1))
    a2 = torch.tanh(F.conv2d(a1, W2, b2, padding=1))
    z = F.conv2d(a2, W3, b3, padding=1)[0, 0]
    return torch.tensor(sn.base_symbol(kappa, n)) * torch.exp(z)


@pytest.mark.parametrize("n,kappa,seed", [(15, 20.0, 0), (31, 55.5, 1), (63, 80.0, 2)])
def test_forward_matches_torch_conv2d(n, kappa, seed):
    theta = symbolnet_params(seed=seed, last_std=0.3)  # a visible correction
    got = sn.forward(theta, kappa, n)
    want = _torch_forward(theta, kappa, n).numpy()
    assert got.shape == ((n - 1) // 2, (n - 1) // 2)
    assert np.max(np.abs(np.exp(np.log(np.abs(got)) - np.log(np.abs(want))) - 1.0)) < 1e-12
    assert np.array_equal(np.sign(got), np.sign(want))


@pytest.mark.parametrize("n,kappa,seed", [(15, 33.0, 3), (31, 70.0, 4)])
def test_backward_matches_torch_autograd(n, kappa, seed):
    theta = symbolnet_params(seed=seed, last_std=0.3)
    nc = (n - 1) // 2
    g = np.random.default_rng(seed).standard_normal((nc, nc))
    got = sn.backward(theta, kappa, n, g)
    shapes = sn.SHAPES
    params = [torch.tensor(a, requires_grad=True) for a in sn.unpack(theta)]
    W1, b1, W2, b2, W3, b3 = params
    X = torch.tensor(sn.features(kappa, n))[None]
    F = torch.nn.functional
    a1 = torch.tanh(F.conv2d(X, W1, b1, padding=1))
    a2 = torch.tanh(F.conv2d(a1, W2, b2, padding=1))
    sym = torch.tensor(sn.base_symbol(kappa, n)) * torch.exp(F.conv2d(a2, W3, b3, padding=1)[0, 0])
    (sym * torch.tensor(g)).sum().backward()
    want = np.concatenate([p.grad.numpy().ravel() for p in params])
    assert len(shapes) == 6 and got.shape == want.shape
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_backward_matches_central_differences():
    n, kappa = 15, 41.0
    theta = symbolnet_params(seed=9, last_std=0.3)
    g = np.random.default_rng(9).standard_normal(((n - 1) // 2,) * 2)
    grad = sn.backward(theta, kappa, n, g)
    J = lambda t: float(np.sum(g * sn.forward(t, kappa, n)))  # noqa: E731
    delta = 1e-6
    # one weight and the bias of every layer
    for k in (5, 431, 432 + 16 + 7, 432 + 16 + 2304 + 3, 2913 - 144 + 11, 2912):
        e = np.zeros_like(theta)
        e[k] = delta
        fd = (J(theta + e) - J(theta - e)) / (2 * delta)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, grad[k])


def test_eigenvalue_feature_against_dense_spectrum():
    n, kappa = 7, 23.0
    h = 1.0 / (n + 1)
    coef = problem.helmholtz_stencil(kappa, n)
    A = np.zeros((n * n, n * n))
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        A[:, k] = problem.apply_A(coef, e.reshape(n, n)).ravel()
    dense = np.linalg.eigvalsh(0.5 * (A + A.T))
    lam = sn.features(kappa, n)[0] * 8.0 / (h * h)
    for v in lam.ravel():
        assert np.min(np.abs(dense - v)) <= 1e-9 * max(1.0, abs(v))


def test_zero_last_layer_gives_the_regularised_inverse():
    n, kappa = 31, 60.0
    theta = symbolnet_params(seed=1)
    k3 = sn.param_count() - 145
    theta[k3:] = 0.0  # W3 and b3
    sym = sn.forward(theta, kappa, n)
    lam = sn.eigenvalues(kappa, n)
    big = np.abs(lam) > 100.0
    assert np.all(np.abs(sym[big] * lam[big] - 1.0) <= 1.0 / lam[big] ** 2 + 1e-15)
