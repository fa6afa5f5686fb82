"""Meta(theta; mu) network and its output head, test infrastructure only.

§2.2: a network maps the PDE parameters mu to the iteration weights; §2.3 uses a
fully connected network whose input is (lg eps, theta).  The figure with its
architecture is not part of the text, so this follows the reading used by the
library: (log10 eps, theta) -> tanh(64) -> tanh(64) -> m + 1 outputs z.
Output head (a reading; the paper states none for this problem):
    omega_i = exp(z_i) / G   (i = 1..m; G = Gershgorin bound of the instance stencil)
    beta    = 1 / (1 + exp(-z_{m+1})),  alpha_i = beta for every i.
Flat parameter layout (row-major weights, out x in):
    W1[64][2], b1[64], W2[64][64], b2[64], W3[m+1][64], b3[m+1].
"""
import numpy as np

H = 64


def n_params(m):
    return H * 2 + H + H * H + H + (m + 1) * H + (m + 1)


def unpack(params, m):
    p = np.asarray(params, dtype=np.float64)
    shapes = [(H, 2), (H,), (H, H), (H,), (m + 1, H), (m + 1,)]
    out, k = [], 0
    for s in shapes:
        size = int(np.prod(s))
        out.append(p[k:k + size].reshape(s))
        k += size
    assert k == p.size, (k, p.size)
    return out


def forward(params, m, log10_eps, theta, gersh):
    """Returns (omega[B, m], alpha[B, m], cache) for a batch of instances."""
    W1, b1, W2, b2, W3, b3 = unpack(params, m)
    x = np.stack([np.asarray(log10_eps, np.float64), np.asarray(theta, np.float64)], axis=1)
    h1 = np.tanh(x @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    z = h2 @ W3.T + b3
    omega = np.exp(z[:, :m]) / np.asarray(gersh, np.float64)[:, None]
    beta = 1.0 / (1.0 + np.exp(-z[:, m]))
    alpha = np.repeat(beta[:, None], m, axis=1)
    return omega, alpha, (x, h1, h2, z, omega, beta)


def backward(params, m, cache, d_omega, d_alpha):
    """Gradient of sum_b <d_omega_b, omega_b> + <d_alpha_b, alpha_b> w.r.t. the flat params."""
    W1, b1, W2, b2, W3, b3 = unpack(params, m)
    x, h1, h2, z, omega, beta = cache
    dz = np.zeros_like(z)
    dz[:, :m] = np.asarray(d_omega) * omega                       # d exp(z)/G = exp(z)/G dz
    dz[:, m] = np.sum(np.asarray(d_alpha), axis=1) * beta * (1.0 - beta)
    gW3 = dz.T @ h2
    gb3 = dz.sum(axis=0)
    dh2 = dz @ W3
    da2 = dh2 * (1.0 - h2 * h2)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (1.0 - h1 * h1)
    gW1 = da1.T @ x
    gb1 = da1.sum(axis=0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])
