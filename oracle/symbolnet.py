"""Symbol network of the two-grid Helmholtz cycle, test infrastructure only.

The multilevel solver of §3 takes its coarse correction H = F T Lambda~ T* F^{-1}
(eq. dl-him-h) with Lambda~ produced by a meta network (Meta-Lambda~) that stands in for
the inverse eigenvalues of A; §3.2 learns the smoother's weights in log form.  The
network's architecture is not given in the text.  The reading built here (the two-grid
form of the cycle, T = I, a real symbol):

  features, per coarse mode (p, q), p, q = 1..nc (nc = (n - 1)/2), stored [q-1][p-1]:
    x0 = lam_pq h^2 / 8, the fine-grid eigenvalue of the 5-point Helmholtz operator
         lam_pq = (4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2)) - kappa^2, h = 1/(n+1);
    x1 = p / (nc + 1);  x2 = q / (nc + 1);
  three 3 x 3 convolutions over the mode grid (zero padding, cross-correlation as in
  torch.nn.functional.conv2d), 3 -> 16 -> 16 -> 1 channels, tanh after the first two;
  symbol = lam / (lam^2 + 1) * exp(z), z the last layer's output: a log-form correction
  of the regularised inverse eigenvalue.

Parameters, one flat vector (torch layout [out][in][ky][kx]):
  W1[16][3][3][3], b1[16], W2[16][16][3][3], b2[16], W3[1][16][3][3], b3[1]  (2913).
Everything in FP64 with plain loops over the kernel offsets.
"""
import numpy as np

from .spectra import helmholtz_eigenvalues

C_IN, C_HID, C_OUT = 3, 16, 1
SHAPES = [(C_HID, C_IN, 3, 3), (C_HID,), (C_HID, C_HID, 3, 3), (C_HID,), (C_OUT, C_HID, 3, 3), (C_OUT,)]


def param_count():
    return int(sum(np.prod(s) for s in SHAPES))


def unpack(theta):
    """Split the flat parameter vector into (W1, b1, W2, b2, W3, b3)."""
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for s in SHAPES:
        size = int(np.prod(s))
        out.append(theta[k:k + size].reshape(s))
        k += size
    if k != theta.size:
        raise ValueError(f"expected {k} parameters, got {theta.size}")
    return out


def eigenvalues(kappa, n):
    """lam[q-1, p-1] for p, q = 1..nc, from the fine-grid closed form."""
    nc = (n - 1) // 2
    return helmholtz_eigenvalues(kappa, n)[:nc, :nc]


def features(kappa, n):
    """X[3, nc, nc]: (lam h^2 / 8, p / (nc + 1), q / (nc + 1)) per mode, [c][q-1][p-1]."""
    nc = (n - 1) // 2
    h = 1.0 / (n + 1)
    lam = eigenvalues(kappa, n)
    k = np.arange(1, nc + 1) / (nc + 1.0)
    X = np.empty((3, nc, nc))
    X[0] = lam * h * h / 8.0
    X[1] = k[None, :]
    X[2] = k[:, None]
    return X


def base_symbol(kappa, n):
    lam = eigenvalues(kappa, n)
    return lam / (lam * lam + 1.0)


def conv3x3(x, W, b):
    """y[co] = b[co] + sum_ci sum_{dy,dx} W[co, ci, dy+1, dx+1] x[ci, y + dy, x + dx], zero outside."""
    cin, H, Wd = x.shape
    xp = np.zeros((cin, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.empty((W.shape[0], H, Wd))
    for co in range(W.shape[0]):
        acc = np.full((H, Wd), b[co])
        for ci in range(cin):
            for ky in range(3):
                for kx in range(3):
                    acc += W[co, ci, ky, kx] * xp[ci, ky:ky + H, kx:kx + Wd]
        y[co] = acc
    return y


def conv3x3_input_grad(g, W, in_shape):
    """d/dx of sum(g * conv3x3(x, W, 0)): each output's gradient flows back to the inputs
    it read, x[ci, y + dy, x + dx] += W[co, ci, dy+1, dx+1] g[co, y, x]."""
    cin, H, Wd = in_shape
    gx = np.zeros((cin, H + 2, Wd + 2))
    for co in range(W.shape[0]):
        for ci in range(cin):
            for ky in range(3):
                for kx in range(3):
                    gx[ci, ky:ky + H, kx:kx + Wd] += W[co, ci, ky, kx] * g[co]
    return gx[:, 1:-1, 1:-1]


def conv3x3_weight_grad(g, x):
    """dW[co, ci, ky, kx] = sum_{y,x} g[co, y, x] x[ci, y + ky - 1, x + kx - 1] (zero outside); db = sum g."""
    cin, H, Wd = x.shape
    xp = np.zeros((cin, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dW = np.empty((g.shape[0], cin, 3, 3))
    for co in range(g.shape[0]):
        for ci in range(cin):
            for ky in range(3):
                for kx in range(3):
                    dW[co, ci, ky, kx] = np.sum(g[co] * xp[ci, ky:ky + H, kx:kx + Wd])
    return dW, g.sum(axis=(1, 2))


def forward(theta, kappa, n, keep=False):
    """symbol[nc, nc] of one instance (and the activations when keep)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = features(kappa, n)
    a1 = np.tanh(conv3x3(X, W1, b1))
    a2 = np.tanh(conv3x3(a1, W2, b2))
    z = conv3x3(a2, W3, b3)[0]
    sym = base_symbol(kappa, n) * np.exp(z)
    if keep:
        return sym, (X, a1, a2, z)
    return sym


def backward(theta, kappa, n, d_symbol):
    """Gradient of sum(d_symbol * symbol) with respect to the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    sym, (X, a1, a2, z) = forward(theta, kappa, n, keep=True)
    gz = (np.asarray(d_symbol, dtype=np.float64) * sym)[None]       # d symbol / d z = symbol
    dW3, db3 = conv3x3_weight_grad(gz, a2)
    g2 = conv3x3_input_grad(gz, W3, a2.shape) * (1.0 - a2 * a2)    # through tanh
    dW2, db2 = conv3x3_weight_grad(g2, a1)
    g1 = conv3x3_input_grad(g2, W2, a1.shape) * (1.0 - a1 * a1)
    dW1, db1 = conv3x3_weight_grad(g1, X)
    return np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3)])
