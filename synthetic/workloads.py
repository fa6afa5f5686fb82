"""Seeded workloads with the shapes and distributions of the paper's experiments.

The paper (§2.3) draws the anisotropy parameters at random, fixes the grid, and
takes the right-hand side vector f ~ N(0, I).  The batches below keep that recipe
with the sizes of the measured configurations:

  single   -- one isotropic problem (eps = 1, theta = 0), n = 63, f from seed 0
  aniso    -- B problems, eps = 10**U(-4, 0), theta = U(0, pi), f ~ N(0, I) per instance
  uneven   -- 512 problems with n drawn from {63, 127, 255, 511, 1023} in the
              proportions 40/25/20/10/5 percent, then eps, theta, f as in ``aniso``
  helmholtz-- B problems with kappa = U(20, 80) and a Gaussian point source

Every draw comes from ``numpy.random.default_rng(seed)`` in the order written
here.  Vectors are FP64, laid out per instance as ``u[j, i]`` (i fastest) and
packed back to back in instance order.
"""
import numpy as np

__all__ = [
    "Batch", "single_isotropic", "aniso_batch", "uneven_batch", "helmholtz_batch",
    "random_batch", "meta_params", "symbolnet_params", "pack", "unpack_vec", "offsets_of", "twogrid_symbol",
    "smoothing_weights",
]

META_HIDDEN = 64


class Batch:
    """A batch of independent problems: sizes, parameters and right-hand sides."""

    def __init__(self, n, eps=None, theta=None, kappa=None, f=None, op="q1"):
        self.n = [int(k) for k in n]
        self.B = len(self.n)
        self.op = op
        self.eps = None if eps is None else np.asarray(eps, dtype=np.float64)
        self.theta = None if theta is None else np.asarray(theta, dtype=np.float64)
        self.kappa = None if kappa is None else np.asarray(kappa, dtype=np.float64)
        self.f = f

    @property
    def offsets(self):
        return offsets_of(self.n)

    @property
    def points(self):
        return int(sum(k * k for k in self.n))

    def f_packed(self):
        return pack(self.f)


def offsets_of(ns):
    off = np.zeros(len(ns) + 1, dtype=np.int64)
    off[1:] = np.cumsum([int(k) * int(k) for k in ns])
    return off


def pack(vecs):
    """Concatenate per-instance [n, n] arrays into one flat vector."""
    return np.concatenate([np.asarray(v, dtype=np.float64).ravel() for v in vecs])


def unpack_vec(flat, ns):
    off = offsets_of(ns)
    return [np.asarray(flat[off[b]:off[b + 1]]).reshape(ns[b], ns[b]) for b in range(len(ns))]


def single_isotropic(n=63, seed=0):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n))
    return Batch([n], eps=[1.0], theta=[0.0], f=[f])


def _draw_params_and_rhs(rng, ns):
    B = len(ns)
    eps = 10.0 ** rng.uniform(-4.0, 0.0, size=B)
    theta = rng.uniform(0.0, np.pi, size=B)
    f = [rng.standard_normal((k, k)) for k in ns]
    return eps, theta, f


def aniso_batch(B, n, seed):
    rng = np.random.default_rng(seed)
    ns = [n] * B
    eps, theta, f = _draw_params_and_rhs(rng, ns)
    return Batch(ns, eps=eps, theta=theta, f=f)


def uneven_batch(seed=4, sizes=(63, 127, 255, 511, 1023), counts=(205, 128, 102, 51, 26)):
    rng = np.random.default_rng(seed)
    ns = []
    for s, c in zip(sizes, counts):
        ns += [s] * c
    ns = list(rng.permutation(np.array(ns)))
    eps, theta, f = _draw_params_and_rhs(rng, ns)
    return Batch(ns, eps=eps, theta=theta, f=f)


def random_batch(ns, seed, eps_range=(1e-4, 1.0)):
    """Small test batches with arbitrary (possibly ragged) sizes."""
    rng = np.random.default_rng(seed)
    B = len(ns)
    lo, hi = np.log10(eps_range[0]), np.log10(eps_range[1])
    eps = 10.0 ** rng.uniform(lo, hi, size=B)
    theta = rng.uniform(0.0, np.pi, size=B)
    f = [rng.standard_normal((k, k)) for k in ns]
    return Batch(ns, eps=eps, theta=theta, f=f)


def helmholtz_batch(B=32, n=511, seed=5, sigma_cells=2.0):
    rng = np.random.default_rng(seed)
    kappa = rng.uniform(20.0, 80.0, size=B)
    centres = rng.uniform(0.1, 0.9, size=(B, 2))
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    f = []
    for b in range(B):
        dx2 = (x[None, :] - centres[b, 0]) ** 2
        dy2 = (x[:, None] - centres[b, 1]) ** 2
        f.append(np.exp(-(dx2 + dy2) / (2.0 * (sigma_cells * h) ** 2)))
    return Batch([n] * B, kappa=kappa, f=f, op="helmholtz")


def twogrid_symbol(kappa, n, seed=None, spread=0.0, reg=1.0):
    """Coarse symbol [nc][nc] ([q-1][p-1] for mode sin(p pi x) sin(q pi y)) standing in
    for a learned one: the reciprocal of lam = (4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2))
    - kappa^2 (h = 1/(n+1), p, q = 1..nc) taken as lam / (lam^2 + reg^2), times an
    optional seeded factor U(1 - spread, 1 + spread).  Returned as float64."""
    nc = (n - 1) // 2
    h = 1.0 / (n + 1)
    k = np.arange(1, nc + 1)
    s = (4.0 / (h * h)) * np.sin(k * np.pi * h / 2.0) ** 2
    lam = s[:, None] + s[None, :] - float(kappa) ** 2
    sym = lam / (lam * lam + reg * reg)
    if spread > 0.0:
        sym = sym * np.random.default_rng(seed).uniform(1.0 - spread, 1.0 + spread, size=sym.shape)
    return sym


def smoothing_weights(lmax, m, lo_frac=0.25):
    """Stand-in smoother weights: reciprocals of the m Chebyshev points of
    [lo_frac * lmax, lmax], ordered largest, smallest, second largest, ... ."""
    a, b = lo_frac * lmax, lmax
    x = np.cos((2.0 * np.arange(1, m + 1) - 1.0) * np.pi / (2.0 * m))
    w = np.sort(2.0 / (a + b + (b - a) * x))
    order = [w[-1 - k // 2] if k % 2 == 0 else w[k // 2] for k in range(m)]
    return np.array(order)


def meta_params(m=16, seed=0, beta0=0.99, last_std=0.01):
    """Initial meta-network parameters, flat, in the layout
    W1[64][2], b1[64], W2[64][64], b2[64], W3[m+1][64], b3[m+1].

    Hidden layers: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases.
    Last layer: N(0, last_std^2) weights; biases 0 except the momentum output,
    whose bias is log(beta0 / (1 - beta0)).
    """
    rng = np.random.default_rng(seed)
    H = META_HIDDEN
    k1 = 1.0 / np.sqrt(2.0)
    k2 = 1.0 / np.sqrt(H)
    W1 = rng.uniform(-k1, k1, size=(H, 2))
    b1 = rng.uniform(-k1, k1, size=H)
    W2 = rng.uniform(-k2, k2, size=(H, H))
    b2 = rng.uniform(-k2, k2, size=H)
    W3 = rng.normal(0.0, last_std, size=(m + 1, H))
    b3 = np.zeros(m + 1)
    b3[m] = np.log(beta0 / (1.0 - beta0))
    return np.concatenate([a.ravel() for a in (W1, b1, W2, b2, W3, b3)])


def symbolnet_params(seed=0, hidden=16, last_std=0.01):
    """Initial parameters of the two-grid symbol network, flat, in the layout
    W1[hidden][3][3][3], b1[hidden], W2[hidden][hidden][3][3], b2[hidden], W3[1][hidden][3][3], b3[1].

    First two layers: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases (fan_in =
    9 x input channels); last layer: N(0, last_std^2) weights and a zero bias, so the
    network's output starts near zero.
    """
    rng = np.random.default_rng(seed)
    k1 = 1.0 / np.sqrt(9.0 * 3)
    k2 = 1.0 / np.sqrt(9.0 * hidden)
    W1 = rng.uniform(-k1, k1, size=(hidden, 3, 3, 3))
    b1 = rng.uniform(-k1, k1, size=hidden)
    W2 = rng.uniform(-k2, k2, size=(hidden, hidden, 3, 3))
    b2 = rng.uniform(-k2, k2, size=hidden)
    W3 = rng.normal(0.0, last_std, size=(1, hidden, 3, 3))
    b3 = np.zeros(1)
    return np.concatenate([a.ravel() for a in (W1, b1, W2, b2, W3, b3)])
