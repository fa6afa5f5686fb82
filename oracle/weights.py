"""Weight providers for Richardson(m), test infrastructure only.

chebyshev_weights  -- §2, eq. chebyshev-weights / chebyshev-weights-cos:
                      omega_i = 2 / (lmax + lmin + (lmax - lmin) x_i),
                      x_i = cos((2i - 1) pi / (2m)), i = 1..m.
semi_iteration     -- §2: the same formula with lmin replaced by alpha * lmax
                      (alpha = 1/30 in the paper's example).
leja_order         -- a reordering of one cycle's weights (not from the paper; a
                      standard device against rounding growth in long cycles).
amplification      -- how much the remaining factors of a cycle can magnify an
                      error injected after inner step j (diagnostic for FP32 runs).
"""
import numpy as np


def chebyshev_weights(lmin, lmax, m):
    """Optimal Richardson(m) weights for an SPD spectrum inside [lmin, lmax], omega_1 first."""
    i = np.arange(1, m + 1)
    x = np.cos((2.0 * i - 1.0) * np.pi / (2.0 * m))
    return 2.0 / (lmax + lmin + (lmax - lmin) * x)


def semi_iteration_weights(lmax, m, alpha=1.0 / 30.0):
    """Chebyshev semi-iteration: lmin := alpha * lmax."""
    return chebyshev_weights(alpha * lmax, lmax, m)


def leja_order(omega):
    """Leja ordering of the nodes 1/omega_i: start at the largest node, then repeatedly
    take the node that maximises the product of distances to the nodes already taken."""
    nodes = 1.0 / np.asarray(omega, dtype=np.float64)
    left = list(range(len(nodes)))
    first = max(left, key=lambda k: abs(nodes[k]))
    order = [first]
    left.remove(first)
    while left:
        nxt = max(left, key=lambda k: np.prod([abs(nodes[k] - nodes[j]) for j in order]))
        order.append(nxt)
        left.remove(nxt)
    return np.asarray(omega)[order]


def cycle_polynomial(omega, lam):
    """prod_i (1 - omega_i lam): the residual polynomial of one Richardson(m) cycle."""
    lam = np.asarray(lam, dtype=np.float64)
    p = np.ones_like(lam)
    for w in omega:
        p = p * (1.0 - w * lam)
    return p


def amplification(omega, lmin, lmax, samples=20001):
    """max over j and lam in [lmin, lmax] of |prod_{i > j} (1 - omega_i lam)|: the largest
    factor by which the rest of a cycle can magnify an error made after step j."""
    lam = np.linspace(lmin, lmax, samples)
    worst = 1.0
    m = len(omega)
    for j in range(m):
        tail = np.ones_like(lam)
        for w in omega[j + 1:]:
            tail = tail * (1.0 - w * lam)
        worst = max(worst, float(np.max(np.abs(tail))))
    return worst
