"""SSOR preconditioning of the Table-1 schemes, test infrastructure only.

§2.1 lists the stationary preconditioners as Richardson forms u += omega B^{-1}(f - A u);
for SSOR with relaxation factor a (at omega = 1)

    B^{-1} = a (2 - a) (D - a U)^{-1} D (D - a L)^{-1},

with A = D - L - U split into its diagonal and strictly lower / upper parts.  The split
depends on the ordering of the unknowns, which the paper does not state.  This oracle
uses the four-colour ordering: colour(i, j) = (i mod 2) + 2 (j mod 2) on 0-based interior
indices, colours in increasing order, grid order (row j, then i) within a colour.  Points
of one colour are never coupled by the 9-point or the 5-point stencil, so each triangular
solve runs colour by colour.

ssor_apply is that definition written out: A assembled as a sparse matrix from the
stencil, permuted to the colour order, split, and the two triangular systems solved with
scipy.  Because A is symmetric, U = L^T and B^{-1} is symmetric.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from .problem import OFFSETS


def colours(n):
    """Colour of every interior point, as c[j, i]."""
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return (i % 2) + 2 * (j % 2)


def colour_order(n):
    """Permutation of the grid-order indices j*n + i into the four-colour order."""
    c = colours(n).ravel()
    return np.concatenate([np.flatnonzero(c == k) for k in range(4)])


def assemble(coef, n):
    """Sparse A in grid order (row j*n + i), from the stencil (zero Dirichlet)."""
    rows, cols, vals = [], [], []
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for (dx, dy), slot in OFFSETS:
        if coef[slot] == 0.0:
            continue
        jj, ii = j + dy, i + dx
        ok = (ii >= 0) & (ii < n) & (jj >= 0) & (jj < n)
        rows.append((j * n + i)[ok])
        cols.append((jj * n + ii)[ok])
        vals.append(np.full(int(ok.sum()), coef[slot]))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n * n, n * n))


def split(coef, n):
    """(D, L, U, perm) of A in the colour order: A_perm = D - L - U."""
    perm = colour_order(n)
    A = assemble(coef, n)[perm][:, perm].tocsr()
    D = sp.diags(A.diagonal()).tocsr()
    L = -sp.tril(A, k=-1, format="csr")
    U = -sp.triu(A, k=1, format="csr")
    return D, L, U, perm


def ssor_apply(coef, r, relax):
    """B^{-1} r for the SSOR preconditioner with relaxation factor `relax`."""
    n = r.shape[0]
    D, L, U, perm = split(coef, n)
    rp = r.ravel()[perm]
    y = spl.spsolve_triangular((D - relax * L).tocsr(), rp, lower=True)
    w = spl.spsolve_triangular((D - relax * U).tocsr(), D @ y, lower=False)
    out = np.empty(n * n)
    out[perm] = relax * (2.0 - relax) * w
    return out.reshape(n, n)


def ssor_binv(coef, relax):
    """The callable r -> B^{-1} r that oracle.iterate and oracle.adjoint take."""
    return lambda r: ssor_apply(coef, r, relax)
