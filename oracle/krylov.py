"""Restarted flexible GMRES with a neural solver as the preconditioner, test
infrastructure only.

§3.2 (Table gmres-Wave-ADR-smoothers) runs FGMRES with restart 20, preconditioned by a
multilevel neural solver whose action may change from one iteration to the next (it is
itself an iteration).  This is Saad's flexible GMRES: Arnoldi on the preconditioned
directions z_j = M_j(v_j), kept alongside the orthonormal v_j,

    w = A z_j;  h_ij = <w, v_i> (i <= j);  w -= sum h_ij v_i;  h_{j+1,j} = ||w||;
    v_{j+1} = w / h_{j+1,j};  y = argmin || beta e_1 - H_j y ||;  x = x_0 + Z_j y,

restarted from the true residual every `restart` steps.  Orthogonalisation here is
modified Gram-Schmidt; the least-squares problem is solved with numpy.linalg.lstsq
after every step (its residual is the relative-residual estimate).

A preconditioner is a callable z = M(j, v) (j = the overall iteration count); None means
z = v, which makes this plain restarted GMRES.
"""
import numpy as np


def fgmres(matvec, b, precond=None, x0=None, restart=20, max_iter=200, tol=1e-6):
    """Returns (x, hist, iters): hist[k] = ||b - A x_k|| / ||b|| estimated after each
    iteration k (x_k the minimiser over the current cycle), iters = iterations taken."""
    x = np.zeros_like(b, dtype=np.float64) if x0 is None else np.array(x0, dtype=np.float64)
    bn = np.linalg.norm(b)
    M = (lambda j, v: v) if precond is None else precond
    hist = []
    it = 0
    while it < max_iter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bn <= tol:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        y = np.zeros(0)
        for j in range(restart):
            z = M(it, V[j])
            Z.append(z)
            w = matvec(z)
            for i in range(j + 1):
                H[i, j] = np.sum(w * V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
            it += 1
            hist.append(res / bn)
            if res / bn <= tol or it >= max_iter or H[j + 1, j] == 0:
                break
        x = x + sum(yk * zk for yk, zk in zip(y, Z))
        if hist and hist[-1] <= tol:
            break
    return x, np.array(hist), it
