"""GPU parity of the FP64-refined solve on the uneven workload's sizes, its per-round and
per-outer-iteration history, and caller-chosen instance offsets.

The refined path's bar: the reported relative residual is <= tol; the oracle's FP64
residual of the returned x agrees with it to 1e-12 (absolute, relative to ||b||);
and, where the mathematics gives the exact solution, ||x - x*|| / ||x*|| <= kappa tol.
For theta in {0, pi/2} the Q1 operator is diagonalised by the orthonormal DST-I, so
x* = S diag(1 / lambda) S b with the closed-form eigenvalues lambda_pq.
"""
import numpy as np
import pytest
import scipy.fft
import torch

from oracle import iterate, problem, spectra
from synthetic import Batch, random_batch, unpack_vec
from tests.gpu_helpers import dev, host, need_gpu, oracle_coef, plan_for, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2412_08076_amd import rm
    return rm.Context(0)


def _rm():
    from paper_2412_08076_amd import rm
    return rm


def exact_solution(eps, theta, b):
    """x* = S diag(1/lambda) S b for a Q1 operator with a vanishing mixed term."""
    lam = spectra.q1_eigenvalues(eps, theta, b.shape[0])
    bh = scipy.fft.dstn(b, type=1, norm="ortho")
    return scipy.fft.idstn(bh / lam, type=1, norm="ortho")


def _weights(batch, m, seed):
    """NAG weights like the meta network's initial head: omega ~ 1/G, momentum ~ 0.99."""
    rng = np.random.default_rng(seed)
    G = np.array([problem.gershgorin(oracle_coef(batch, b)) for b in range(batch.B)])
    om = (rng.uniform(0.9, 1.0, (batch.B, m)) / G[:, None]).astype(np.float32)
    al = rng.uniform(0.985, 0.99, (batch.B, m)).astype(np.float32)
    return om, al


def test_refined_solve_all_uneven_sizes(ctx):
    """Every size of the uneven workload, with theta = 0 and pi/2 instances at n = 511
    and n = 1023, refined to 1e-10."""
    rm = _rm()
    ns = [63, 127, 255, 511, 511, 1023, 1023, 63, 255]
    eps = [1.0, 0.3, 0.5, 1.0, 0.2, 1.0, 0.5, 1e-2, 0.05]
    theta = [0.0, np.pi / 2, 0.0, 0.0, np.pi / 2, np.pi / 2, 0.0, 0.7, 2.2]
    rng = np.random.default_rng(123)
    f = [rng.standard_normal((n, n)) for n in ns]
    batch = Batch(ns, eps=eps, theta=theta, f=f)
    say("refined all uneven sizes", ns)
    plan = plan_for(ctx, batch)
    say("kernels", {n: plan.get_kernel(n) for n in sorted(set(ns))})
    m = 16
    om, al = _weights(batch, m, seed=5)
    tol = 1e-10
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=tol, tol_inner=1e-3, max_outer=40000, max_rounds=10)
    rep = rm.rm_solve(ctx, plan, rm.RM_NAG, opts, dev(om, torch.float32), dev(al, torch.float32),
                      dev(batch.f_packed()), x)
    say("outer", rep["outer_iters"], "rounds", rep["rounds"], "relres", rep["relres"])
    assert rep["status"] == rm.RM_OK
    xs = unpack_vec(host(x), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        assert rep["relres"][b] <= tol, b
        assert abs(problem.relres(c, batch.f[b], xs[b]) - rep["relres"][b]) <= 1e-12, b
        if theta[b] in (0.0, np.pi / 2):
            th = 0.0 if theta[b] == 0.0 else np.pi / 2
            lam = spectra.q1_eigenvalues(eps[b], th, ns[b])
            kappa = lam.max() / lam.min()
            xstar = exact_solution(eps[b], th, batch.f[b])
            err = np.linalg.norm(xs[b] - xstar) / np.linalg.norm(xstar)
            say("instance", b, "n", ns[b], "kappa", kappa, "error", err)
            assert err <= kappa * tol, (b, err, kappa * tol)


def test_refined_history(ctx):
    """rep['history'][j] is rho_j of round j: the oracle's FP64 residual of the iterate a
    solve capped at j rounds returns.  hist holds ||r_j - A d||^2 per outer iteration;
    its first-round rows equal the FP32 unroll's history of A d = fl32(b) from d = 0."""
    rm = _rm()
    ns = [33, 63, 100]
    say("refined history", ns)
    batch = random_batch(ns, seed=131, eps_range=(0.05, 1.0))
    plan = plan_for(ctx, batch)
    m = 8
    om, al = _weights(batch, m, seed=9)
    al[:] = 0.9
    omd, ald, bd = dev(om, torch.float32), dev(al, torch.float32), dev(batch.f_packed())
    H = 4000
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-11, tol_inner=1e-3, max_outer=20000, max_rounds=8,
                         hist_len=H)
    hist = torch.empty(H * plan.B, dtype=torch.float64, device="cuda")
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    rep = rm.rm_solve(ctx, plan, rm.RM_NAG, opts, omd, ald, bd, x, hist=hist)
    say("rounds", rep["rounds"], "outer", rep["outer_iters"])
    assert rep["status"] == rm.RM_OK
    hs = host(hist).reshape(H, plan.B)
    rh = rep["history"]
    assert np.all(rh[0] == 1.0)  # x_0 = 0
    for b in range(plan.B):
        R = rep["rounds"][b]
        assert np.all(rh[R + 1:, b] == -1.0)
        assert abs(rh[R, b] - rep["relres"][b]) == 0.0
        k = rep["outer_iters"][b]
        assert k < H and np.all(hs[:k, b] >= 0.0) and np.all(hs[k:, b] == -1.0)
    # rho_j against the oracle: rerun capped at j rounds (same kernels, same iterates)
    for j in range(1, int(rep["rounds"].max())):
        xj = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
        oj = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-11, tol_inner=1e-3, max_outer=20000, max_rounds=j)
        rm.rm_solve(ctx, plan, rm.RM_NAG, oj, omd, ald, bd, xj)
        xs = unpack_vec(host(xj), ns)
        for b in range(plan.B):
            if rep["rounds"][b] < j:
                continue
            rho = problem.relres(oracle_coef(batch, b), batch.f[b], xs[b])
            assert abs(rho - rh[j, b]) <= 1e-12, (j, b, rho, rh[j, b])
    # first round: the inner solve is A d = fl32(b) from d = v = 0, for as many outer
    # iterations as it took to bring ||r_0 - A d|| below tol_inner ||r_0|| (that row
    # included): the FP32 unroll of the same scheme from zero on fl32(b)
    b32 = dev(batch.f_packed(), torch.float32)
    K = m * 16
    d = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    u_hist = torch.empty(K // m * plan.B, dtype=torch.float64, device="cuda")
    ou = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K)
    rm.rm_solve(ctx, plan, rm.RM_NAG, ou, omd, ald, b32, d, hist=u_hist)
    uh = host(u_hist).reshape(K // m, plan.B)
    for b in range(plan.B):
        bn2 = float(np.sum(batch.f[b] ** 2))
        above = hs[:, b] > 1e-6 * bn2
        n0 = min(K // m, int(np.argmin(above)) + 1)
        assert n0 >= 2, (b, n0)
        assert np.allclose(hs[:n0, b], uh[:n0, b], rtol=1e-9, atol=0.0), b
        f32 = batch.f[b].astype(np.float32).astype(np.float64)
        _, _, h = iterate.run(iterate.NAG, oracle_coef(batch, b), f32, om[b].astype(np.float64), n0 * m,
                              alpha=al[b].astype(np.float64), history=True)
        fn2 = float(np.sum(f32 ** 2))
        assert np.allclose(np.sqrt(hs[:n0, b] / fn2), h, rtol=1e-3, atol=1e-5), b


def test_plan_offsets_with_gaps(ctx):
    """Instances placed at caller offsets with gaps give, on their own points, the same
    bits as the packed plan (unrolled FP32 sweep and refined solve)."""
    rm = _rm()
    ns = [15, 64, 130]
    say("plan offsets with gaps", ns)
    batch = random_batch(ns, seed=141)
    packed = plan_for(ctx, batch)
    off = [5]
    for n in ns:
        off.append(off[-1] + n * n + 37)
    gapped = rm.Plan(ctx, ns, eps=batch.eps, theta=batch.theta, offsets=off)
    assert gapped.P == off[-1] and list(gapped.offsets) == off
    m, K = 8, 32
    om, al = _weights(batch, m, seed=3)
    omd, ald = dev(om, torch.float32), dev(al, torch.float32)

    def place(vecs, dtype):
        buf = np.full(off[-1], np.nan)
        for b, v in enumerate(vecs):
            buf[off[b]:off[b] + v.size] = v.ravel()
        return dev(buf, dtype)

    def take(t):
        h = host(t)
        return [h[off[b]:off[b] + n * n] for b, n in enumerate(ns)]

    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K)
    x0 = torch.zeros(packed.P, dtype=torch.float32, device="cuda")
    rm.rm_solve(ctx, packed, rm.RM_NAG, opts, omd, ald, dev(batch.f_packed(), torch.float32), x0)
    x1 = place([np.zeros((n, n)) for n in ns], torch.float32)
    rm.rm_solve(ctx, gapped, rm.RM_NAG, opts, omd, ald, place(batch.f, torch.float32), x1)
    for a, b in zip(unpack_vec(host(x0), ns), take(x1)):
        assert np.array_equal(a.ravel(), b)
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, tol_inner=1e-3, max_outer=20000, max_rounds=8)
    y0 = torch.zeros(packed.P, dtype=torch.float64, device="cuda")
    r0 = rm.rm_solve(ctx, packed, rm.RM_NAG, opts, omd, ald, dev(batch.f_packed()), y0)
    y1 = place([np.zeros((n, n)) for n in ns], torch.float64)
    r1 = rm.rm_solve(ctx, gapped, rm.RM_NAG, opts, omd, ald, place(batch.f, torch.float64), y1)
    assert r0["status"] == rm.RM_OK and r1["status"] == rm.RM_OK
    assert np.array_equal(r0["relres"], r1["relres"])
    for a, b in zip(unpack_vec(host(y0), ns), take(y1)):
        assert np.array_equal(a.ravel(), b)
    with pytest.raises(rm.RMError):
        rm.Plan(ctx, ns, eps=batch.eps, theta=batch.theta, offsets=[0, 200, 300, 20000])
