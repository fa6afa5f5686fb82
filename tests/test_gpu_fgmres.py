"""Batched FGMRES on the GPU against the FGMRES oracle: plain GMRES (with the same FP32
rounding of the basis vector as preconditioner), a Table-1 neural-solver preconditioner,
a two-grid preconditioner solving Helmholtz problems to 1e-10, statuses and errors."""
import numpy as np
import pytest
import torch

from oracle import iterate, krylov, problem, twogrid
from synthetic import Batch, random_batch, twogrid_symbol, unpack_vec
from tests.gpu_helpers import dev, host, need_gpu, oracle_coef, plan_for, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2412_08076_amd import rm
    return rm.Context(0)


def _fl32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def test_gmres_matches_oracle(ctx):
    from paper_2412_08076_amd import rm
    ns = [9, 17, 33, 40]
    batch = random_batch(ns, seed=61, eps_range=(1e-2, 1.0))
    plan = plan_for(ctx, batch)
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    say("gmres", ns)
    rep = rm.rm_fgmres(ctx, plan, dev(batch.f_packed()), x, restart=6, max_iter=15, tol=1e-14)
    assert np.all(rep["outer_iters"] == 15) and np.all(rep["inst_status"] == rm.RM_ENOTCONV)
    xs = unpack_vec(host(x), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        A = lambda v, c=c: problem.apply_A(c, v)
        xo, hist, it = krylov.fgmres(A, batch.f[b], precond=lambda j, v: _fl32(v), restart=6, max_iter=15, tol=1e-14)
        err = np.linalg.norm(xs[b] - xo) / np.linalg.norm(xo)
        say("  n", ns[b], "relres", hist[-1], rep["relres"][b], "err", err)
        assert err <= 1e-10
        assert abs(problem.relres(c, batch.f[b], xs[b]) - hist[-1]) <= 1e-10 * max(1.0, hist[-1])


def test_fgmres_with_neural_solver_preconditioner(ctx):
    """K = 8 steps of NAG-Richardson(4) as the preconditioner: FP32 on the GPU, FP64 on
    the oracle (same FP32 input), so the directions differ at FP32 rounding."""
    from paper_2412_08076_amd import rm
    ns = [17, 33, 64]
    batch = random_batch(ns, seed=63, eps_range=(1e-3, 1.0))
    plan = plan_for(ctx, batch)
    m, K = 4, 8
    rng = np.random.default_rng(5)
    om = np.stack([_fl32(rng.uniform(0.4, 1.0, m) / problem.gershgorin(oracle_coef(batch, b))) for b in range(batch.B)])
    al = _fl32(np.full((batch.B, m), 0.5))
    inner = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K)
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    say("fgmres NS preconditioner", ns)
    rep = rm.rm_fgmres(ctx, plan, dev(batch.f_packed()), x, restart=5, max_iter=12, tol=1e-14, method=rm.RM_NAG,
                       inner=inner, omega=dev(om, torch.float32), alpha=dev(al, torch.float32))
    xs = unpack_vec(host(x), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        A = lambda v, c=c: problem.apply_A(c, v)
        M = lambda j, v, c=c, b=b: iterate.run("nag", c, _fl32(v), om[b], K, alpha=al[b])[0]
        xo, hist, it = krylov.fgmres(A, batch.f[b], precond=M, restart=5, max_iter=12, tol=1e-14)
        err = np.linalg.norm(xs[b] - xo) / np.linalg.norm(xo)
        rr = problem.relres(c, batch.f[b], xs[b])
        say("  n", ns[b], "relres", hist[-1], rr, "err", err)
        assert err <= 1e-5
        assert abs(rr - hist[-1]) <= 1e-5 * max(1.0, hist[-1])


def test_fgmres_two_grid_preconditioner_reaches_1e10(ctx):
    from paper_2412_08076_amd import rm
    ns = [31, 63, 127, 127]
    rng = np.random.default_rng(67)
    kappa = np.array([10.0, 25.0, 30.0, 45.0])
    f = [rng.standard_normal((k, k)) for k in ns]
    batch = Batch(ns, kappa=kappa, f=f, op="helmholtz")
    plan = plan_for(ctx, batch)
    m = 4
    om = np.stack([np.full(m, 0.5 / problem.gershgorin(oracle_coef(batch, b))) for b in range(batch.B)])
    coff = plan.coarse_offsets()
    sym = np.zeros(plan.coarse_points())
    for b in range(batch.B):
        s_b = twogrid_symbol(kappa[b], ns[b])
        sym[coff[b]:coff[b] + s_b.size] = s_b.ravel()
    inner = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=1)
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    say("fgmres two-grid preconditioner", ns)
    rep = rm.rm_fgmres(ctx, plan, dev(batch.f_packed()), x, restart=20, max_iter=400, tol=1e-10,
                       method=rm.RM_RICHARDSON, inner=inner, omega=dev(om, torch.float32),
                       symbol=dev(sym, torch.float32))
    say("  iters", rep["outer_iters"], "rounds", rep["rounds"], "relres", rep["relres"])
    assert rep["status"] == rm.RM_OK
    xs = unpack_vec(host(x), ns)
    for b in range(batch.B):
        rr = problem.relres(oracle_coef(batch, b), batch.f[b], xs[b])
        assert rr <= 1e-10 and abs(rr - rep["relres"][b]) <= 1e-12


def test_fgmres_statuses_and_errors(ctx):
    from paper_2412_08076_amd import rm
    batch = random_batch([17, 33], seed=69, eps_range=(1e-4, 1e-3))
    plan = plan_for(ctx, batch)
    b = dev(batch.f_packed())
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    rep = rm.rm_fgmres(ctx, plan, b, x, restart=3, max_iter=4, tol=1e-12)
    assert rep["status"] == rm.RM_ENOTCONV and np.all(rep["outer_iters"] == 4) and np.all(rep["rounds"] == 2)
    for kw in (dict(restart=0), dict(restart=65), dict(max_iter=0), dict(tol=0.0)):
        with pytest.raises(rm.RMError):
            rm.rm_fgmres(ctx, plan, b, x, **kw)
    # an exact initial guess finishes before any Arnoldi step
    x2 = torch.zeros_like(x)
    rep = rm.rm_fgmres(ctx, plan, torch.zeros_like(b), x2, restart=3, max_iter=4, tol=1e-12)
    assert rep["status"] == rm.RM_OK and np.all(rep["outer_iters"] == 0)
