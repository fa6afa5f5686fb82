"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances
  FP64 sweeps       a few ulp per step times the cycle's rounding amplification:
                    relative 1e-9 on iterates after 50 cycles of Chebyshev(8).
  FP32 sweeps       element-wise max|x_gpu - u_oracle| <= 2 eps32 K max|u_oracle| after K
                    steps with the same weights (tests.gpu_helpers.FP32_C), and
                    ||A (x_gpu - x_oracle)|| / ||f|| <= 1e-5.
  Refined (FP64)    reported relres <= tol; the oracle's FP64 residual of the GPU's x
                    agrees with the reported one to 1e-12 (absolute, relative to ||b||);
                    ||x - x*|| / ||x*|| <= kappa * tol.
  Adjoint (FP32)    loss to 1e-5 relative, gradients (also those of the meta network's
                    parameters) element-wise to 1e-4 of their max magnitude.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint, iterate, meta, problem, refine, spectra, weights
from synthetic import Batch, meta_params, pack, random_batch, single_isotropic, unpack_vec
from tests.gpu_helpers import assert_fp32_close, dev, host, need_gpu, oracle_coef, plan_for, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2412_08076_amd import rm
    return rm.Context(0)


def _rm():
    from paper_2412_08076_amd import rm
    return rm


RAGGED = [1, 2, 3, 7, 63, 64, 65, 100, 130]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_apply_A_parity(ctx, dtype):
    rm = _rm()
    say("apply_A", dtype, RAGGED)
    batch = random_batch(RAGGED, seed=11)
    plan = plan_for(ctx, batch)
    x = batch.f_packed()
    y = torch.empty(plan.P, dtype=dtype, device="cuda")
    rm.rm_apply_A(ctx, plan, dev(x, dtype), y)
    ys = unpack_vec(host(y), batch.n)
    xs = unpack_vec(x.astype(np.float32).astype(np.float64) if dtype == torch.float32 else x, batch.n)
    tol = 1e-14 if dtype == torch.float64 else 1e-6
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        want = problem.apply_A(c, xs[b])
        scale = np.sum(np.abs(c)) * np.max(np.abs(xs[b]))
        assert np.max(np.abs(ys[b] - want)) <= tol * scale, (b, batch.n[b])


def test_apply_A_helmholtz_parity(ctx):
    rm = _rm()
    say("apply_A helmholtz")
    rng = np.random.default_rng(4)
    ns = [5, 64, 97]
    batch = Batch(ns, kappa=rng.uniform(20, 80, len(ns)), f=[rng.standard_normal((k, k)) for k in ns],
                  op="helmholtz")
    plan = plan_for(ctx, batch)
    y = torch.empty(plan.P, dtype=torch.float64, device="cuda")
    rm.rm_apply_A(ctx, plan, dev(batch.f_packed()), y)
    ys = unpack_vec(host(y), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        want = problem.apply_A(c, batch.f[b])
        assert np.max(np.abs(ys[b] - want)) <= 1e-14 * np.sum(np.abs(c)) * np.max(np.abs(batch.f[b]))


def test_residual_and_norms(ctx):
    rm = _rm()
    say("residual")
    batch = random_batch([9, 64, 70], seed=5)
    plan = plan_for(ctx, batch)
    rng = np.random.default_rng(6)
    xs = [rng.standard_normal((k, k)) for k in batch.n]
    r = torch.empty(plan.P, dtype=torch.float64, device="cuda")
    r2 = torch.empty(plan.B, dtype=torch.float64, device="cuda")
    b2 = torch.empty_like(r2)
    rel2 = torch.empty(plan.B, dtype=torch.float32, device="cuda")
    rm.rm_residual(ctx, plan, dev(batch.f_packed()), dev(pack(xs)), r, r2, b2, rel2)
    rs = unpack_vec(host(r), batch.n)
    for b in range(batch.B):
        want = problem.residual(oracle_coef(batch, b), batch.f[b], xs[b])
        assert np.allclose(rs[b], want, rtol=0, atol=1e-12 * np.max(np.abs(want)))
        assert abs(host(r2)[b] - np.sum(want * want)) <= 1e-12 * np.sum(want * want)
        assert abs(host(b2)[b] - np.sum(batch.f[b] ** 2)) <= 1e-12 * np.sum(batch.f[b] ** 2)
        assert abs(host(rel2)[b] - np.sum(want * want) / np.sum(batch.f[b] ** 2)) <= 1e-6 * host(rel2)[b]


def test_fp64_richardson_single_isotropic(ctx):
    """n = 63, eps = 1, Richardson(8) with Chebyshev weights, 400 inner steps, FP64 sweeps."""
    rm = _rm()
    say("fp64 richardson(8) n=63 K=400")
    batch = single_isotropic(63, seed=0)
    lmin, lmax = spectra.q1_extreme_eigenvalues(1.0, 0.0, 63)
    w32 = weights.chebyshev_weights(lmin, lmax, 8).astype(np.float32)
    plan = plan_for(ctx, batch)
    K = 400
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    hist = torch.empty(K // 8 * plan.B, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F64, m=8, K=K)
    rm.rm_solve(ctx, plan, rm.RM_RICHARDSON, opts, dev(w32, torch.float32), None, dev(batch.f[0]), x, hist=hist)
    coef = oracle_coef(batch, 0)
    u, _, h = iterate.run(iterate.RICHARDSON, coef, batch.f[0], w32.astype(np.float64), K, history=True)
    got = host(x).reshape(63, 63)
    assert np.linalg.norm(got - u) <= 1e-9 * np.linalg.norm(u)
    fn2 = np.sum(batch.f[0] ** 2)
    assert np.allclose(np.sqrt(host(hist) / fn2), h, rtol=1e-8)


def _nag_weights(batch, m, seed, lo=0.5, hi=1.0, alo=0.8, ahi=0.95):
    rng = np.random.default_rng(seed)
    G = np.array([problem.gershgorin(oracle_coef(batch, b)) for b in range(batch.B)])
    om = (rng.uniform(lo, hi, (batch.B, m)) / G[:, None]).astype(np.float32)
    al = rng.uniform(alo, ahi, (batch.B, m)).astype(np.float32)
    return om, al


@pytest.mark.parametrize("method", ["nag", "richardson"])
def test_fp32_unroll_parity(ctx, method):
    rm = _rm()
    ns = [1, 5, 63, 64, 65, 130]
    say("fp32 unroll", method, ns)
    batch = random_batch(ns, seed=21)
    plan = plan_for(ctx, batch)
    m, K = 16, 64
    om, al = _nag_weights(batch, m, seed=3)
    meth = rm.RM_NAG if method == "nag" else rm.RM_RICHARDSON
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    hist = torch.empty(K // m * plan.B, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K)
    rm.rm_solve(ctx, plan, meth, opts, dev(om, torch.float32), dev(al, torch.float32),
                dev(batch.f_packed(), torch.float32), x, hist=hist)
    xs = unpack_vec(host(x), ns)
    hs = host(hist).reshape(K // m, plan.B)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        f32 = batch.f[b].astype(np.float32).astype(np.float64)
        if method == "nag":
            u, _, h = iterate.run(iterate.NAG, c, f32, om[b].astype(np.float64), K, alpha=al[b].astype(np.float64),
                                  history=True)
        else:
            u, _, h = iterate.run(iterate.RICHARDSON, c, f32, om[b].astype(np.float64), K, history=True)
        fn = np.linalg.norm(f32)
        err = np.linalg.norm(problem.apply_A(c, xs[b] - u)) / fn
        assert err <= 1e-5, (b, ns[b], err)
        assert_fp32_close(xs[b], u, K, (method, ns[b]))
        assert np.allclose(np.sqrt(hs[:, b]) / fn, h, rtol=1e-4, atol=1e-6)


def test_unroll_checkpoints_and_odd_K(ctx):
    rm = _rm()
    ns = [33, 70]
    say("checkpoints, odd K", ns)
    batch = random_batch(ns, seed=8)
    plan = plan_for(ctx, batch)
    m, K, E = 3, 9, 3
    om, al = _nag_weights(batch, m, seed=2)
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    ck = torch.empty(K // E * 2 * plan.P, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F64, m=m, K=K, ckpt_every=E)
    rm.rm_solve(ctx, plan, rm.RM_NAG, opts, dev(om, torch.float32), dev(al, torch.float32),
                dev(batch.f_packed()), x, ckpt=ck)
    ckh = host(ck).reshape(K // E, 2, plan.P)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        us, vs = adjoint.unroll_states(c, batch.f[b], om[b].astype(np.float64), al[b].astype(np.float64), K)
        assert np.allclose(unpack_vec(host(x), ns)[b], us[K], rtol=0, atol=1e-12 * np.max(np.abs(us[K])))
        for cidx in range(K // E):
            s = cidx * E
            got_u = unpack_vec(ckh[cidx, 0], ns)[b]
            got_v = unpack_vec(ckh[cidx, 1], ns)[b]
            assert np.allclose(got_u, us[s], atol=1e-12 * (1 + np.max(np.abs(us[s]))))
            assert np.allclose(got_v, vs[s], atol=1e-12 * (1 + np.max(np.abs(vs[s]))))


@pytest.mark.parametrize("tol", [1e-10, 1e-12])
def test_refined_solve_parity(ctx, tol):
    rm = _rm()
    ns = [7, 33, 63, 65]
    say("refined solve", ns, tol)
    batch = random_batch(ns, seed=31, eps_range=(1e-2, 1.0))
    plan = plan_for(ctx, batch)
    m = 16
    om, al = _nag_weights(batch, m, seed=4, lo=0.9, hi=0.95, alo=0.9, ahi=0.9)
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=tol, tol_inner=1e-4, max_outer=20000, max_rounds=12,
                         check_every=2)
    rep = rm.rm_solve(ctx, plan, rm.RM_NAG, opts, dev(om, torch.float32), dev(al, torch.float32),
                      dev(batch.f_packed()), x)
    say("report", rep)
    assert rep["status"] == rm.RM_OK
    xs = unpack_vec(host(x), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        rho = problem.relres(c, batch.f[b], xs[b])
        assert rep["relres"][b] <= tol
        assert abs(rho - rep["relres"][b]) <= 1e-12
        xr, _, rhos, _ = refine.refined_solve(iterate.NAG, c, batch.f[b], om[b].astype(np.float64),
                                              tol=1e-14, alpha=al[b].astype(np.float64))
        n = ns[b]
        if n <= 33:
            from tests.test_oracle_problem import q1_assembled_matrix
            lam = np.linalg.eigvalsh(q1_assembled_matrix(batch.eps[b], batch.theta[b], n))
            kappa = lam.max() / lam.min()
        else:
            kappa = 4.0 * (n + 1) ** 2 / batch.eps[b]
        assert np.linalg.norm(xs[b] - xr) / np.linalg.norm(xr) <= kappa * tol


def test_refined_solve_richardson_and_statuses(ctx):
    rm = _rm()
    say("refined solve statuses")
    batch = random_batch([16, 16, 16], seed=41, eps_range=(0.1, 1.0))
    plan = plan_for(ctx, batch)
    m = 4
    G = np.array([problem.gershgorin(oracle_coef(batch, b)) for b in range(3)])
    om = np.tile((0.9 / G)[:, None], (1, m)).astype(np.float32)
    om[1, :] = 3.0 / G[1]       # omega * lambda_max > 2: Richardson diverges
    f = batch.f_packed()
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, max_outer=50, max_rounds=2, check_every=1)
    rep = rm.rm_solve(ctx, plan, rm.RM_RICHARDSON, opts, dev(om, torch.float32), None, dev(f), x)
    say("report", rep)
    assert rep["inst_status"][1] == rm.RM_EDIVERGED
    assert rep["inst_status"][0] in (rm.RM_OK, rm.RM_ENOTCONV)
    assert rep["status"] == rm.RM_EDIVERGED
    # a NaN in one right-hand side stops only that instance
    f2 = f.copy()
    f2[batch.offsets[2] + 5] = np.nan
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    om[1, :] = 0.9 / G[1]
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, max_outer=4000, max_rounds=6, check_every=2)
    rep = rm.rm_solve(ctx, plan, rm.RM_RICHARDSON, opts, dev(om, torch.float32), None, dev(f2), x)
    say("report", rep)
    assert rep["inst_status"][2] == rm.RM_EDIVERGED
    assert rep["inst_status"][0] == rm.RM_OK and rep["inst_status"][1] == rm.RM_OK


@pytest.mark.parametrize("graph", [False, True])
def test_refined_solve_iteration_cap_and_repeat(ctx, graph):
    # An unreachable tolerance with a small per-round cap: every round runs exactly
    # max_outer outer iterations (the stagnation window is longer), the report says
    # RM_ENOTCONV, and repeating the call in the same context, whose bookkeeping words
    # are numbered across calls, reproduces the result bit for bit.
    rm = _rm()
    batch = random_batch([17, 40, 65], seed=43, eps_range=(0.1, 1.0))
    plan = plan_for(ctx, batch)
    m = 4
    G = np.array([problem.gershgorin(oracle_coef(batch, b)) for b in range(batch.B)])
    om = dev(np.tile((0.9 / G)[:, None], (1, m)), torch.float32)
    al = dev(np.full((batch.B, m), 0.5), torch.float32)
    f = dev(batch.f_packed())
    for max_outer in (1, 2, 5):
        say("refined solve cap", max_outer, "graph", graph)
        opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-15, tol_inner=1e-14, max_outer=max_outer, max_rounds=2,
                             check_every=3, graph=graph)
        xs, reps = [], []
        for _ in range(2):
            x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
            reps.append(rm.rm_solve(ctx, plan, rm.RM_NAG, opts, om, al, f, x))
            xs.append(host(x))
        for rep in reps:
            assert rep["status"] == rm.RM_ENOTCONV
            assert np.all(rep["inst_status"] == rm.RM_ENOTCONV)
            assert np.all(rep["rounds"] == 2)
            assert np.all(rep["outer_iters"] == 2 * max_outer)
        assert np.array_equal(xs[0], xs[1])
        assert np.array_equal(reps[0]["relres"], reps[1]["relres"])


@pytest.mark.parametrize("method,E", [("nag", 4), ("nag", 8), ("richardson", 4)])
def test_adjoint_parity(ctx, method, E):
    rm = _rm()
    ns = [7, 40, 65]
    say("adjoint", method, E, ns)
    batch = random_batch(ns, seed=51)
    plan = plan_for(ctx, batch)
    m, K = 4, 16
    om, al = _nag_weights(batch, m, seed=5, alo=0.5, ahi=0.9)
    meth = rm.RM_NAG if method == "nag" else rm.RM_RICHARDSON
    if method == "richardson":
        al = np.zeros_like(al)
    f32 = batch.f_packed().astype(np.float32)
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=E)
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    ck = torch.empty(K // E * 2 * plan.P, dtype=torch.float32, device="cuda")
    omd, ald, fd = dev(om, torch.float32), dev(al, torch.float32), dev(f32, torch.float32)
    rm.rm_solve(ctx, plan, meth, opts, omd, ald, fd, x, ckpt=ck)
    dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
    da = torch.empty_like(dw)
    db = torch.empty(plan.P, dtype=torch.float32, device="cuda")
    loss = torch.empty(plan.B, dtype=torch.float32, device="cuda")
    gl = dev(np.array([1.0, 0.5, 2.0]), torch.float32)
    rm.rm_solve_adjoint(ctx, plan, meth, opts, omd, ald, fd, ck, dw, da, g_loss=gl, d_b=db, loss=loss)
    dwh, dah = host(dw).reshape(plan.B, m), host(da).reshape(plan.B, m)
    dbs = unpack_vec(host(db), ns)
    fs = unpack_vec(f32.astype(np.float64), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        L, gw, ga, gf = adjoint.loss_and_grads(c, fs[b], om[b].astype(np.float64), al[b].astype(np.float64), K)
        g = [1.0, 0.5, 2.0][b]
        assert abs(host(loss)[b] - L) <= 1e-5 * L
        assert np.max(np.abs(dwh[b] - g * gw)) <= 1e-4 * np.max(np.abs(g * gw))
        if method == "nag":
            assert np.max(np.abs(dah[b] - g * ga)) <= 1e-4 * np.max(np.abs(g * ga))
        else:
            assert np.all(dah[b] == 0.0)
        assert np.max(np.abs(dbs[b] - g * gf)) <= 1e-4 * np.max(np.abs(g * gf))
    # seed mode: J = <g_uK, u_K>
    rng = np.random.default_rng(9)
    gu = rng.standard_normal(plan.P).astype(np.float32)
    rm.rm_solve_adjoint(ctx, plan, meth, opts, omd, ald, fd, ck, dw, da, g_uK=dev(gu, torch.float32), d_b=db)
    gus = unpack_vec(gu.astype(np.float64), ns)
    dwh, dah = host(dw).reshape(plan.B, m), host(da).reshape(plan.B, m)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        _, gw, ga, gf = adjoint.loss_and_grads(c, fs[b], om[b].astype(np.float64), al[b].astype(np.float64), K,
                                               g_uK=gus[b])
        assert np.max(np.abs(dwh[b] - gw)) <= 1e-4 * np.max(np.abs(gw))
        assert np.max(np.abs(unpack_vec(host(db), ns)[b] - gf)) <= 1e-4 * np.max(np.abs(gf))


def test_meta_forward_backward_parity(ctx):
    rm = _rm()
    say("meta network")
    batch = random_batch([5, 9, 17, 33, 8, 8, 8, 12], seed=61)
    plan = plan_for(ctx, batch)
    m = 16
    params = meta_params(m=m, seed=0)
    p32 = params.astype(np.float32)
    om = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
    al = torch.empty_like(om)
    rm.rm_meta_forward(ctx, plan, m, dev(p32, torch.float32), om, al)
    coef, G = plan.coefficients()
    leps = np.log10(batch.eps).astype(np.float32).astype(np.float64)
    th = batch.theta.astype(np.float32).astype(np.float64)
    G32 = G.astype(np.float32).astype(np.float64)
    o_or, a_or, cache = meta.forward(p32.astype(np.float64), m, leps, th, G32)
    assert np.allclose(host(om).reshape(-1, m), o_or, rtol=2e-6)
    assert np.allclose(host(al).reshape(-1, m), a_or, rtol=2e-6)
    rng = np.random.default_rng(2)
    gw = rng.standard_normal((plan.B, m)).astype(np.float32)
    ga = rng.standard_normal((plan.B, m)).astype(np.float32)
    dp = torch.empty(len(params), dtype=torch.float32, device="cuda")
    rm.rm_meta_backward(ctx, plan, m, dev(p32, torch.float32), dev(gw, torch.float32), dev(ga, torch.float32), dp)
    want = meta.backward(p32.astype(np.float64), m, cache, gw.astype(np.float64), ga.astype(np.float64))
    assert np.max(np.abs(host(dp) - want)) <= 1e-5 * np.max(np.abs(want))
    # the plan's coefficients are the oracle's
    for b in range(batch.B):
        assert np.allclose(coef[b], oracle_coef(batch, b), rtol=1e-15, atol=1e-15)


def test_training_step_gradient(ctx):
    """MLP -> weights -> K-step NAG unroll -> loss -> adjoint -> MLP gradient, against the
    oracle chain (meta.forward, adjoint.loss_and_grads, meta.backward)."""
    rm = _rm()
    from paper_2412_08076_amd.autograd import MetaWeights, UnrollLoss
    say("training step")
    ns = [31, 31, 47, 64]
    batch = random_batch(ns, seed=71)
    plan = plan_for(ctx, batch)
    m, K, E = 16, 32, 16
    params = meta_params(m=m, seed=0).astype(np.float32)
    pt = dev(params, torch.float32).requires_grad_(True)
    f32 = batch.f_packed().astype(np.float32)
    om, al = MetaWeights.apply(pt, ctx, plan, m)
    loss = UnrollLoss.apply(om, al, dev(f32, torch.float32), ctx, plan, rm.RM_NAG, m, K, E)
    J = loss.mean()
    J.backward()
    _, G = plan.coefficients()
    leps = np.log10(batch.eps).astype(np.float32).astype(np.float64)
    th = batch.theta.astype(np.float32).astype(np.float64)
    o_or, a_or, cache = meta.forward(params.astype(np.float64), m, leps, th, G.astype(np.float32))
    fs = unpack_vec(f32.astype(np.float64), ns)
    gw = np.zeros((plan.B, m))
    ga = np.zeros((plan.B, m))
    Ls = []
    for b in range(plan.B):
        c = oracle_coef(batch, b)
        L, w_, a_, _ = adjoint.loss_and_grads(c, fs[b], o_or[b], a_or[b], K)
        Ls.append(L)
        gw[b], ga[b] = w_ / plan.B, a_ / plan.B
    assert abs(J.item() - np.mean(Ls)) <= 1e-5 * np.mean(Ls)
    want = meta.backward(params.astype(np.float64), m, cache, gw, ga)
    got = host(pt.grad)
    assert np.max(np.abs(got - want)) <= 1e-4 * np.max(np.abs(want))


def test_determinism(ctx):
    rm = _rm()
    say("determinism")
    batch = random_batch([65, 100], seed=81)
    plan = plan_for(ctx, batch)
    m, K = 8, 32
    om, al = _nag_weights(batch, m, seed=8)
    omd, ald = dev(om, torch.float32), dev(al, torch.float32)
    fd = dev(batch.f_packed(), torch.float32)
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=8)
    outs = []
    for _ in range(2):
        x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
        ck = torch.empty(K // 8 * 2 * plan.P, dtype=torch.float32, device="cuda")
        rm.rm_solve(ctx, plan, rm.RM_NAG, opts, omd, ald, fd, x, ckpt=ck)
        dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
        da = torch.empty_like(dw)
        rm.rm_solve_adjoint(ctx, plan, rm.RM_NAG, opts, omd, ald, fd, ck, dw, da)
        outs.append((host(x), host(dw), host(da)))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_invalid_arguments(ctx):
    rm = _rm()
    say("invalid arguments")
    with pytest.raises(rm.RMError) as e:
        rm.Plan(ctx, [8, 0], eps=[0.5, 0.5], theta=[0, 0])
    assert e.value.status == 1
    with pytest.raises(rm.RMError):
        rm.Plan(ctx, [8], eps=[0.0], theta=[0.0])
    with pytest.raises(rm.RMError):
        rm.Plan(ctx, [8], eps=[float("nan")], theta=[0.0])
    batch = random_batch([8], seed=1)
    plan = plan_for(ctx, batch)
    om = torch.full((8,), 0.1, dtype=torch.float32, device="cuda")
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    b = dev(batch.f_packed(), torch.float32)
    for bad in (dict(m=8, K=12), dict(m=0, K=0), dict(m=65, K=65), dict(m=8, K=16, ckpt_every=3)):
        opts = rm.solve_opts(mode=rm.RM_UNROLL, **bad)
        with pytest.raises((rm.RMError, ValueError)):
            rm.rm_solve(ctx, plan, rm.RM_RICHARDSON, opts, om[:max(bad["m"], 1)] if bad["m"] <= 8 else
                        torch.full((bad["m"],), 0.1, device="cuda"), None, b, x)
    opts = rm.solve_opts(mode=rm.RM_UNROLL, m=8, K=8)
    with pytest.raises(rm.RMError):
        rm.rm_solve(ctx, plan, rm.RM_NAG, opts, om, None, b, x)  # NAG needs alpha


def test_config2_full_size_sampled(ctx):
    """B = 256, n = 255 (the measured workload): FP32 unroll with meta-network weights
    checked on sampled instances, and the refined solve to 1e-10 checked on all
    instances through the oracle's FP64 residual of a sample."""
    rm = _rm()
    from synthetic import aniso_batch
    say("config B=256 n=255 sampled parity")
    batch = aniso_batch(256, 255, seed=2)
    plan = plan_for(ctx, batch)
    m = 16
    params = dev(meta_params(m=m, seed=0), torch.float32)
    om = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
    al = torch.empty_like(om)
    rm.rm_meta_forward(ctx, plan, m, params, om, al)
    fd32 = dev(batch.f_packed(), torch.float32)
    K = 32
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K)
    rm.rm_solve(ctx, plan, rm.RM_NAG, opts, om, al, fd32, x)
    omh, alh = host(om).reshape(-1, m), host(al).reshape(-1, m)
    xh = host(x)
    for b in (0, 77, 255):
        c = oracle_coef(batch, b)
        f32 = batch.f[b].astype(np.float32).astype(np.float64)
        u, _ = iterate.run(iterate.NAG, c, f32, omh[b], K, alpha=alh[b])
        got = xh[batch.offsets[b]:batch.offsets[b + 1]].reshape(255, 255)
        assert np.linalg.norm(problem.apply_A(c, got - u)) / np.linalg.norm(f32) <= 1e-5
        assert_fp32_close(got, u, K, ("n=255 meta weights", b))
    x64 = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, tol_inner=1e-4, max_outer=20000, max_rounds=10,
                         check_every=4)
    rep = rm.rm_solve(ctx, plan, rm.RM_NAG, opts, om, al, dev(batch.f_packed()), x64)
    say("outer iterations min/median/max", rep["outer_iters"].min(), np.median(rep["outer_iters"]),
        rep["outer_iters"].max(), "rounds max", rep["rounds"].max())
    assert rep["status"] == rm.RM_OK
    assert np.all(rep["relres"] <= 1e-10)
    xh = host(x64)
    for b in (3, 128, 200):
        c = oracle_coef(batch, b)
        got = xh[batch.offsets[b]:batch.offsets[b + 1]].reshape(255, 255)
        assert abs(problem.relres(c, batch.f[b], got) - rep["relres"][b]) <= 1e-12


def test_uneven_batch_sampled(ctx):
    """Mixed sizes from the uneven workload's size set in one plan (one size class each):
    FP32 NAG unroll against the oracle on one instance of every size."""
    rm = _rm()
    ns = [63] * 4 + [127] * 3 + [255] * 2 + [511] + [1023]
    say("uneven batch", ns)
    batch = random_batch(ns, seed=91)
    plan = plan_for(ctx, batch)
    say("kernels", {n: plan.get_kernel(n) for n in sorted(set(ns))})
    m, K = 16, 32
    om, al = _nag_weights(batch, m, seed=7, lo=0.9, hi=1.0, alo=0.9, ahi=0.99)
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    hist = torch.empty(K // m * plan.B, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K)
    rm.rm_solve(ctx, plan, rm.RM_NAG, opts, dev(om, torch.float32), dev(al, torch.float32),
                dev(batch.f_packed(), torch.float32), x, hist=hist)
    xs = unpack_vec(host(x), ns)
    hs = host(hist).reshape(K // m, plan.B)
    for b in (0, 4, 7, 9, 10):
        c = oracle_coef(batch, b)
        f32 = batch.f[b].astype(np.float32).astype(np.float64)
        u, _, h = iterate.run(iterate.NAG, c, f32, om[b].astype(np.float64), K, alpha=al[b].astype(np.float64),
                              history=True)
        fn = np.linalg.norm(f32)
        err = np.linalg.norm(problem.apply_A(c, xs[b] - u)) / fn
        assert err <= 1e-5, (b, ns[b], err)
        assert_fp32_close(xs[b], u, K, ("uneven", ns[b]))
        assert np.allclose(np.sqrt(hs[:, b]) / fn, h, rtol=1e-4)


def test_uneven_refined_solve(ctx):
    rm = _rm()
    ns = [7, 63, 63, 127, 200, 33]
    say("uneven refined", ns)
    batch = random_batch(ns, seed=93, eps_range=(1e-2, 1.0))
    plan = plan_for(ctx, batch)
    m = 16
    om, al = _nag_weights(batch, m, seed=8, lo=0.9, hi=1.0, alo=0.95, ahi=0.95)
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, tol_inner=1e-3, max_outer=20000, max_rounds=10)
    rep = rm.rm_solve(ctx, plan, rm.RM_NAG, opts, dev(om, torch.float32), dev(al, torch.float32),
                      dev(batch.f_packed()), x)
    say("report", rep)
    assert rep["status"] == rm.RM_OK and np.all(rep["relres"] <= 1e-10)
    xs = unpack_vec(host(x), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        assert abs(problem.relres(c, batch.f[b], xs[b]) - rep["relres"][b]) <= 1e-12


SCHEMES = [("mom", False), ("nagex", False), ("mom", True), ("nagex", True), ("nag", True), ("richardson", True)]


def _scheme_weights(batch, m, seed, jacobi):
    """omega scaled so that omega * lambda_max / (jacobi ? D : 1) stays below about 1."""
    rng = np.random.default_rng(seed)
    om = np.zeros((batch.B, m))
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        G = problem.gershgorin(c)
        om[b] = rng.uniform(0.5, 1.0, m) / G * (c[0] if jacobi else 1.0)
    al = rng.uniform(0.5, 0.9, (batch.B, m))
    at = rng.uniform(0.2, 0.9, (batch.B, m))
    return om.astype(np.float32), al.astype(np.float32), at.astype(np.float32)


def _meth(rm, name):
    return {"richardson": rm.RM_RICHARDSON, "nag": rm.RM_NAG, "mom": rm.RM_MOM, "nagex": rm.RM_NAGEX}[name]


@pytest.mark.parametrize("name,jacobi", SCHEMES)
def test_fp32_unroll_all_schemes(ctx, name, jacobi):
    """MOM- and NAGex-Richardson(m), and weighted-Jacobi preconditioning, against the
    oracle's Table-1 iterations (B^{-1} = I / D)."""
    rm = _rm()
    ns = [5, 63, 65, 130]
    say("fp32 unroll", name, "jacobi" if jacobi else "")
    batch = random_batch(ns, seed=101)
    plan = plan_for(ctx, batch)
    m, K = 4, 32
    om, al, at = _scheme_weights(batch, m, 3, jacobi)
    alpha = np.concatenate([al.ravel(), at.ravel()]) if name == "nagex" else al.ravel()
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, jacobi=jacobi)
    rm.rm_solve(ctx, plan, _meth(rm, name), opts, dev(om, torch.float32), dev(alpha, torch.float32),
                dev(batch.f_packed(), torch.float32), x)
    xs = unpack_vec(host(x), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        f32 = batch.f[b].astype(np.float32).astype(np.float64)
        binv = (lambda r, d=c[0]: r / d) if jacobi else None
        kw = dict(alpha=al[b].astype(np.float64), alpha_t=at[b].astype(np.float64))
        if name == "richardson":
            kw = {}
        u, _ = iterate.run(name, c, f32, om[b].astype(np.float64), K, binv=binv, **kw)
        err = np.linalg.norm(problem.apply_A(c, xs[b] - u)) / np.linalg.norm(f32)
        assert err <= 1e-5, (name, jacobi, b, err)
        assert_fp32_close(xs[b], u, K, (name, jacobi, ns[b]))


@pytest.mark.parametrize("name,jacobi", SCHEMES)
def test_adjoint_all_schemes(ctx, name, jacobi):
    rm = _rm()
    ns = [7, 40, 65]
    say("adjoint", name, "jacobi" if jacobi else "")
    batch = random_batch(ns, seed=103)
    plan = plan_for(ctx, batch)
    m, K, E = 4, 16, 8
    om, al, at = _scheme_weights(batch, m, 5, jacobi)
    alpha = np.concatenate([al.ravel(), at.ravel()]) if name == "nagex" else al.ravel()
    na = 2 if name == "nagex" else 1
    f32 = batch.f_packed().astype(np.float32)
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=E, jacobi=jacobi)
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    ck = torch.empty(K // E * 2 * plan.P, dtype=torch.float32, device="cuda")
    omd, ald, fd = dev(om, torch.float32), dev(alpha, torch.float32), dev(f32, torch.float32)
    meth = _meth(rm, name)
    rm.rm_solve(ctx, plan, meth, opts, omd, ald, fd, x, ckpt=ck)
    dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
    da = torch.empty(na * plan.B * m, dtype=torch.float32, device="cuda")
    db = torch.empty(plan.P, dtype=torch.float32, device="cuda")
    loss = torch.empty(plan.B, dtype=torch.float32, device="cuda")
    rm.rm_solve_adjoint(ctx, plan, meth, opts, omd, ald, fd, ck, dw, da, d_b=db, loss=loss)
    dwh = host(dw).reshape(plan.B, m)
    dah = host(da).reshape(na, plan.B, m)
    dbs = unpack_vec(host(db), ns)
    fs = unpack_vec(f32.astype(np.float64), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        dinv = 1.0 / c[0] if jacobi else 1.0
        L, gw, ga, gat, gf = adjoint.loss_and_grads_general(name, c, fs[b], om[b].astype(np.float64), K,
                                                            alpha=al[b].astype(np.float64),
                                                            alpha_t=at[b].astype(np.float64), dinv=dinv)
        assert abs(host(loss)[b] - L) <= 1e-5 * L
        assert np.max(np.abs(dwh[b] - gw)) <= 1e-4 * np.max(np.abs(gw))
        assert np.max(np.abs(dbs[b] - gf)) <= 1e-4 * np.max(np.abs(gf))
        if name == "nag":
            want = ga + gat
        elif name == "richardson":
            want = np.zeros(m)
        else:
            want = ga
        if name == "richardson":
            assert np.all(dah[0, b] == 0.0)
        else:
            assert np.max(np.abs(dah[0, b] - want)) <= 1e-4 * np.max(np.abs(want))
        if name == "nagex":
            assert np.max(np.abs(dah[1, b] - gat)) <= 1e-4 * np.max(np.abs(gat))


@pytest.mark.parametrize("name,jacobi", [("mom", True), ("nagex", False)])
def test_refined_solve_other_schemes(ctx, name, jacobi):
    rm = _rm()
    ns = [33, 64]
    say("refined", name, jacobi)
    batch = random_batch(ns, seed=107, eps_range=(0.1, 1.0))
    plan = plan_for(ctx, batch)
    m = 8
    om, al, at = _scheme_weights(batch, m, 7, jacobi)
    al[:] = 0.9
    at[:] = 0.7
    alpha = np.concatenate([al.ravel(), at.ravel()]) if name == "nagex" else al.ravel()
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, max_outer=20000, max_rounds=10, jacobi=jacobi)
    rep = rm.rm_solve(ctx, plan, _meth(rm, name), opts, dev(om, torch.float32), dev(alpha, torch.float32),
                      dev(batch.f_packed()), x)
    say("report", rep)
    assert rep["status"] == rm.RM_OK
    xs = unpack_vec(host(x), ns)
    for b in range(batch.B):
        assert abs(problem.relres(oracle_coef(batch, b), batch.f[b], xs[b]) - rep["relres"][b]) <= 1e-12
        assert rep["relres"][b] <= 1e-10


def test_context_destroyed_before_its_plans():
    """Destroying a context first detaches its plans: freeing them afterwards must not
    reach the freed context (C level), and the binding closes live plans first."""
    need_gpu()
    import ctypes
    from paper_2412_08076_amd import _lib, rm
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.rm_create(ctypes.byref(h), 0, None) == rm.RM_OK
    inst = (_lib.rm_instance * 2)()
    for b, n in enumerate((15, 33)):
        inst[b].n, inst[b].op, inst[b].eps, inst[b].theta, inst[b].kappa = n, rm.RM_Q1_ANISO, 0.5, 0.3, 0.0
    plans = []
    for _ in range(2):
        p = ctypes.c_void_p()
        assert lib.rm_plan(h, 2, inst, None, ctypes.byref(p)) == rm.RM_OK
        plans.append(p)
    assert lib.rm_plan_free(plans[0]) == rm.RM_OK
    assert lib.rm_destroy(h) == rm.RM_OK
    assert lib.rm_plan_free(plans[1]) == rm.RM_OK
    ctx = rm.Context(0)
    plan = rm.Plan(ctx, [15, 33], eps=[0.5, 0.5], theta=[0.3, 0.3])
    ctx.close()
    assert plan.handle is None
    plan.close()
