"""Two-grid Helmholtz cycle on the GPU against the oracle: forward iterates and
residual history, the adjoint (smoother weights, momentum factors, symbol, right-hand
side), bitwise agreement of blocked and one-step smoothing, determinism, and the
full-size batch (32 instances, n = 511) on sampled instances."""
import numpy as np
import pytest
import torch

from oracle import problem, twogrid
from synthetic import Batch, helmholtz_batch, twogrid_symbol, unpack_vec
from tests.gpu_helpers import dev, host, need_gpu, oracle_coef, plan_for, say

pytestmark = pytest.mark.gpu

NS = [7, 15, 31, 63, 127, 255]


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2412_08076_amd import rm
    return rm.Context(0)


def _meth(rm, name):
    return {"richardson": rm.RM_RICHARDSON, "nag": rm.RM_NAG, "mom": rm.RM_MOM, "nagex": rm.RM_NAGEX}[name]


def _batch(ns, seed, kappa_range=(2.0, 12.0)):
    rng = np.random.default_rng(seed)
    kappa = rng.uniform(*kappa_range, size=len(ns))
    f = [rng.standard_normal((k, k)) for k in ns]
    return Batch(ns, kappa=kappa, f=f, op="helmholtz")


def _inputs(batch, m, seed, jacobi=False, spread=0.2, resonant=True):
    """Smoother weights, momentum factors and symbols (rounded to FP32).  resonant=True
    inverts the fine-grid eigenvalues almost exactly (near-zero eigenvalues give
    large symbol entries); resonant=False regularises at 5 % of the Gershgorin bound."""
    rng = np.random.default_rng(seed)
    om = np.zeros((batch.B, m))
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        om[b] = rng.uniform(0.3, 0.9, m) / problem.gershgorin(c) * (c[0] if jacobi else 1.0)
    al = rng.uniform(0.1, 0.5, (batch.B, m))
    at = rng.uniform(0.1, 0.5, (batch.B, m))
    syms = []
    for b in range(batch.B):
        reg = 1.0 if resonant else 0.05 * problem.gershgorin(oracle_coef(batch, b))
        syms.append(twogrid_symbol(batch.kappa[b], batch.n[b], seed=seed + b, spread=spread, reg=reg))
    # every input rounded to FP32 once, so both sides see the same values
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return r32(om), r32(al), r32(at), [r32(s) for s in syms]


def _symbol_dev(plan, syms):
    coff = plan.coarse_offsets()
    flat = np.zeros(plan.coarse_points())
    for b, s in enumerate(syms):
        flat[coff[b]:coff[b] + s.size] = s.ravel()
    return dev(flat, torch.float32), coff


def _alpha_dev(name, al, at):
    return dev(np.concatenate([al.ravel(), at.ravel()]) if name == "nagex" else al.ravel(), torch.float32)


@pytest.mark.parametrize("resonant", [False, True])
@pytest.mark.parametrize("name,jacobi", [("nag", False), ("nagex", True), ("mom", False), ("richardson", False)])
def test_twogrid_forward_matches_oracle(ctx, name, jacobi, resonant):
    from paper_2412_08076_amd import rm
    batch = _batch(NS, seed=31)
    plan = plan_for(ctx, batch)
    m, K = 4, 3
    say("two-grid forward", name, jacobi, "resonant" if resonant else "regularised", NS)
    om, al, at, syms = _inputs(batch, m, 1, jacobi, resonant=resonant)
    sym_d, _ = _symbol_dev(plan, syms)
    f32 = batch.f_packed().astype(np.float32)
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    ck = torch.zeros(K * plan.P, dtype=torch.float32, device="cuda")
    hist = torch.zeros(K * plan.B, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, jacobi=jacobi)
    rm.rm_twogrid_solve(ctx, plan, _meth(rm, name), opts, dev(om, torch.float32), _alpha_dev(name, al, at), sym_d,
                        dev(f32, torch.float32), x, ckpt=ck, hist=hist)
    xs = unpack_vec(host(x), batch.n)
    hs = host(hist).reshape(K, plan.B)
    cks = [unpack_vec(host(ck)[k * plan.P:(k + 1) * plan.P], batch.n) for k in range(K)]
    fs = unpack_vec(f32.astype(np.float64), batch.n)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        binv = (lambda r, d=c[0]: r / d) if jacobi else None
        kw = {} if name == "richardson" else dict(alpha=al[b], alpha_t=at[b])
        u, hist_o = twogrid.run(name, c, fs[b], om[b], syms[b], K, binv=binv, history=True, **kw)
        fn = np.linalg.norm(fs[b])
        err = np.linalg.norm(xs[b] - u) / np.linalg.norm(u)
        # element by element as well, relative to the largest entry
        sup = np.max(np.abs(xs[b] - u)) / np.max(np.abs(u))
        rr_gpu = problem.relres(c, fs[b], xs[b])
        tol = 1e-5
        say("  n", batch.n[b], "kappa", round(batch.kappa[b], 3), "relres", hist_o[-1], rr_gpu, "err", err,
            "sup err", sup)
        assert err <= tol, (b, err, tol)
        assert sup <= tol, (b, sup, tol)
        assert abs(rr_gpu - hist_o[-1]) <= tol * max(1.0, hist_o[-1])
        np.testing.assert_allclose(np.sqrt(hs[:, b]) / fn, hist_o, rtol=1e-3, atol=1e-5)
        assert np.array_equal(cks[0][b], np.zeros_like(cks[0][b]))
        u1 = twogrid.run(name, c, fs[b], om[b], syms[b], 1, binv=binv, **kw)
        assert np.linalg.norm(cks[1][b] - u1) / np.linalg.norm(u1) <= tol


@pytest.mark.parametrize("resonant", [False, True])
@pytest.mark.parametrize("name,jacobi", [("nag", False), ("nagex", True), ("mom", False)])
def test_twogrid_adjoint_matches_oracle(ctx, name, jacobi, resonant):
    from paper_2412_08076_amd import rm
    ns = [7, 15, 63, 127]
    batch = _batch(ns, seed=37)
    plan = plan_for(ctx, batch)
    m, K = 3, 2
    say("two-grid adjoint", name, jacobi, "resonant" if resonant else "regularised", ns)
    om, al, at, syms = _inputs(batch, m, 3, jacobi, resonant=resonant)
    sym_d, coff = _symbol_dev(plan, syms)
    f32 = batch.f_packed().astype(np.float32)
    fd = dev(f32, torch.float32)
    omd, ald = dev(om, torch.float32), _alpha_dev(name, al, at)
    meth = _meth(rm, name)
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, jacobi=jacobi)
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    ck = torch.zeros(K * plan.P, dtype=torch.float32, device="cuda")
    rm.rm_twogrid_solve(ctx, plan, meth, opts, omd, ald, sym_d, fd, x, ckpt=ck)
    na = 2 if name == "nagex" else 1
    dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
    da = torch.empty(na * plan.B * m, dtype=torch.float32, device="cuda")
    ds = torch.empty(plan.coarse_points(), dtype=torch.float32, device="cuda")
    db = torch.empty(plan.P, dtype=torch.float32, device="cuda")
    loss = torch.empty(plan.B, dtype=torch.float32, device="cuda")
    rm.rm_twogrid_adjoint(ctx, plan, meth, opts, omd, ald, sym_d, fd, ck, dw, da, ds, d_b=db, loss=loss)
    dwh, dah, dsh = host(dw).reshape(plan.B, m), host(da).reshape(na, plan.B, m), host(ds)
    dbs = unpack_vec(host(db), ns)
    fs = unpack_vec(f32.astype(np.float64), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        dinv = 1.0 / c[0] if jacobi else 1.0
        L, gw, ga, gat, gs, gf = twogrid.loss_and_grads(name, c, fs[b], om[b], syms[b], K, alpha=al[b],
                                                        alpha_t=at[b], dinv=dinv)
        nc = (ns[b] - 1) // 2
        gsym = dsh[coff[b]:coff[b] + nc * nc].reshape(nc, nc)
        rel = lambda got, want: np.max(np.abs(got - want)) / np.max(np.abs(want))
        want_a = ga + gat if name == "nag" else ga
        errs = [abs(host(loss)[b] - L) / L, rel(dwh[b], gw), rel(gsym, gs), rel(dbs[b], gf), rel(dah[0, b], want_a)]
        if name == "nagex":
            errs.append(rel(dah[1, b], gat))
        say("  n", ns[b], "kappa", round(batch.kappa[b], 3), "loss", L, "errs", ["%.2e" % e for e in errs])
        assert errs[0] <= 1e-5
        assert max(errs[1:]) <= 1e-4


def test_twogrid_blocked_equals_one_step_and_is_deterministic(ctx):
    from paper_2412_08076_amd import rm
    ns = [15, 63, 127, 255, 255]
    batch = _batch(ns, seed=41)
    m, K = 8, 3
    om, al, _, syms = _inputs(batch, m, 5)
    outs = []
    for cfg in (None, (-1, 1), (2, 4)):
        plan = plan_for(ctx, batch)
        if cfg is not None:
            plan.set_kernel(*cfg)
        sym_d, _ = _symbol_dev(plan, syms)
        fd = dev(batch.f_packed(), torch.float32)
        omd, ald = dev(om, torch.float32), dev(al, torch.float32)
        opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K)
        x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
        ck = torch.zeros(K * plan.P, dtype=torch.float32, device="cuda")
        rm.rm_twogrid_solve(ctx, plan, rm.RM_NAG, opts, omd, ald, sym_d, fd, x, ckpt=ck)
        grads = []
        for _ in range(2):
            dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
            da = torch.empty_like(dw)
            ds = torch.empty(plan.coarse_points(), dtype=torch.float32, device="cuda")
            db = torch.empty(plan.P, dtype=torch.float32, device="cuda")
            rm.rm_twogrid_adjoint(ctx, plan, rm.RM_NAG, opts, omd, ald, sym_d, fd, ck, dw, da, ds, d_b=db)
            grads.append([host(t) for t in (dw, da, ds, db)])
        for a, b in zip(grads[0], grads[1]):
            assert np.array_equal(a, b)
        say("config", cfg, "done")
        outs.append([host(x)] + grads[0])
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_twogrid_rejects_sizes_and_handles_zero_cycles(ctx):
    from paper_2412_08076_amd import rm
    bad = _batch([15, 100], seed=43)
    plan = plan_for(ctx, bad)
    assert plan.coarse_points() == -1
    m = 2
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=1)
    om = torch.ones(plan.B * m, dtype=torch.float32, device="cuda") * 1e-4
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    f = dev(bad.f_packed(), torch.float32)
    lib = ctx.lib
    st = lib.rm_twogrid_solve(ctx.handle, plan.handle, rm.RM_RICHARDSON, opts, om.data_ptr(), None,
                              x.data_ptr(), f.data_ptr(), x.data_ptr(), None, None)
    assert st == rm._lib.RM_EUNSUPPORTED
    good = _batch([31], seed=44)
    plan = plan_for(ctx, good)
    _, _, _, syms = _inputs(good, m, 6)
    sym_d, _ = _symbol_dev(plan, syms)
    x0 = torch.randn(plan.P, dtype=torch.float32, device="cuda")
    x = x0.clone()
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=0)
    rm.rm_twogrid_solve(ctx, plan, rm.RM_RICHARDSON, opts, om[:m].contiguous(), None, sym_d,
                        dev(good.f_packed(), torch.float32), x)
    assert torch.equal(x, x0)


def test_twogrid_full_size_sampled(ctx):
    """32 Helmholtz instances at n = 511, kappa in [20, 80], Gaussian point sources,
    NAG-Richardson(8) smoothing: forward iterates of sampled instances against the oracle."""
    from paper_2412_08076_amd import rm
    batch = helmholtz_batch(B=32, n=511, seed=5)
    plan = plan_for(ctx, batch)
    m, K = 8, 2
    rng = np.random.default_rng(7)
    om = np.zeros((batch.B, m))
    for b in range(batch.B):
        om[b] = rng.uniform(0.25, 1.0, m) / problem.gershgorin(oracle_coef(batch, b))
    om = om.astype(np.float32).astype(np.float64)
    al = np.full((batch.B, m), 0.2, dtype=np.float32).astype(np.float64)
    f32 = batch.f_packed().astype(np.float32)
    fs = unpack_vec(f32.astype(np.float64), batch.n)
    for resonant in (False, True):
        syms = []
        for b in range(batch.B):
            reg = 1.0 if resonant else 0.05 * problem.gershgorin(oracle_coef(batch, b))
            syms.append(twogrid_symbol(batch.kappa[b], 511, reg=reg).astype(np.float32).astype(np.float64))
        sym_d, _ = _symbol_dev(plan, syms)
        x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
        opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K)
        say("two-grid full size B=32 n=511", "resonant" if resonant else "regularised")
        rm.rm_twogrid_solve(ctx, plan, rm.RM_NAG, opts, dev(om, torch.float32), dev(al, torch.float32), sym_d,
                            dev(f32, torch.float32), x)
        xs = unpack_vec(host(x), batch.n)
        for b in (0, 13, 31):
            c = oracle_coef(batch, b)
            u = twogrid.run("nag", c, fs[b], om[b], syms[b], K, alpha=al[b])
            rr = problem.relres(c, fs[b], u)
            rr_gpu = problem.relres(c, fs[b], xs[b])
            err = np.linalg.norm(xs[b] - u) / np.linalg.norm(u)
            # how far an FP32 rounding of the iterate alone moves the relative residual
            # (large near resonance, where the symbol amplifies the high modes): the GPU
            # rounds once per smoothing step, so its residual may differ by m K times that
            e32 = float(np.finfo(np.float32).eps)
            prng = np.random.default_rng(b)
            drr = max(abs(problem.relres(c, fs[b], u * (1.0 + e32 * prng.choice([-1.0, 1.0], u.shape))) - rr)
                      for _ in range(2))
            say("  instance", b, "kappa", round(batch.kappa[b], 2), "relres", rr, rr_gpu, "err", err,
                "fp32 residual sensitivity", drr)
            assert err <= 1e-5
            assert abs(rr_gpu - rr) <= 1e-5 * max(1.0, rr) + m * K * drr


def test_twogrid_autograd_function(ctx):
    """TwoGridLoss: weighted per-instance losses back-propagated through torch autograd
    equal the oracle's gradients for omega, alpha, the symbol and b."""
    from paper_2412_08076_amd import rm
    from paper_2412_08076_amd.autograd import TwoGridLoss
    ns = [15, 31, 63]
    batch = _batch(ns, seed=71)
    plan = plan_for(ctx, batch)
    m, K = 3, 2
    om, al, _, syms = _inputs(batch, m, 8, resonant=False)
    sym_d, coff = _symbol_dev(plan, syms)
    f32 = batch.f_packed().astype(np.float32)
    omega = dev(om, torch.float32).requires_grad_(True)
    alpha = dev(al, torch.float32).requires_grad_(True)
    symbol = sym_d.clone().requires_grad_(True)
    b = dev(f32, torch.float32).requires_grad_(True)
    wts = torch.tensor([0.5, 1.0, 2.0], dtype=torch.float32, device="cuda")
    loss = TwoGridLoss.apply(omega, alpha, symbol, b, ctx, plan, rm.RM_NAG, m, K)
    (loss * wts).sum().backward()
    gb = unpack_vec(host(b.grad), ns)
    fs = unpack_vec(f32.astype(np.float64), ns)
    for i in range(batch.B):
        c = oracle_coef(batch, i)
        L, gw, ga, gat, gs, gf = twogrid.loss_and_grads("nag", c, fs[i], om[i], syms[i], K, alpha=al[i])
        w = float(wts[i])
        nc = (ns[i] - 1) // 2
        rel = lambda got, want: np.max(np.abs(got - want)) / np.max(np.abs(want))
        assert abs(host(loss)[i] - L) <= 1e-5 * L
        assert rel(host(omega.grad)[i], w * gw) <= 1e-4
        assert rel(host(alpha.grad)[i], w * (ga + gat)) <= 1e-4
        assert rel(host(symbol.grad)[coff[i]:coff[i] + nc * nc].reshape(nc, nc), w * gs) <= 1e-4
        assert rel(gb[i], w * gf) <= 1e-4
