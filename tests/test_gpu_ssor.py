"""SSOR-preconditioned Table-1 schemes on the GPU against the oracle (four-colour
SSOR written as sparse triangular solves): FP64 and FP32 unrolls, the adjoint, the
FP64-refined solve, option errors, and independence from the blocked-kernel setting."""
import numpy as np
import pytest
import torch

from oracle import adjoint, iterate, precond, problem
from synthetic import random_batch, unpack_vec
from tests.gpu_helpers import dev, host, need_gpu, oracle_coef, plan_for, say

pytestmark = pytest.mark.gpu

NS = [1, 2, 3, 5, 17, 40, 64, 65, 97, 130]


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2412_08076_amd import rm
    return rm.Context(0)


def _meth(rm, name):
    return {"richardson": rm.RM_RICHARDSON, "nag": rm.RM_NAG, "mom": rm.RM_MOM, "nagex": rm.RM_NAGEX}[name]


def _weights(B, m, seed):
    rng = np.random.default_rng(seed)
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return r32(rng.uniform(0.6, 1.2, (B, m))), r32(rng.uniform(0.2, 0.7, (B, m))), r32(rng.uniform(0.2, 0.7, (B, m)))


def _alpha(name, al, at):
    return dev(np.concatenate([al.ravel(), at.ravel()]) if name == "nagex" else al.ravel(), torch.float32)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", ["nagex", "nag", "mom", "richardson"])
def test_ssor_unroll_matches_oracle(ctx, name, dtype):
    from paper_2412_08076_amd import rm
    batch = random_batch(NS, seed=51)
    plan = plan_for(ctx, batch)
    m, K, relax = 3, 12, 1.3
    om, al, at = _weights(batch.B, m, 2)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    f = batch.f_packed()
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)
    x = torch.zeros(plan.P, dtype=tdt, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F64 if dtype == "f64" else rm.RM_F32, m=m, K=K, ssor=relax)
    say("ssor unroll", name, dtype)
    rm.rm_solve(ctx, plan, _meth(rm, name), opts, dev(om, torch.float32), _alpha(name, al, at), dev(f, tdt), x)
    xs = unpack_vec(host(x), batch.n)
    fs = unpack_vec(f, batch.n)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        kw = {} if name == "richardson" else dict(alpha=al[b], alpha_t=at[b])
        # the kernel applies the relaxation factor in its own precision
        rl = relax if dtype == "f64" else float(np.float32(relax))
        u, _ = iterate.run(name, c, fs[b], om[b], K, binv=precond.ssor_binv(c, rl), **kw)
        err = np.linalg.norm(xs[b] - u) / np.linalg.norm(u)
        # element by element as well: a wrong point or colour pass shows in the largest
        # deviation even where the norm of the whole field hides it
        sup = np.max(np.abs(xs[b] - u)) / np.max(np.abs(u))
        rr_o, rr_g = problem.relres(c, fs[b], u), problem.relres(c, fs[b], xs[b])
        say("  n", batch.n[b], "relres", rr_o, "err", err, "sup err", sup)
        tol = 1e-12 if dtype == "f64" else 1e-5
        assert err <= tol, (b, err)
        assert sup <= tol, (b, sup)
        assert abs(rr_g - rr_o) <= tol * max(1.0, rr_o)


@pytest.mark.parametrize("name", ["nagex", "nag", "mom", "richardson"])
def test_ssor_adjoint_matches_oracle(ctx, name):
    from paper_2412_08076_amd import rm
    ns = [9, 40, 64, 97]
    batch = random_batch(ns, seed=53)
    plan = plan_for(ctx, batch)
    # few enough steps that no loss falls where an FP32 residual is mostly rounding
    m, K, E, relax = 3, 6, 3, 1.1
    om, al, at = _weights(batch.B, m, 4)
    f32 = batch.f_packed().astype(np.float32)
    fd = dev(f32, torch.float32)
    omd, ald = dev(om, torch.float32), _alpha(name, al, at)
    meth = _meth(rm, name)
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=E, ssor=relax)
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    ck = torch.empty(K // E * 2 * plan.P, dtype=torch.float32, device="cuda")
    say("ssor adjoint", name)
    rm.rm_solve(ctx, plan, meth, opts, omd, ald, fd, x, ckpt=ck)
    na = 2 if name == "nagex" else 1
    dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
    da = torch.empty(na * plan.B * m, dtype=torch.float32, device="cuda")
    db = torch.empty(plan.P, dtype=torch.float32, device="cuda")
    loss = torch.empty(plan.B, dtype=torch.float32, device="cuda")
    rm.rm_solve_adjoint(ctx, plan, meth, opts, omd, ald, fd, ck, dw, da, d_b=db, loss=loss)
    dwh, dah = host(dw).reshape(plan.B, m), host(da).reshape(na, plan.B, m)
    dbs = unpack_vec(host(db), ns)
    fs = unpack_vec(f32.astype(np.float64), ns)
    for b in range(batch.B):
        c = oracle_coef(batch, b)
        L, gw, ga, gat, gf = adjoint.loss_and_grads_general(name, c, fs[b], om[b], K, alpha=al[b], alpha_t=at[b],
                                                            binv=precond.ssor_binv(c, float(np.float32(relax))))
        rel = lambda got, want: np.max(np.abs(got - want)) / np.max(np.abs(want))
        errs = [abs(host(loss)[b] - L) / L, rel(dwh[b], gw), rel(dbs[b], gf)]
        if name == "nag":
            errs.append(rel(dah[0, b], ga + gat))
        elif name in ("mom", "nagex"):
            errs.append(rel(dah[0, b], ga))
        if name == "nagex":
            errs.append(rel(dah[1, b], gat))
        say("  n", ns[b], "loss", L, "errs", ["%.2e" % e for e in errs])
        assert errs[0] <= 1e-5
        assert max(errs[1:]) <= 1e-4
        if name == "richardson":
            assert np.all(dah[0, b] == 0.0)


def test_ssor_refined_solve(ctx):
    from paper_2412_08076_amd import rm
    ns = [33, 64, 100]
    batch = random_batch(ns, seed=57, eps_range=(1e-2, 1.0))
    plan = plan_for(ctx, batch)
    m = 3
    om = np.full((batch.B, m), 1.2)
    al = np.full((batch.B, m), 0.8)
    x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, tol_inner=1e-3, max_outer=20000, max_rounds=10,
                         ssor=1.0)
    rep = rm.rm_solve(ctx, plan, rm.RM_NAGEX, opts, dev(om, torch.float32), _alpha("nagex", al, al),
                      dev(batch.f_packed()), x)
    say("ssor refined", rep["outer_iters"], rep["rounds"], rep["relres"])
    assert rep["status"] == rm.RM_OK
    xs = unpack_vec(host(x), ns)
    for b in range(batch.B):
        rr = problem.relres(oracle_coef(batch, b), batch.f[b], xs[b])
        assert abs(rr - rep["relres"][b]) <= 1e-12 and rr <= 1e-10


def test_ssor_options_and_blocking_independence(ctx):
    from paper_2412_08076_amd import rm
    batch = random_batch([40, 64], seed=59)
    plan = plan_for(ctx, batch)
    m, K = 3, 6
    om, al, _ = _weights(batch.B, m, 6)
    omd, ald = dev(om, torch.float32), dev(al, torch.float32)
    f = dev(batch.f_packed(), torch.float32)
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    for bad in (dict(ssor=2.0), dict(ssor=0.0), dict(ssor=1.0, jacobi=True)):
        with pytest.raises(rm.RMError):
            rm.rm_solve(ctx, plan, rm.RM_NAG, rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, **bad),
                        omd, ald, f, x)
    outs = []
    for cfg in ((-1, 1), (2, 4), (3, 8)):
        plan.set_kernel(*cfg)
        x.zero_()
        rm.rm_solve(ctx, plan, rm.RM_NAG, rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ssor=1.4),
                    omd, ald, f, x)
        outs.append(host(x))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_unroll_loss_autograd_with_ssor(ctx):
    """UnrollLoss with SSOR preconditioning: autograd gradients equal the oracle's."""
    from paper_2412_08076_amd import rm
    from paper_2412_08076_amd.autograd import UnrollLoss
    ns = [17, 40]
    batch = random_batch(ns, seed=73)
    plan = plan_for(ctx, batch)
    m, K, E, relax = 3, 6, 3, 1.2
    om, al, at = _weights(batch.B, m, 9)
    f32 = batch.f_packed().astype(np.float32)
    omega = dev(om, torch.float32).requires_grad_(True)
    alpha = dev(np.stack([al, at]), torch.float32).requires_grad_(True)
    b = dev(f32, torch.float32).requires_grad_(True)
    loss = UnrollLoss.apply(omega, alpha, b, ctx, plan, rm.RM_NAGEX, m, K, E, ("ssor", relax))
    loss.sum().backward()
    gb = unpack_vec(host(b.grad), ns)
    fs = unpack_vec(f32.astype(np.float64), ns)
    ga_all = host(alpha.grad)
    for i in range(batch.B):
        c = oracle_coef(batch, i)
        L, gw, ga, gat, gf = adjoint.loss_and_grads_general("nagex", c, fs[i], om[i], K, alpha=al[i], alpha_t=at[i],
                                                            binv=precond.ssor_binv(c, float(np.float32(relax))))
        rel = lambda got, want: np.max(np.abs(got - want)) / np.max(np.abs(want))
        assert abs(host(loss)[i] - L) <= 1e-5 * L
        assert rel(host(omega.grad)[i], gw) <= 1e-4
        assert rel(ga_all[0, i], ga) <= 1e-4 and rel(ga_all[1, i], gat) <= 1e-4
        assert rel(gb[i], gf) <= 1e-4
