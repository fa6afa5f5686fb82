"""Mixed-size launch (rm_plan_set_mixed): one launch per chunk of steps over every size
class that runs the 8-step row pipeline, bit for bit equal to one launch per class and to
one launch per inner step.  Covered: K-step unrolls with the residual history (all four
schemes, Jacobi) and chunks of fewer than 8 steps; sizes whose sub-groups leave threads
over (n = 300: three windows of 320 threads and a rest of 64; n = 700: one window of
704 threads and a rest of 320); several windows per instance, including a shorter last
window; a class outside the launch (a tiled main configuration); inactive instances;
the refined solve to 1e-10 with its reports and iteration counts, eager and with captured
outer iterations; plans with no class, or a single class, on the row pipeline."""
import numpy as np
import pytest
import torch

from oracle import problem
from synthetic import Batch, random_batch
from tests.gpu_helpers import dev, host, need_gpu, oracle_coef, plan_for, say

pytestmark = pytest.mark.gpu

# size -> row-window height of the row pipeline (n = windows of the whole height)
WINDOWS = {63: 63, 127: 127, 255: 66, 300: 100, 511: 117, 700: 260, 1023: 130}
NS = [63] * 5 + [127] * 4 + [255] * 3 + [300] * 2 + [511] * 2 + [700] + [1023] + [40] * 2


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2412_08076_amd import rm
    return rm.Context(0)


def _weights(batch, m, seed, lo=0.5, mom=(0.8, 0.97)):
    rng = np.random.default_rng(seed)
    G = np.array([problem.gershgorin(oracle_coef(batch, b)) for b in range(batch.B)])
    om = (rng.uniform(lo, 1.0, (batch.B, m)) / G[:, None]).astype(np.float32)
    al = rng.uniform(*mom, (batch.B, m)).astype(np.float32)
    return om, al


def _configure(plan, rm):
    for n, w in WINDOWS.items():
        if n in plan.n:
            plan.set_kernel(rm.STREAM_SHAPE, 8, n=n, cw=w)
    if 40 in plan.n:
        plan.set_kernel(0, 4, n=40)  # a tiled class: keeps its own launches


def _unroll(ctx, plan, method, om, al, f, m, K, jacobi=False):
    from paper_2412_08076_amd import rm
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    h = torch.zeros(K // m * plan.B, dtype=torch.float64, device="cuda")
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, jacobi=jacobi)
    rm.rm_solve(ctx, plan, method, opts, om, al, f, x, hist=h)
    return host(x), host(h)


@pytest.mark.parametrize("method_name,jacobi", [("nag", False), ("richardson", False), ("mom", True),
                                                ("nagex", True)])
def test_mixed_unroll_bitwise(ctx, method_name, jacobi):
    from paper_2412_08076_amd import rm
    method = {"nag": rm.RM_NAG, "richardson": rm.RM_RICHARDSON, "mom": rm.RM_MOM,
              "nagex": rm.RM_NAGEX}[method_name]
    batch = random_batch(NS, seed=17)
    plan = plan_for(ctx, batch)
    m, K = 8, 40  # 40 steps: five chunks of 8
    om, al = _weights(batch, m, 3)
    omd, ald = dev(om, torch.float32), dev(al, torch.float32)
    if method_name == "nagex":
        ald = torch.cat([ald, 0.5 * ald])
    f = dev(batch.f_packed(), torch.float32)
    plan.set_kernel(-1, 1)
    ref, ref_h = _unroll(ctx, plan, method, omd, ald, f, m, K, jacobi)
    _configure(plan, rm)
    say("mixed unroll", method_name, jacobi, {n: plan.get_kernel(n) for n in sorted(set(NS))})
    per, per_h = _unroll(ctx, plan, method, omd, ald, f, m, K, jacobi)
    plan.set_mixed(True)
    assert plan.get_mixed()
    got, got_h = _unroll(ctx, plan, method, omd, ald, f, m, K, jacobi)
    plan.set_mixed(False)
    assert np.array_equal(per, ref), np.max(np.abs(per - ref))
    assert np.array_equal(got, per), np.max(np.abs(got - per))
    # the residual partials are the same tiles' sums in the same order
    assert np.array_equal(got_h, per_h)
    assert np.allclose(got_h, ref_h, rtol=1e-12, atol=0)


def test_mixed_short_chunks_and_odd_counts(ctx):
    """K = 21 with m = 7: chunks of 7 steps (mixed launches of T = 7), three outer
    iterations with the residual after each."""
    from paper_2412_08076_amd import rm
    ns = [300, 63, 1023, 127, 700, 255, 255]
    batch = random_batch(ns, seed=23)
    plan = plan_for(ctx, batch)
    m, K = 7, 21
    om, al = _weights(batch, m, 4)
    omd, ald = dev(om, torch.float32), dev(al, torch.float32)
    f = dev(batch.f_packed(), torch.float32)
    plan.set_kernel(-1, 1)
    ref, ref_h = _unroll(ctx, plan, rm.RM_NAG, omd, ald, f, m, K)
    _configure(plan, rm)
    plan.set_mixed(True)
    say("mixed short chunks", ns)
    got, got_h = _unroll(ctx, plan, rm.RM_NAG, omd, ald, f, m, K)
    assert np.array_equal(got, ref), np.max(np.abs(got - ref))
    assert np.allclose(got_h, ref_h, rtol=1e-12, atol=0)


def test_mixed_refined_solve_equals_per_class(ctx):
    """The refined solve to 1e-10 on all sizes: the same iterate, reports and iteration
    counts with the mixed launch as with one launch per class (instances converge at
    different times, so the launch runs with inactive windows and left-out classes)."""
    from paper_2412_08076_amd import rm
    ns = [63, 63, 127, 255, 300, 511, 1023, 40]
    eps = [1.0, 0.05, 0.3, 1.0, 0.5, 0.2, 1.0, 0.7]
    theta = [0.0, 1.0, np.pi / 2, 0.3, 2.0, np.pi / 2, 0.0, 0.1]
    rng = np.random.default_rng(29)
    batch = Batch(ns, eps=eps, theta=theta, f=[rng.standard_normal((n, n)) for n in ns])
    plan = plan_for(ctx, batch)
    _configure(plan, rm)
    m = 16
    om, al = _weights(batch, m, 5, lo=0.9, mom=(0.985, 0.99))
    omd, ald, bd = dev(om, torch.float32), dev(al, torch.float32), dev(batch.f_packed())
    opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, tol_inner=0.05, max_outer=40000, max_rounds=16)
    out = []
    for mixed in (False, True):
        plan.set_mixed(mixed)
        x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
        rep = rm.rm_solve(ctx, plan, rm.RM_NAG, opts, omd, ald, bd, x)
        say("refined, mixed" if mixed else "refined, per class", "outer", rep["outer_iters"], "rounds",
            rep["rounds"])
        assert rep["status"] == rm.RM_OK
        out.append((host(x), rep))
    (x0, r0), (x1, r1) = out
    assert np.array_equal(x0, x1)
    for key in ("outer_iters", "rounds", "relres"):
        assert np.array_equal(np.asarray(r0[key]), np.asarray(r1[key])), key
    assert np.all(np.asarray(r1["relres"]) <= 1e-10)


def test_mixed_refined_solve_with_graphs(ctx):
    """The refined solve with captured outer iterations (one graph per combination of
    class configurations, the mixed launch inside): the same iterate and reports as the
    eager per-class solve, on two calls in a row."""
    from paper_2412_08076_amd import rm
    ns = [63, 127, 255, 511, 1023, 63]
    batch = random_batch(ns, seed=41, eps_range=(0.1, 1.0))
    plan = plan_for(ctx, batch)
    _configure(plan, rm)
    m = 16
    om, al = _weights(batch, m, 6, lo=0.9, mom=(0.985, 0.99))
    omd, ald, bd = dev(om, torch.float32), dev(al, torch.float32), dev(batch.f_packed())
    base = dict(mode=rm.RM_TO_TOL, m=m, tol=1e-10, tol_inner=0.05, max_outer=40000, max_rounds=16)
    runs = []
    for mixed, graph in ((False, False), (True, True), (True, True)):
        plan.set_mixed(mixed)
        x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
        rep = rm.rm_solve(ctx, plan, rm.RM_NAG, rm.solve_opts(graph=graph, **base), omd, ald, bd, x)
        say("refined", "mixed" if mixed else "per class", "graph" if graph else "eager", "outer",
            rep["outer_iters"])
        assert rep["status"] == rm.RM_OK
        runs.append((host(x), rep))
    for x1, r1 in runs[1:]:
        assert np.array_equal(x1, runs[0][0])
        for key in ("outer_iters", "rounds", "relres"):
            assert np.array_equal(np.asarray(r1[key]), np.asarray(runs[0][1][key])), key


def test_mixed_without_row_pipeline_classes(ctx):
    """A plan whose classes all run tiled kernels (nothing for the mixed launch) and a plan
    of a single row-pipeline class: the setting changes nothing in the results."""
    from paper_2412_08076_amd import rm
    for ns, cfg in (([40, 63, 100], lambda plan: plan.set_kernel(0, 4)),
                    ([511, 511, 511], lambda plan: plan.set_kernel(rm.STREAM_SHAPE, 8, cw=117))):
        batch = random_batch(ns, seed=43)
        plan = plan_for(ctx, batch)
        cfg(plan)
        m, K = 8, 24
        om, al = _weights(batch, m, 7)
        omd, ald = dev(om, torch.float32), dev(al, torch.float32)
        f = dev(batch.f_packed(), torch.float32)
        say("mixed setting on", ns)
        a, ah = _unroll(ctx, plan, rm.RM_NAG, omd, ald, f, m, K)
        plan.set_mixed(True)
        b, bh = _unroll(ctx, plan, rm.RM_NAG, omd, ald, f, m, K)
        assert np.array_equal(a, b)
        assert np.array_equal(ah, bh)


def test_mixed_setting_round_trip(ctx):
    from paper_2412_08076_amd import rm
    batch = random_batch([31, 64], seed=1)
    plan = plan_for(ctx, batch)
    assert not plan.get_mixed()
    plan.set_mixed(True)
    assert plan.get_mixed()
    plan.set_mixed(False)
    assert not plan.get_mixed()
