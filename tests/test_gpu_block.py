"""Temporal-blocked FP32 sweeps: bitwise equal to one launch per inner step (the LDS
race / halo detector), for every kernel variant (tiled and row-streaming),
steps-per-launch T and several tile widths / row windows, on ragged sizes; autotuner
choices and cache."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import problem
from synthetic import random_batch
from tests.gpu_helpers import dev, host, need_gpu, oracle_coef, plan_for, say

pytestmark = pytest.mark.gpu

NS = [1, 3, 17, 40, 63, 64, 65, 97, 130, 200]


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2412_08076_amd import rm
    return rm.Context(0)


def _weights(batch, m, seed):
    rng = np.random.default_rng(seed)
    G = np.array([problem.gershgorin(oracle_coef(batch, b)) for b in range(batch.B)])
    om = (rng.uniform(0.5, 1.0, (batch.B, m)) / G[:, None]).astype(np.float32)
    al = rng.uniform(0.8, 0.97, (batch.B, m)).astype(np.float32)
    return dev(om, torch.float32), dev(al, torch.float32)


def _unroll(ctx, plan, method, om, al, f, m, K, hist=False, ckpt_every=0, jacobi=False):
    from paper_2412_08076_amd import rm
    x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
    h = torch.zeros(K // m * plan.B, dtype=torch.float64, device="cuda") if hist else None
    ck = torch.zeros(K // ckpt_every * 2 * plan.P, dtype=torch.float32, device="cuda") if ckpt_every else None
    opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=ckpt_every, jacobi=jacobi)
    rm.rm_solve(ctx, plan, method, opts, om, al, f, x, ckpt=ck, hist=h)
    return host(x), (host(h) if hist else None), (host(ck) if ckpt_every else None)


@pytest.mark.parametrize("method_name,jacobi", [("nag", False), ("richardson", False), ("mom", True),
                                                ("nagex", False), ("nagex", True)])
def test_blocked_equals_one_step_bitwise(ctx, method_name, jacobi):
    from paper_2412_08076_amd import rm
    method = {"nag": rm.RM_NAG, "richardson": rm.RM_RICHARDSON, "mom": rm.RM_MOM,
              "nagex": rm.RM_NAGEX}[method_name]
    batch = random_batch(NS, seed=5)
    plan = plan_for(ctx, batch)
    m, K = 16, 48
    om, al = _weights(batch, m, 1)
    if method_name == "nagex":
        al = torch.cat([al, 0.5 * al])
    f = dev(batch.f_packed(), torch.float32)
    plan.set_kernel(-1, 1)
    ref, ref_h, _ = _unroll(ctx, plan, method, om, al, f, m, K, hist=True, jacobi=jacobi)
    for shape in range(rm.STREAM_SHAPE + 1):
        for T in (1, 2, 3, 8, 16):
            for cw in (0, 24, 64, 128):
                try:
                    plan.set_kernel(shape, T, cw=cw)
                except rm.RMError:
                    continue  # halo T + 1 or width does not fit this variant
                say("blocked vs one-step", method_name, jacobi, "variant", shape, "T", T, "cw", cw)
                got, got_h, _ = _unroll(ctx, plan, method, om, al, f, m, K, hist=True, jacobi=jacobi)
                assert np.array_equal(got, ref), (shape, T, cw, np.max(np.abs(got - ref)))
                # the per-tile residual sums differ only in summation order
                assert np.allclose(got_h, ref_h, rtol=1e-12, atol=0), (shape, T, cw)


def test_blocked_checkpoints_and_mixed_classes(ctx):
    """Different (shape, T) per size class in one plan; checkpoints at a spacing that
    is not a multiple of T; the adjoint's recompute agrees with the forward."""
    from paper_2412_08076_amd import rm
    ns = [63, 63, 127, 255, 31]
    batch = random_batch(ns, seed=9)
    plan = plan_for(ctx, batch)
    m, K, E = 8, 24, 6
    om, al = _weights(batch, m, 2)
    f = dev(batch.f_packed(), torch.float32)
    plan.set_kernel(-1, 1)
    ref, _, ref_ck = _unroll(ctx, plan, rm.RM_NAG, om, al, f, m, K, ckpt_every=E)
    plan.set_kernel(0, 2, n=63)
    plan.set_kernel(2, 4, n=127)
    plan.set_kernel(4, 8, n=255)
    plan.set_kernel(3, 1, n=31)
    say("mixed classes", [plan.get_kernel(k) for k in (31, 63, 127, 255)])
    got, _, got_ck = _unroll(ctx, plan, rm.RM_NAG, om, al, f, m, K, ckpt_every=E)
    assert np.array_equal(got, ref)
    assert np.array_equal(got_ck, ref_ck)
    # row-streaming classes: whole height, and row windows with cuts
    plan.set_kernel(rm.STREAM_SHAPE, 5)
    plan.set_kernel(rm.STREAM_SHAPE, 3, n=127, cw=40)
    plan.set_kernel(rm.STREAM_SHAPE, 8, n=255, cw=100)
    say("stream classes", [plan.get_kernel(k) for k in (31, 63, 127, 255)])
    got, _, got_ck = _unroll(ctx, plan, rm.RM_NAG, om, al, f, m, K, ckpt_every=E)
    assert np.array_equal(got, ref)
    assert np.array_equal(got_ck, ref_ck)


def test_refined_solve_blocked_matches_one_step(ctx):
    from paper_2412_08076_amd import rm
    ns = [33, 64, 100]
    batch = random_batch(ns, seed=13, eps_range=(1e-2, 1.0))
    plan = plan_for(ctx, batch)
    m = 16
    om, al = _weights(batch, m, 3)
    b = dev(batch.f_packed())
    reps = []
    # the row-streaming shape with its tail (a tiled variant) never, always, or once
    # half of the instances have converged
    for cfg, frac in (((-1, 1), -1), ((2, 4), -1), ((4, 8), -1), ((9, 8), 0.0), ((9, 7), 1.0), ((9, 8), 0.5)):
        plan.set_kernel(*cfg)
        plan.set_tail_switch(frac)
        x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
        opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, tol_inner=1e-3, max_outer=20000, max_rounds=10)
        rep = rm.rm_solve(ctx, plan, rm.RM_NAG, opts, om, al, b, x)
        say("refined", cfg, frac, [plan.get_tail_kernel(k) for k in ns], rep["outer_iters"], rep["rounds"])
        assert rep["status"] == rm.RM_OK and np.all(rep["relres"] <= 1e-10)
        reps.append((rep, host(x)))
    for rep, x in reps[1:]:
        assert np.array_equal(rep["outer_iters"], reps[0][0]["outer_iters"])
        assert np.array_equal(x, reps[0][1])


def test_autotune_and_cache(ctx, tmp_path):
    from paper_2412_08076_amd import rm
    ns = [63, 255, 255]
    batch = random_batch(ns, seed=17)
    plan = plan_for(ctx, batch)
    m = 16
    om, al = _weights(batch, m, 4)
    f = dev(batch.f_packed(), torch.float32)
    cache = str(tmp_path / "tune.json")
    us = rm.rm_tune(ctx, plan, rm.RM_NAG, m, om, al, f, cache_path=cache)
    say("tuned", us, [plan.get_kernel(k) for k in (63, 255)])
    assert us > 0
    table = json.load(open(cache))
    # [shape, T, cw, us, tail shape, tail T, tail cw, tail us, one-active us]
    assert len(table) == 2 and all(len(v) == 9 for v in table.values())
    for k in (63, 255):
        assert plan.get_tail_kernel(k)[0] != rm.STREAM_SHAPE
    # a second plan reads the cache (no timing) and lands on the same choices
    plan2 = plan_for(ctx, batch)
    us2 = rm.rm_tune(ctx, plan2, rm.RM_NAG, m, om, al, f, cache_path=cache)
    assert abs(us2 - us) < 1e-2
    for k in (63, 255):
        assert plan2.get_kernel(k) == plan.get_kernel(k)
        assert plan2.get_tail_kernel(k) == plan.get_tail_kernel(k)
    # tuned plan still computes the same iterates as the one-step kernel
    ref_plan = plan_for(ctx, batch)
    ref_plan.set_kernel(-1, 1)
    a, _, _ = _unroll(ctx, plan, rm.RM_NAG, om, al, f, m, 32)
    r, _, _ = _unroll(ctx, ref_plan, rm.RM_NAG, om, al, f, m, 32)
    assert np.array_equal(a, r)


def test_adjoint_blocked_recompute_bitwise(ctx):
    """The adjoint whose forward recompute runs blocked launches that store every
    intermediate state (tiled and row-streaming) gives the same vectors as one launch
    per step, bit for bit; the gradients of omega and alpha are dot products summed over
    different tiles, so they agree to rounding order."""
    from paper_2412_08076_amd import rm
    ns = [40, 63, 127, 130]
    batch = random_batch(ns, seed=23)
    m, K, E = 8, 32, 16
    f = dev(batch.f_packed(), torch.float32)
    outs = []
    for cfg in ((-1, 1), (0, 4), (2, 8), (9, 8), (9, 5)):
        plan = plan_for(ctx, batch)
        om, al = _weights(batch, m, 6)
        plan.set_kernel(*cfg)
        say("adjoint recompute", cfg)
        x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
        ck = torch.empty(K // E * 2 * plan.P, dtype=torch.float32, device="cuda")
        opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=E)
        rm.rm_solve(ctx, plan, rm.RM_NAG, opts, om, al, f, x, ckpt=ck)
        dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
        da = torch.empty_like(dw)
        db = torch.empty(plan.P, dtype=torch.float32, device="cuda")
        loss = torch.empty(plan.B, dtype=torch.float32, device="cuda")
        rm.rm_solve_adjoint(ctx, plan, rm.RM_NAG, opts, om, al, f, ck, dw, da, d_b=db, loss=loss)
        outs.append([host(t) for t in (x, dw, da, db, loss)])
    for o in outs[1:]:
        for k, (a, b) in enumerate(zip(o, outs[0])):
            if k in (1, 2):  # d_omega, d_alpha
                np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-7 * np.max(np.abs(b)))
            else:
                assert np.array_equal(a, b), k


@pytest.mark.parametrize("method_name", ["nag", "nagex", "mom", "richardson"])
def test_blocked_reverse_matches_one_step_reverse(ctx, method_name):
    """Every Table-1 scheme, forward recompute through several kernel shapes and steps
    per launch, uneven sizes: d_b and the loss bit for bit equal to the one-step
    recompute and reverse, the weight gradients to rounding order.  With every class on
    the row-streaming shape the reverse steps run in its row pipeline as well."""
    from paper_2412_08076_amd import rm
    method = {"nag": rm.RM_NAG, "richardson": rm.RM_RICHARDSON, "mom": rm.RM_MOM, "nagex": rm.RM_NAGEX}[method_name]
    batch = random_batch([17, 40, 64, 65, 130], seed=27)
    # E = 8: the row-streaming reverse runs launches of 3, 3 and 2 reverse steps per segment
    m, K, E = 8, 24, 8
    f = dev(batch.f_packed(), torch.float32)
    ref = None
    for cfg in ((-1, 1), (0, 4), (3, 8), (6, 3), (2, 6), (5, 12), (1, 5), (4, 8), (9, 6), (9, 8)):
        plan = plan_for(ctx, batch)
        om, al = _weights(batch, m, 7)
        if method_name == "nagex":
            al = torch.cat([al, 0.5 * al])
        try:
            plan.set_kernel(*cfg)
        except rm.RMError:
            continue
        say("blocked reverse", method_name, cfg)
        x = torch.zeros(plan.P, dtype=torch.float32, device="cuda")
        ck = torch.empty(K // E * 2 * plan.P, dtype=torch.float32, device="cuda")
        opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=E)
        rm.rm_solve(ctx, plan, method, opts, om, al, f, x, ckpt=ck)
        na = 2 if method_name == "nagex" else 1
        dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
        da = torch.empty(na * plan.B * m, dtype=torch.float32, device="cuda")
        db = torch.empty(plan.P, dtype=torch.float32, device="cuda")
        loss = torch.empty(plan.B, dtype=torch.float32, device="cuda")
        rm.rm_solve_adjoint(ctx, plan, method, opts, om, al, f, ck, dw, da, d_b=db, loss=loss)
        out = [host(t) for t in (db, loss, dw, da)]
        if ref is None:
            ref = out
            continue
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), cfg
        for a, b in zip(out[2:], ref[2:]):
            np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-7 * max(1e-30, np.max(np.abs(b))))


@pytest.mark.parametrize("ns,m", [([63], 8), ([33, 64, 100, 255], 16), ([40, 41], 3)])
def test_refined_solve_graph_replays_match_eager(ctx, ns, m):
    """The refined solve replays one captured outer iteration per step, with its own
    eager refinement kernels and host polls between replays; every result must equal
    the run that launches the kernels one by one."""
    from paper_2412_08076_amd import rm
    batch = random_batch(ns, seed=29, eps_range=(1e-2, 1.0))
    om, al = _weights(batch, m, 9)
    b = dev(batch.f_packed())
    outs = []
    for graph in (False, True, True):  # eager reference, then two calls with graph replay
        plan = plan_for(ctx, batch)
        if max(ns) <= 512:
            # row-streaming main configuration, tiled tail from half the batch on:
            # two captured iterations, switched between at the polls
            plan.set_kernel(rm.STREAM_SHAPE, 8)
            plan.set_tail_switch(0.5)
        x = torch.zeros(plan.P, dtype=torch.float64, device="cuda")
        opts = rm.solve_opts(mode=rm.RM_TO_TOL, m=m, tol=1e-10, tol_inner=1e-3, max_outer=20000, max_rounds=10,
                             check_every=3, graph=graph)
        rep = rm.rm_solve(ctx, plan, rm.RM_NAG, opts, om, al, b, x)
        say("graph" if graph else "eager", ns, m, rep["outer_iters"], rep["rounds"])
        assert rep["status"] == rm.RM_OK
        outs.append((host(x), rep["outer_iters"], rep["rounds"], rep["relres"]))
    for o in outs[1:]:
        for a, e in zip(o, outs[0]):
            assert np.array_equal(a, e)


def test_tail_configuration_calls(ctx):
    """The tail follows rm_plan_set_kernel (a tiled variant under a row-streaming main
    configuration, the main configuration otherwise), can be set on its own, and bad
    arguments are rejected."""
    from paper_2412_08076_amd import rm
    batch = random_batch([63, 255], seed=31)
    plan = plan_for(ctx, batch)
    plan.set_kernel(rm.STREAM_SHAPE, 8)
    for k in (63, 255):
        assert plan.get_kernel(k)[0] == rm.STREAM_SHAPE
        assert plan.get_tail_kernel(k)[0] != rm.STREAM_SHAPE
    plan.set_tail_kernel(rm.STREAM_SHAPE, 4, n=255)
    assert plan.get_tail_kernel(255)[:2] == (rm.STREAM_SHAPE, 4)
    with pytest.raises(rm.RMError):
        plan.set_tail_switch(1.5)
    with pytest.raises(rm.RMError):
        plan.set_tail_kernel(rm.STREAM_SHAPE, 16)  # more steps per launch than are built
    with pytest.raises(rm.RMError):
        plan.set_tail_kernel(0, 8, n=77)  # no instance of that size
    with pytest.raises(rm.RMError):
        plan.set_kernel(rm.STREAM_SHAPE + 1, 8)
    plan.set_kernel(3, 8)
    assert plan.get_tail_kernel(255) == plan.get_kernel(255)


@pytest.mark.parametrize("method_name", ["nag", "nagex"])
def test_stream_wide_instances_bitwise(ctx, method_name):
    """Row-streaming forward and reverse at the widths where a workgroup holds 4, 5, 7
    and 8 waves (n = 256, 257, 448, 512, the largest it takes): the unroll with
    checkpoints and residual history, and the adjoint, equal one launch per step bit for
    bit (weight gradients to rounding order), over the whole height and over row windows."""
    from paper_2412_08076_amd import rm
    method = rm.RM_NAG if method_name == "nag" else rm.RM_NAGEX
    batch = random_batch([256, 257, 448, 512], seed=37)
    m, K, E = 8, 16, 8
    f = dev(batch.f_packed(), torch.float32)
    outs = []
    for cfg in ((-1, 1, 0), (rm.STREAM_SHAPE, 8, 0), (rm.STREAM_SHAPE, 5, 120)):
        plan = plan_for(ctx, batch)
        om, al = _weights(batch, m, 11)
        if method_name == "nagex":
            al = torch.cat([al, 0.5 * al])
        plan.set_kernel(cfg[0], cfg[1], cw=cfg[2])
        say("wide stream", method_name, cfg, [plan.get_kernel(k) for k in (256, 512)])
        x, h, ck = _unroll(ctx, plan, method, om, al, f, m, K, hist=True, ckpt_every=E)
        opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=E)
        na = 2 if method_name == "nagex" else 1
        dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
        da = torch.empty(na * plan.B * m, dtype=torch.float32, device="cuda")
        db = torch.empty(plan.P, dtype=torch.float32, device="cuda")
        loss = torch.empty(plan.B, dtype=torch.float32, device="cuda")
        rm.rm_solve_adjoint(ctx, plan, method, opts, om, al, f, dev(ck, torch.float32), dw, da, d_b=db, loss=loss)
        outs.append((x, h, ck, host(db), host(loss), host(dw), host(da)))
    ref = outs[0]
    for o in outs[1:]:
        assert np.array_equal(o[0], ref[0]) and np.array_equal(o[2], ref[2])
        assert np.allclose(o[1], ref[1], rtol=1e-12, atol=0)
        assert np.array_equal(o[3], ref[3]) and np.array_equal(o[4], ref[4])
        for a, b in zip(o[5:], ref[5:]):
            np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-7 * max(1e-30, np.max(np.abs(b))))


@pytest.mark.parametrize("method_name", ["nag", "richardson"])
def test_stream_widest_instances_bitwise(ctx, method_name):
    """Row-streaming forward on 1024-thread workgroups (n = 513 .. 1024: 9 to 16 waves
    holding whole rows): the unroll with checkpoints and residual history equals one
    launch per step bit for bit, over the whole height and over row windows, with
    several steps per launch; the adjoint (one reverse step per launch at these widths)
    agrees too."""
    from paper_2412_08076_amd import rm
    method = rm.RM_NAG if method_name == "nag" else rm.RM_RICHARDSON
    batch = random_batch([513, 700, 1023, 1024], seed=41)
    m, K, E = 8, 16, 8
    f = dev(batch.f_packed(), torch.float32)
    outs = []
    for cfg in ((-1, 1, 0), (rm.STREAM_SHAPE, 8, 0), (rm.STREAM_SHAPE, 7, 300), (rm.STREAM_SHAPE, 4, 130)):
        plan = plan_for(ctx, batch)
        om, al = _weights(batch, m, 13)
        plan.set_kernel(cfg[0], cfg[1], cw=cfg[2])
        say("widest stream", method_name, cfg, [plan.get_kernel(k) for k in (513, 1024)])
        x, h, ck = _unroll(ctx, plan, method, om, al, f, m, K, hist=True, ckpt_every=E)
        opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=E)
        dw = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
        da = torch.empty(plan.B * m, dtype=torch.float32, device="cuda")
        db = torch.empty(plan.P, dtype=torch.float32, device="cuda")
        loss = torch.empty(plan.B, dtype=torch.float32, device="cuda")
        rm.rm_solve_adjoint(ctx, plan, method, opts, om, al, f, dev(ck, torch.float32), dw, da, d_b=db, loss=loss)
        outs.append((x, h, ck, host(db), host(loss), host(dw), host(da)))
    ref = outs[0]
    for o in outs[1:]:
        assert np.array_equal(o[0], ref[0]) and np.array_equal(o[2], ref[2])
        assert np.allclose(o[1], ref[1], rtol=1e-12, atol=0)
        assert np.array_equal(o[3], ref[3]) and np.array_equal(o[4], ref[4])
        for a, b in zip(o[5:], ref[5:]):
            np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-7 * max(1e-30, np.max(np.abs(b))))
