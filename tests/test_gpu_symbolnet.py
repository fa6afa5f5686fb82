"""Symbol network of the two-grid Helmholtz cycle on the GPU against the oracle: the
symbol of every instance, the parameter gradient of a weighted sum of symbols, the
chain through TwoGridLoss, determinism, and the full-size batch (32 instances, n = 511)
on sampled instances."""
import numpy as np
import pytest
import torch

from oracle import symbolnet, twogrid
from synthetic import Batch, symbolnet_params, unpack_vec
from tests.gpu_helpers import dev, host, need_gpu, oracle_coef, plan_for, say

pytestmark = pytest.mark.gpu

# n + 1 a power of two: coarse grids of 3 .. 127 modes, one to 64 tiles of 16 x 16, the
# larger ones with a ragged last row and column of tiles
NS = [7, 15, 31, 63, 127, 255]


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2412_08076_amd import rm
    return rm.Context(0)


def _batch(ns, seed, kappa_range=(2.0, 12.0)):
    rng = np.random.default_rng(seed)
    # kappa rounded to FP32: the device holds it in FP32, the oracle takes the same value
    kappa = rng.uniform(*kappa_range, size=len(ns)).astype(np.float32).astype(np.float64)
    f = [rng.standard_normal((k, k)) for k in ns]
    return Batch(ns, kappa=kappa, f=f, op="helmholtz")


def _params(seed, last_std=0.3):
    th = symbolnet_params(seed, last_std=last_std).astype(np.float32)
    return th.astype(np.float64), dev(th, torch.float32)


def _coarse(plan, flat, ns):
    coff = plan.coarse_offsets()
    out = []
    for b, n in enumerate(ns):
        nc = (n - 1) // 2
        out.append(flat[coff[b]:coff[b] + nc * nc].reshape(nc, nc))
    return out


def _pack_coarse(plan, per_inst):
    coff = plan.coarse_offsets()
    flat = np.zeros(plan.coarse_points())
    for b, s in enumerate(per_inst):
        flat[coff[b]:coff[b] + s.size] = s.ravel()
    return flat


# FP32 bars.  The symbol is base * exp(z) with the base formed in FP64 on both sides, so
# its relative error is the absolute error of z: three layers of at most 145 products each,
# tanh bounded by 1, the weights O(1/sqrt(fan-in)): a few hundred eps32 at most, 1e-5 here.
# The gradient sums up to 127^2 points per tile and over the tiles in FP64: 1e-4 of its
# largest entry.  A transposed kernel offset or a dropped tanh derivative moves the
# result by O(1e-1) of its size.
SYM_RTOL = 1e-5
GRAD_RTOL = 1e-4


def test_symbolnet_forward_matches_oracle(ctx):
    from paper_2412_08076_amd import rm
    batch = _batch(NS, seed=5)
    plan = plan_for(ctx, batch)
    th, thd = _params(11)
    say("symbol network forward", NS, "params", thd.numel())
    assert thd.numel() == rm.rm_symbolnet_param_count() == symbolnet.param_count()
    sym = torch.full((plan.coarse_points(),), float("nan"), dtype=torch.float32, device="cuda")
    rm.rm_symbolnet_forward(ctx, plan, thd, sym)
    got = _coarse(plan, host(sym), NS)
    for b, n in enumerate(NS):
        want = symbolnet.forward(th, batch.kappa[b], n)
        err = np.max(np.abs(got[b] - want) / np.abs(want))
        say("  n", n, "kappa", batch.kappa[b], "max rel err %.2e" % err)
        assert np.all(np.isfinite(got[b]))
        assert err <= SYM_RTOL


def test_symbolnet_backward_matches_oracle(ctx):
    from paper_2412_08076_amd import rm
    batch = _batch(NS, seed=6)
    plan = plan_for(ctx, batch)
    th, thd = _params(12)
    rng = np.random.default_rng(13)
    dsyms = [rng.standard_normal(((n - 1) // 2,) * 2).astype(np.float32).astype(np.float64) for n in NS]
    dsd = dev(_pack_coarse(plan, dsyms), torch.float32)
    say("symbol network backward", NS)
    d = torch.full((thd.numel(),), float("nan"), dtype=torch.float32, device="cuda")
    rm.rm_symbolnet_backward(ctx, plan, thd, dsd, d)
    got = host(d)
    want = sum(symbolnet.backward(th, batch.kappa[b], n, dsyms[b]) for b, n in enumerate(NS))
    # per parameter block, so that a wrong small block (b3, the first layer) is seen
    bounds = np.cumsum([0] + [int(np.prod(s)) for s in symbolnet.SHAPES])
    for k in range(len(symbolnet.SHAPES)):
        g, w = got[bounds[k]:bounds[k + 1]], want[bounds[k]:bounds[k + 1]]
        err = np.max(np.abs(g - w)) / np.max(np.abs(w))
        say("  block", k, "size", w.size, "rel err %.2e" % err)
        assert err <= GRAD_RTOL
    # the same call again gives the same bits (partials reduced in tile order)
    d2 = torch.empty_like(d)
    rm.rm_symbolnet_backward(ctx, plan, thd, dsd, d2)
    assert torch.equal(d, d2)


def test_symbolnet_through_twogrid_loss(ctx):
    """SymbolNet composed with TwoGridLoss: the parameter gradient of a weighted sum of
    per-instance losses equals the oracle's chain, symbolnet.backward of the two-grid
    loss's symbol gradient."""
    from paper_2412_08076_amd import rm
    from paper_2412_08076_amd.autograd import SymbolNet, TwoGridLoss
    from oracle import problem
    ns = [15, 31, 63]
    batch = _batch(ns, seed=7)
    plan = plan_for(ctx, batch)
    m, K = 3, 2
    rng = np.random.default_rng(17)
    om = np.zeros((batch.B, m))
    for b in range(batch.B):
        om[b] = rng.uniform(0.3, 0.9, m) / problem.gershgorin(oracle_coef(batch, b))
    om = om.astype(np.float32).astype(np.float64)
    al = rng.uniform(0.1, 0.5, (batch.B, m)).astype(np.float32).astype(np.float64)
    th, thd = _params(14, last_std=0.2)
    params = thd.clone().requires_grad_(True)
    f32 = batch.f_packed().astype(np.float32)
    wts = torch.tensor([0.5, 1.0, 2.0], dtype=torch.float32, device="cuda")
    say("symbol network through the two-grid loss", ns)
    symbol = SymbolNet.apply(params, ctx, plan)
    loss = TwoGridLoss.apply(dev(om, torch.float32), dev(al, torch.float32), symbol, dev(f32, torch.float32),
                             ctx, plan, rm.RM_NAG, m, K)
    (loss * wts).sum().backward()
    fs = unpack_vec(f32.astype(np.float64), ns)
    syms = _coarse(plan, host(symbol), ns)
    want = np.zeros_like(th)
    for b, n in enumerate(ns):
        # the oracle's symbol of these parameters (FP64) drives the oracle's cycle
        so = symbolnet.forward(th, batch.kappa[b], n)
        assert np.max(np.abs(syms[b] - so) / np.abs(so)) <= SYM_RTOL
        L, gw, ga, gat, gs, gf = twogrid.loss_and_grads("nag", oracle_coef(batch, b), fs[b], om[b], so, K,
                                                        alpha=al[b])
        assert abs(host(loss)[b] - L) <= 1e-5 * L
        want += float(wts[b]) * symbolnet.backward(th, batch.kappa[b], n, gs)
    got = host(params.grad)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    say("  params grad rel err %.2e" % err)
    assert err <= GRAD_RTOL


def test_symbolnet_full_size_sampled(ctx):
    """32 instances of n = 511 (nc = 255, 256 tiles each): the symbol of sampled
    instances, and the gradient of d_symbol supported on those instances only, which is
    the sum of their oracle gradients (the gradient is linear in d_symbol)."""
    from paper_2412_08076_amd import rm
    B, n = 32, 511
    batch = _batch([n] * B, seed=8)
    plan = plan_for(ctx, batch)
    th, thd = _params(15)
    sym = torch.empty(plan.coarse_points(), dtype=torch.float32, device="cuda")
    say("symbol network full size", B, "x", n)
    rm.rm_symbolnet_forward(ctx, plan, thd, sym)
    got = _coarse(plan, host(sym), batch.n)
    picks = [0, 13, 31]
    for b in picks:
        want = symbolnet.forward(th, batch.kappa[b], n)
        err = np.max(np.abs(got[b] - want) / np.abs(want))
        say("  instance", b, "max rel err %.2e" % err)
        assert err <= SYM_RTOL
    assert all(np.all(np.isfinite(s)) for s in got)
    rng = np.random.default_rng(16)
    nc = (n - 1) // 2
    dsyms = [np.zeros((nc, nc)) for _ in range(B)]
    for b in picks[:2]:
        dsyms[b] = rng.standard_normal((nc, nc)).astype(np.float32).astype(np.float64)
    d = torch.empty(thd.numel(), dtype=torch.float32, device="cuda")
    rm.rm_symbolnet_backward(ctx, plan, thd, dev(_pack_coarse(plan, dsyms), torch.float32), d)
    want = sum(symbolnet.backward(th, batch.kappa[b], n, dsyms[b]) for b in picks[:2])
    err = np.max(np.abs(host(d) - want)) / np.max(np.abs(want))
    say("  gradient rel err %.2e" % err)
    assert err <= GRAD_RTOL


def test_symbolnet_largest_size(ctx):
    """n = 1023 (the largest two-grid size: 511 x 511 modes, 32 x 32 tiles) beside n = 7:
    the symbol of both and the gradient against the oracle."""
    from paper_2412_08076_amd import rm
    ns = [1023, 7]
    batch = _batch(ns, seed=9, kappa_range=(20.0, 80.0))
    plan = plan_for(ctx, batch)
    th, thd = _params(19)
    say("symbol network largest size", ns)
    sym = torch.empty(plan.coarse_points(), dtype=torch.float32, device="cuda")
    rm.rm_symbolnet_forward(ctx, plan, thd, sym)
    got = _coarse(plan, host(sym), ns)
    for b, n in enumerate(ns):
        want = symbolnet.forward(th, batch.kappa[b], n)
        err = np.max(np.abs(got[b] - want) / np.abs(want))
        say("  n", n, "max rel err %.2e" % err)
        assert err <= SYM_RTOL
    rng = np.random.default_rng(21)
    dsyms = [rng.standard_normal(((n - 1) // 2,) * 2).astype(np.float32).astype(np.float64) for n in ns]
    d = torch.empty(thd.numel(), dtype=torch.float32, device="cuda")
    rm.rm_symbolnet_backward(ctx, plan, thd, dev(_pack_coarse(plan, dsyms), torch.float32), d)
    want = sum(symbolnet.backward(th, batch.kappa[b], n, dsyms[b]) for b, n in enumerate(ns))
    err = np.max(np.abs(host(d) - want)) / np.max(np.abs(want))
    say("  gradient rel err %.2e" % err)
    assert err <= GRAD_RTOL


def test_symbolnet_rejects_bad_plans(ctx):
    """Called through the C-ABI: a plan of Q1 instances and a plan whose n + 1 is not a
    power of two are refused with an error status, and nothing is written."""
    import ctypes
    from paper_2412_08076_amd import rm
    thd = torch.zeros(rm.rm_symbolnet_param_count(), dtype=torch.float32, device="cuda")
    out = torch.full((256,), 7.0, dtype=torch.float32, device="cuda")
    q1 = Batch([15, 31], eps=[1.0, 0.1], theta=[0.0, 0.5], f=[np.zeros((15, 15)), np.zeros((31, 31))])
    for batch in (q1, _batch([12], seed=1)):
        plan = plan_for(ctx, batch)
        st = ctx.lib.rm_symbolnet_forward(ctx.handle, plan.handle, ctypes.c_void_p(thd.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()))
        say("  rejected", batch.op, batch.n, "status", st)
        assert st != rm.RM_OK
    assert torch.all(out == 7.0)
