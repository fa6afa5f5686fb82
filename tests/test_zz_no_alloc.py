"""rm_residual_noalloc (the entry point for callers that cannot allocate) against
rm_residual, called through the C ABI: the same kernels over the same tiles, so r,
||r||^2, ||b||^2 and their ratio must agree bit for bit.  Two calls in a row, the
second on a smaller plan, so that the shared static scratch is reused with different
contents; then a plan over the scratch's tile limit is rejected before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from synthetic import random_batch
from tests.gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _plan(lib, h, ns, seed):
    from paper_2412_08076_amd import _lib
    batch = random_batch(ns, seed=seed)
    inst = (_lib.rm_instance * len(ns))()
    for b, n in enumerate(ns):
        inst[b].n, inst[b].op, inst[b].eps, inst[b].theta, inst[b].kappa = n, 0, batch.eps[b], batch.theta[b], 0.0
    p = ctypes.c_void_p()
    assert lib.rm_plan(h, len(ns), inst, None, ctypes.byref(p)) == 0, lib.rm_last_error()
    return p, batch


@pytest.mark.parametrize("dtype", [0, 1])
def test_residual_noalloc_matches_residual(dtype):
    need_gpu()
    from paper_2412_08076_amd import _lib
    lib = _lib.load()
    tdt = torch.float32 if dtype == 0 else torch.float64
    h = ctypes.c_void_p()
    assert lib.rm_create(ctypes.byref(h), 0, None) == 0
    try:
        # first a larger batch (several tiles per instance, ragged edges), then a smaller one
        for ns, seed in (([200, 65, 7, 130, 1], 31), ([33, 3], 32)):
            say("noalloc residual", dtype, ns)
            p, batch = _plan(lib, h, ns, seed)
            try:
                P = int(lib.rm_plan_points(p))
                g = torch.Generator().manual_seed(seed)
                bv = torch.randn(P, generator=g, dtype=torch.float64).to(tdt).cuda()
                xv = torch.randn(P, generator=g, dtype=torch.float64).to(tdt).cuda()
                B = len(ns)
                outs = []
                for fn in (lib.rm_residual, lib.rm_residual_noalloc):
                    r = torch.full((P,), float("nan"), dtype=tdt, device="cuda")
                    r2 = torch.full((B,), -1.0, dtype=torch.float64, device="cuda")
                    b2 = torch.full((B,), -1.0, dtype=torch.float64, device="cuda")
                    rel = torch.full((B,), -1.0, dtype=torch.float32, device="cuda")
                    st = fn(h, p, dtype, _ptr(bv), _ptr(xv), _ptr(r), _ptr(r2), _ptr(b2), _ptr(rel))
                    assert st == 0, lib.rm_last_error()
                    torch.cuda.synchronize()
                    outs.append([t.cpu().numpy() for t in (r, r2, b2, rel)])
                for a, c in zip(outs[0], outs[1]):
                    assert np.array_equal(a, c)
                assert np.all(outs[1][1] > 0) and np.all(np.isfinite(outs[1][0]))
                # without r the norms are still formed
                r2n = torch.full((B,), -1.0, dtype=torch.float64, device="cuda")
                assert lib.rm_residual_noalloc(h, p, dtype, _ptr(bv), _ptr(xv), None, _ptr(r2n), None, None) == 0
                torch.cuda.synchronize()
                assert np.array_equal(r2n.cpu().numpy(), outs[0][1])
            finally:
                lib.rm_plan_free(p)
    finally:
        lib.rm_destroy(h)


def test_residual_noalloc_rejects_plans_over_the_limit():
    need_gpu()
    from paper_2412_08076_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.rm_create(ctypes.byref(h), 0, None) == 0
    try:
        # 65537 instances of n = 1: one tile each, one more than the scratch holds
        ns = [1] * 65537
        inst = (_lib.rm_instance * len(ns))()
        for b in range(len(ns)):
            inst[b].n, inst[b].op, inst[b].eps, inst[b].theta, inst[b].kappa = 1, 0, 1.0, 0.0, 0.0
        p = ctypes.c_void_p()
        assert lib.rm_plan(h, len(ns), inst, None, ctypes.byref(p)) == 0
        try:
            v = torch.zeros(len(ns), dtype=torch.float32, device="cuda")
            st = lib.rm_residual_noalloc(h, p, 0, _ptr(v), _ptr(v), None, None, None, None)
            assert st == _lib.RM_EINVAL
            assert b"tiles" in lib.rm_last_error()
        finally:
            lib.rm_plan_free(p)
    finally:
        lib.rm_destroy(h)
