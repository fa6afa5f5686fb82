"""Shared set-up for the GPU parity tests: build a plan from a synthetic batch and
move packed vectors between numpy and the device."""
import sys

import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_08076_amd import _lib
    _lib.load()  # raises when librm.so is missing: the HIP path must be the one that runs


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda().contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def plan_for(ctx, batch):
    from paper_2412_08076_amd import rm
    if batch.op == "helmholtz":
        return rm.Plan(ctx, batch.n, kappa=batch.kappa, op=rm.RM_FD5_HELMHOLTZ)
    return rm.Plan(ctx, batch.n, eps=batch.eps, theta=batch.theta)


def oracle_coef(batch, b):
    from oracle import problem
    if batch.op == "helmholtz":
        return problem.helmholtz_stencil(batch.kappa[b], batch.n[b])
    return problem.q1_stencil(batch.eps[b], batch.theta[b])


# Element-wise bar of the FP32 sweeps: after K inner steps from the same inputs,
#   max |x_gpu - u_oracle| <= FP32_C * eps32 * K * max |u_oracle|.
# A float32 CPU emulation of the same recurrences (every parity case: NAG with
# momentum up to 0.99, meta-network weights, n up to 1023) stays at or below 0.41 of
# eps32 * K * max |u|; FP32_C = 2 leaves a factor of about five for the GPU's fused
# multiply-adds and summation order.  A dropped stencil term or a wrong weight index
# moves the iterate by O(1e-2) of its size, far above 2 eps32 K (about 7.6e-6 at K = 32).
FP32_C = 2.0


def assert_fp32_close(got, want, K, what=""):
    e32 = float(np.finfo(np.float32).eps)
    bound = FP32_C * e32 * K * float(np.max(np.abs(want)))
    err = float(np.max(np.abs(got - want)))
    assert err <= bound, (what, err, bound)
