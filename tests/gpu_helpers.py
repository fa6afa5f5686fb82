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
