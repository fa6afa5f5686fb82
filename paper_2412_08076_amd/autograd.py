"""torch.autograd glue for training the weight network (§2.2, Algorithm 1) and the
coarse symbol of the multilevel variant (§3).

MetaWeights   params -> (omega, alpha) through rm_meta_forward / rm_meta_backward.
UnrollLoss    (omega, alpha, b) -> per-instance ||b - A u_K||^2 / ||b||^2 after a K-step
              unroll from u_0 = 0 (rm_solve RM_UNROLL with checkpoints); the backward
              pass runs rm_solve_adjoint.  `precond` selects None, "jacobi" or
              ("ssor", relaxation factor).
TwoGridLoss   (omega, alpha, symbol, b) -> the same loss after K two-grid cycles from 0
              (rm_twogrid_solve); the backward pass runs rm_twogrid_adjoint and also
              returns the gradient of the symbol.
SymbolNet     params -> the coarse symbol of every instance through rm_symbolnet_forward /
              rm_symbolnet_backward; composed with TwoGridLoss it carries the loss's
              gradient to the symbol network's parameters.
All passes run in the HIP kernels; these classes only allocate outputs and pass
pointers.  For RM_NAGEX, alpha has shape [2][B][m] (momentum, look-ahead).
"""
import torch

from . import rm


class MetaWeights(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, solver_ctx, plan, m):
        omega = torch.empty(plan.B, m, dtype=torch.float32, device=params.device)
        alpha = torch.empty_like(omega)
        rm.rm_meta_forward(solver_ctx, plan, m, params.detach(), omega, alpha)
        ctx.save_for_backward(params)
        ctx.meta = (solver_ctx, plan, m)
        return omega, alpha

    @staticmethod
    def backward(ctx, d_omega, d_alpha):
        (params,) = ctx.saved_tensors
        solver_ctx, plan, m = ctx.meta
        d_omega = torch.zeros_like(params.new_empty(plan.B, m)) if d_omega is None else d_omega.contiguous()
        d_alpha = torch.zeros_like(params.new_empty(plan.B, m)) if d_alpha is None else d_alpha.contiguous()
        d_params = torch.empty_like(params)
        rm.rm_meta_backward(solver_ctx, plan, m, params.detach(), d_omega, d_alpha, d_params)
        return d_params, None, None, None


def _precond_kw(precond):
    if precond is None:
        return {}
    if precond == "jacobi":
        return {"jacobi": True}
    if isinstance(precond, tuple) and precond[0] == "ssor":
        return {"ssor": float(precond[1])}
    raise ValueError(f"unknown preconditioner {precond!r}")


class UnrollLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, omega, alpha, b, solver_ctx, plan, method, m, K, ckpt_every, precond=None):
        opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, ckpt_every=ckpt_every,
                             **_precond_kw(precond))
        x = torch.zeros(plan.P, dtype=torch.float32, device=b.device)
        ckpt = torch.empty((K // ckpt_every) * 2 * plan.P, dtype=torch.float32, device=b.device)
        om = omega.detach().contiguous()
        al = alpha.detach().contiguous()
        rm.rm_solve(solver_ctx, plan, method, opts, om, al, b.detach(), x, ckpt=ckpt)
        loss = torch.empty(plan.B, dtype=torch.float32, device=b.device)
        rm.rm_residual(solver_ctx, plan, b.detach(), x, rel2=loss)
        ctx.save_for_backward(om, al, b, ckpt)
        ctx.meta = (solver_ctx, plan, method, opts)
        return loss

    @staticmethod
    def backward(ctx, g_loss):
        om, al, b, ckpt = ctx.saved_tensors
        solver_ctx, plan, method, opts = ctx.meta
        d_omega = torch.empty_like(om)
        d_alpha = torch.empty_like(al)
        d_b = torch.empty_like(b) if ctx.needs_input_grad[2] else None
        rm.rm_solve_adjoint(solver_ctx, plan, method, opts, om, al, b.detach(), ckpt, d_omega, d_alpha,
                            g_loss=g_loss.contiguous().float(), d_b=d_b)
        return d_omega, d_alpha, d_b, None, None, None, None, None, None, None


class TwoGridLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, omega, alpha, symbol, b, solver_ctx, plan, method, m, K, precond=None):
        opts = rm.solve_opts(mode=rm.RM_UNROLL, dtype=rm.RM_F32, m=m, K=K, **_precond_kw(precond))
        x = torch.zeros(plan.P, dtype=torch.float32, device=b.device)
        ckpt = torch.empty(K * plan.P, dtype=torch.float32, device=b.device)
        om = omega.detach().contiguous()
        al = alpha.detach().contiguous()
        sy = symbol.detach().contiguous()
        rm.rm_twogrid_solve(solver_ctx, plan, method, opts, om, al, sy, b.detach(), x, ckpt=ckpt)
        loss = torch.empty(plan.B, dtype=torch.float32, device=b.device)
        rm.rm_residual(solver_ctx, plan, b.detach(), x, rel2=loss)
        ctx.save_for_backward(om, al, sy, b, ckpt)
        ctx.meta = (solver_ctx, plan, method, opts)
        return loss

    @staticmethod
    def backward(ctx, g_loss):
        om, al, sy, b, ckpt = ctx.saved_tensors
        solver_ctx, plan, method, opts = ctx.meta
        d_omega = torch.empty_like(om)
        d_alpha = torch.empty_like(al)
        d_symbol = torch.empty_like(sy)
        d_b = torch.empty_like(b) if ctx.needs_input_grad[3] else None
        rm.rm_twogrid_adjoint(solver_ctx, plan, method, opts, om, al, sy, b.detach(), ckpt, d_omega, d_alpha,
                              d_symbol, g_loss=g_loss.contiguous().float(), d_b=d_b)
        return d_omega, d_alpha, d_symbol, d_b, None, None, None, None, None, None


class SymbolNet(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, solver_ctx, plan):
        symbol = torch.empty(plan.coarse_points(), dtype=torch.float32, device=params.device)
        rm.rm_symbolnet_forward(solver_ctx, plan, params.detach(), symbol)
        ctx.save_for_backward(params)
        ctx.meta = (solver_ctx, plan)
        return symbol

    @staticmethod
    def backward(ctx, d_symbol):
        (params,) = ctx.saved_tensors
        solver_ctx, plan = ctx.meta
        d_params = torch.empty_like(params)
        rm.rm_symbolnet_backward(solver_ctx, plan, params.detach(), d_symbol.contiguous(), d_params)
        return d_params, None, None
