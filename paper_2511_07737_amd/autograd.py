"""torch.autograd.Functions over the gfx950 kernels of the differentiable path.

The paper's graph (Sec. III-B, Fig. 3): logits theta [V][N] -> per-variable
normalization (Eq. 5) -> binarization B (Eq. 2, straight-through estimator
backward) -> R = P A (Eq. 1) -> SmoothMin per candidate (Eq. 4) -> loss
(Eq. 3).  Every step, forward and backward, runs in the HIP library through
its device-pointer entry points; this module only allocates the tensors,
passes their pointers and torch's current stream, and wires the backward.

* ``smoothmin_sat(assign)``: binary assignment A [V][N] (0/1 floats) -> S [N];
  backward dS -> dA through the transpose product (+1 for x_v, -1 for not x_v).
* ``binarize(theta, mode)``: Eq. 5 then Eq. 2 -> A (0/1 floats); backward is
  the Eq. 5 backward of the gradient the STE passes through Eq. 2.
* ``loss_of(theta)``: the whole chain to the scalar loss in one call, its
  backward in one fused pass (adjoint, Eq. 5 backward).
"""
from __future__ import annotations

import torch

from . import tsat


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _logits(theta: torch.Tensor, solver: tsat.Solver) -> torch.Tensor:
    if not theta.is_cuda or theta.dtype != torch.float32 or theta.dim() != 2:
        raise ValueError("logits must be a 2-D float32 CUDA tensor [V][N]")
    if theta.shape[0] != solver.V:
        raise ValueError(f"logits have {theta.shape[0]} rows, the loaded CNF has {solver.V} variables")
    return theta.contiguous()


def _upstream(t: torch.Tensor) -> torch.Tensor:
    if t.dtype != torch.float32:
        raise ValueError(f"upstream gradient must be float32 (got {t.dtype})")
    return t.contiguous()


class SmoothMinSat(torch.autograd.Function):
    @staticmethod
    def forward(ctx, assign: torch.Tensor, solver: tsat.Solver, tau: float):
        assign = _logits(assign, solver)
        V, N = assign.shape
        W = (N + 63) // 64
        stream = _stream(assign)
        bits = torch.empty((V, W), dtype=torch.int64, device=assign.device)
        solver.pack_dev(assign.data_ptr(), N, bits.data_ptr(), stream)
        S = torch.empty(N, dtype=torch.float32, device=assign.device)
        solver.fwd_dev(bits.data_ptr(), N, tau, S.data_ptr(), None, stream)
        ctx.save_for_backward(bits)
        ctx.solver = solver
        ctx.tau = tau
        ctx.shape = (V, N)
        return S

    @staticmethod
    def backward(ctx, dS: torch.Tensor):
        (bits,) = ctx.saved_tensors
        V, N = ctx.shape
        dS = _upstream(dS)
        U = torch.empty((V, N), dtype=torch.float32, device=bits.device)
        ctx.solver.bwd_dev(bits.data_ptr(), N, ctx.tau, dS.data_ptr(), U.data_ptr(), _stream(bits))
        return U, None, None


def smoothmin_sat(assign: torch.Tensor, solver: tsat.Solver, tau: float = 1.0) -> torch.Tensor:
    """S[N] of the binary assignment ``assign`` [V][N] (differentiable via the STE adjoint)."""
    return SmoothMinSat.apply(assign, solver, float(tau))


class Binarize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, solver: tsat.Solver, mode: int):
        theta = _logits(theta, solver)
        assign = torch.empty_like(theta)
        solver.binarize_dev(theta.data_ptr(), theta.shape[1], mode, None, assign.data_ptr(), None, _stream(theta))
        ctx.save_for_backward(theta)
        ctx.solver = solver
        ctx.mode = mode
        return assign

    @staticmethod
    def backward(ctx, dA: torch.Tensor):
        (theta,) = ctx.saved_tensors
        dA = _upstream(dA)
        g = torch.empty_like(theta)
        ctx.solver.norm_backward_dev(theta.data_ptr(), dA.data_ptr(), theta.shape[1], ctx.mode, g.data_ptr(),
                                     _stream(theta))
        return g, None, None


def binarize(theta: torch.Tensor, solver: tsat.Solver, mode: int = tsat.MODE_MEAN) -> torch.Tensor:
    """A = B(theta / mean_row(theta)) (Eq. 5, Eq. 2; mode ``tsat.MODE_NONE``: B(theta))
    as 0/1 floats, with the straight-through estimator and the Eq. 5 backward."""
    return Binarize.apply(theta, solver, int(mode))


class LogitLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, solver: tsat.Solver, tau: float, mode: int):
        theta = _logits(theta, solver)
        loss = torch.empty((), dtype=torch.float32, device=theta.device)
        solver.loss_dev(theta.data_ptr(), theta.shape[1], tau, mode, loss.data_ptr(), None, None, _stream(theta))
        ctx.save_for_backward(theta)
        ctx.solver = solver
        ctx.tau = tau
        ctx.mode = mode
        return loss

    @staticmethod
    def backward(ctx, dloss: torch.Tensor):
        (theta,) = ctx.saved_tensors
        dloss = _upstream(dloss)
        g = torch.empty_like(theta)
        ctx.solver.loss_backward_dev(theta.data_ptr(), theta.shape[1], ctx.tau, ctx.mode, dloss.data_ptr(),
                                     g.data_ptr(), None, _stream(theta))
        return g, None, None, None


def loss_of(theta: torch.Tensor, solver: tsat.Solver, tau: float = 1.0, normalize: bool = True) -> torch.Tensor:
    """L = -sum_i S_i (Eq. 3) of the logits theta [V][N], as a 0-d tensor."""
    return LogitLoss.apply(theta, solver, float(tau), tsat.MODE_MEAN if normalize else tsat.MODE_NONE)
