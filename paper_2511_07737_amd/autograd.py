"""torch.autograd.Function over the gfx950 forward and adjoint kernels.

The layer is the paper's binarized matrix product followed by SmoothMin
(Sec. III-B, Eq. 1 and Eq. 4): given the binary assignment A of the positive
literals (a [V][N] float tensor of 0/1 values on the GPU; the negated
literals are the complements, Sec. III-A), forward returns
S_i = SmoothMin_c(R_ci) for every candidate, and backward maps dLoss/dS to
dLoss/dA through the transpose product with the straight-through sign (+1 for
x_v, -1 for not-x_v).  All arithmetic runs in the HIP library; torch provides
the device memory and the stream (``torch.cuda.current_stream()``).

``binarize_ste`` and ``normalize_rows`` build the paper's full differentiable
graph (Fig. 3): theta -> theta / mean_row(theta) (Eq. 5) -> B with the
straight-through estimator (Eq. 2) -> SmoothMin layer -> loss (Eq. 3).
"""
from __future__ import annotations

import torch

from . import tsat


class SmoothMinSat(torch.autograd.Function):
    @staticmethod
    def forward(ctx, assign: torch.Tensor, solver: tsat.Solver, tau: float):
        if not assign.is_cuda or assign.dtype != torch.float32 or assign.dim() != 2:
            raise ValueError("assign must be a 2-D float32 CUDA tensor [V][N]")
        assign = assign.contiguous()
        V, N = assign.shape
        if V != solver.V:
            raise ValueError(f"assign has {V} rows, the loaded CNF has {solver.V} variables")
        W = (N + 63) // 64
        stream = torch.cuda.current_stream(assign.device).cuda_stream
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
        dS = dS.contiguous().to(torch.float32)
        U = torch.empty((V, N), dtype=torch.float32, device=bits.device)
        stream = torch.cuda.current_stream(bits.device).cuda_stream
        ctx.solver.bwd_dev(bits.data_ptr(), N, ctx.tau, dS.data_ptr(), U.data_ptr(), stream)
        return U, None, None


def smoothmin_sat(assign: torch.Tensor, solver: tsat.Solver, tau: float = 1.0) -> torch.Tensor:
    """S[N] of the binary assignment ``assign`` [V][N] (differentiable via the STE adjoint)."""
    return SmoothMinSat.apply(assign, solver, float(tau))


class _BinarizeSTE(torch.autograd.Function):
    """B(x) = clip(sign(x), 0, 1) forward, identity backward (Eq. 2 with the STE)."""

    @staticmethod
    def forward(ctx, x):
        return (x > 0).to(x.dtype)

    @staticmethod
    def backward(ctx, g):
        return g


def binarize_ste(x: torch.Tensor) -> torch.Tensor:
    return _BinarizeSTE.apply(x)


def normalize_rows(theta: torch.Tensor, eps: float = 1e-12) -> torch.Tensor:
    """Eq. 5: theta / mean over candidates of each variable row; |mean| < eps is
    clamped to +-eps (0 -> +eps) and treated as a constant there."""
    mu = theta.mean(dim=1, keepdim=True)
    small = mu.abs() < eps
    safe = torch.where(small, torch.where(mu >= 0, torch.full_like(mu, eps), torch.full_like(mu, -eps)), mu)
    mu_used = torch.where(small, safe.detach(), mu)
    return theta / mu_used


def loss_of(theta: torch.Tensor, solver: tsat.Solver, tau: float = 1.0, normalize: bool = True) -> torch.Tensor:
    """L = -sum_i S_i (Eq. 3) of the logits theta [V][N]."""
    x = normalize_rows(theta) if normalize else theta
    return -smoothmin_sat(binarize_ste(x), solver, tau).sum()
