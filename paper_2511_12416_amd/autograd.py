"""Differentiable log-probabilities (torch.autograd.Function wrappers).

``log_prob`` maps (rotation layers, CPhase angles) to log p_b with its
backward computed by the library's adjoint kernel; ``spin_rotations`` maps
anti-Hermitian generators K_l to layers exp(K_l) (+) exp(K_l), forward and
backward computed by the library (xf_spin_rotations,
xf_spin_rotations_adjoint).  Complex gradients follow PyTorch's convention
dL/dRe + i dL/dIm.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


class _LogProb(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rot, theta, plan, bits, mode, t, seed):
        plan.set_params(rot.detach().cpu().numpy(), theta.detach().cpu().numpy())
        B = bits.shape[0]
        p = torch.empty(B, dtype=torch.float64, device=plan.device)
        logp = torch.empty(B, dtype=torch.float64, device=plan.device)
        plan.probabilities(bits, mode, t, seed, out=p, logp=logp)
        ctx.plan, ctx.bits, ctx.mode, ctx.t, ctx.seed = plan, bits, mode, t, seed
        ctx.rot_meta = (rot.dtype, rot.device)
        ctx.theta_meta = (theta.dtype, theta.device)
        return logp

    @staticmethod
    def backward(ctx, grad_logp):
        grot, gth = ctx.plan.log_prob_backward(ctx.bits, grad_logp.contiguous(), ctx.mode, ctx.t, ctx.seed)
        g_rot = torch.from_numpy(np.ascontiguousarray(grot)).to(dtype=ctx.rot_meta[0], device=ctx.rot_meta[1])
        g_th = torch.from_numpy(np.ascontiguousarray(gth)).to(dtype=ctx.theta_meta[0], device=ctx.theta_meta[1])
        return g_rot, g_th, None, None, None, None, None


def log_prob(plan: "api.Plan", bits: torch.Tensor, rot: torch.Tensor, theta: torch.Tensor,
             mode: str = "approx", t: int = 0, seed: int = 0) -> torch.Tensor:
    """log p_b of every bitstring (device tensor), differentiable with respect to
    ``rot`` (complex128 [n_rot, n, n]) and ``theta`` (float64 [k]).  In Raw
    Estimate mode the trajectories stay those sampled from the plan's frozen
    table."""
    return _LogProb.apply(rot, theta, plan, bits, mode, t, seed)


class _SpinRotations(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gens):
        K = gens.detach().cpu().numpy()
        ctx.K = K
        return torch.from_numpy(api.spin_rotations(K)).to(dtype=gens.dtype, device=gens.device)

    @staticmethod
    def backward(ctx, g_rot):
        out = api.spin_rotations_adjoint(ctx.K, g_rot.detach().cpu().numpy())
        return torch.from_numpy(out).to(dtype=g_rot.dtype, device=g_rot.device)


def spin_rotations(gens: torch.Tensor) -> torch.Tensor:
    """Layers exp(K_l) (+) exp(K_l) for anti-Hermitian K_l (complex128 [n_rot, d, d])."""
    return _SpinRotations.apply(gens)


def generator_reals_grad(G_K: np.ndarray) -> np.ndarray:
    """Gradient with respect to the real parameters of an anti-Hermitian K
    ((Re K_ij, Im K_ij) for i < j, then Im K_ii) from dL/dRe K + i dL/dIm K of
    the full matrix (xf_antihermitian_reals_grad)."""
    return api.antihermitian_reals_grad(G_K)
