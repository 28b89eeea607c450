"""Reverse-mode derivative of a final-state objective through the HIP adjoint.

``qlg_objective(psi0, g, ...)`` returns L(psi_T) (energy, or fidelity to a
target) of the QLG evolution of psi0 as a differentiable torch scalar:
backward() yields dL/dpsi0 (torch's complex convention dL/dRe + i dL/dIm) and
dL/d(g0, g1, g2).  Forward and reverse sweeps run in libqlg's kernels
(checkpoint every K steps, FP64 self-interaction Jacobian); this module only
moves buffers between torch and the C ABI.
"""
from __future__ import annotations

from typing import Optional

import torch

from .qlg import Lattice


class QLGObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0: torch.Tensor, g: torch.Tensor, ndim: int, eps: float, nsteps: int,
                checkpoint_every: int, dtype: str, split: str, kind: str, target: Optional[torch.Tensor],
                V, mu: float):
        shape = psi0.shape
        nx = [shape[-1]]
        ny = [shape[-2]] if ndim >= 2 else None
        nz = [shape[-3]] if ndim == 3 else None
        lat = Lattice(ndim, nx, ny, nz, g=[float(v) for v in g.detach().cpu()], eps=eps, dtype=dtype, split=split,
                      device=psi0.device if psi0.is_cuda else "cuda:0")
        if V is not None or mu != 0.0:
            lat.set_potential(V, mu)
        lat.set_psi([psi0.detach()])
        ckpt = lat.forward_record(nsteps, checkpoint_every)
        value, lam, dg_explicit = lat.objective_grad(kind, [target.detach()] if target is not None else None)
        ctx.lat, ctx.ckpt, ctx.lam, ctx.dg_explicit = lat, ckpt, lam, dg_explicit
        ctx.nsteps, ctx.K = nsteps, checkpoint_every
        ctx.psi_shape, ctx.psi_dtype, ctx.psi_device = shape, psi0.dtype, psi0.device
        ctx.g_dtype, ctx.g_device = g.dtype, g.device
        return torch.tensor(value, dtype=torch.float64, device=psi0.device)

    @staticmethod
    def backward(ctx, grad_out):
        lat = ctx.lat
        dg = lat.adjoint_step(ctx.nsteps, ctx.K, ctx.ckpt, ctx.lam)
        # psi0 enters as a = b = psi0 / 2: the library's adjoint of that encoding
        dpsi = lat.set_psi_adjoint(ctx.lam)[0]
        dgt = torch.tensor([a + b for a, b in zip(dg, ctx.dg_explicit)], dtype=ctx.g_dtype, device=ctx.g_device)
        go = grad_out.to(torch.float64)
        dpsi = (go.to(dpsi.device) * dpsi).to(ctx.psi_dtype).to(ctx.psi_device)
        lat.close()
        return dpsi, go.to(dgt.device) * dgt, None, None, None, None, None, None, None, None, None, None


def qlg_objective(psi0: torch.Tensor, g: torch.Tensor, *, eps: float, nsteps: int, checkpoint_every: int = 64,
                  dtype: str = "c128", split: str = "interleaved", kind: str = "energy",
                  target: Optional[torch.Tensor] = None, V=None, mu: float = 0.0) -> torch.Tensor:
    """L(psi_T) for psi0 of shape (5, nx), (5, ny, nx) or (5, nz, ny, nx); differentiable in psi0 and g.
    V (an array of the spatial shape, or None) and mu add the external and chemical potential
    (V + mu) psi_m to the equation of motion; they are constants of the derivative."""
    ndim = psi0.dim() - 1
    return QLGObjective.apply(psi0, g, ndim, float(eps), int(nsteps), int(checkpoint_every), dtype, split,
                              kind, target, V, float(mu))
