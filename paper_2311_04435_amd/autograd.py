"""The SCA potential as a differentiable torch function.

Forward: factorise every A_ns = i w_n I - H_s(phi) (sca_factorize) and
return (Omega, Omega~) of Eq. (7).  The factors stay in a caller-owned
device buffer attached to the autograd node.

Backward: sca_grad_from_factors turns the kept factors into
dOmega/dphi_i = 2 phi_i / U - 2 T sum_s s sum_n Re (A_ns^-1)_ii without
factorising again (on the FP64 blocked path it runs the triangular inverses
and the diagonal there; the fused small path and the FP32-refined route
finish the diagonal in the forward and the backward only reduces it).
Omega and Omega~ differ by a constant, so the incoming gradients of both
outputs add onto the same dOmega/dphi.

Not twice differentiable.  phi must not change in place between forward
and backward; torch's version counter on the saved tensor enforces that.
A repeated backward of the same graph (retain_graph=True) factorises again
first, because the FP64 blocked backward inverts the factors in place.
"""
from __future__ import annotations

import torch

from . import Params, default_context


class SCAPotential(torch.autograd.Function):
    """(Omega, Omega~) = SCAPotential.apply(phi, params)."""

    @staticmethod
    def forward(ctx, phi: torch.Tensor, p: Params):
        c = default_context()
        contiguous = phi.is_contiguous()
        x = phi.detach() if contiguous else phi.detach().contiguous()
        if p.factor == "eigh":
            # the spectral route keeps no factors: its gradient costs the
            # same pass as the potential, so the forward keeps it
            g, o2 = c.grad(p, x)
            ctx.save_for_backward(phi if contiguous else x)
            ctx.sca = (c, p, g)
            ctx.used = False
            return o2
        factors = torch.empty(c.factor_bytes(p), dtype=torch.uint8,
                              device=x.device)
        o2 = c.factorize(p, x, factors)
        # the input itself when possible, so that an in-place change of phi
        # before the backward is caught by torch
        ctx.save_for_backward(phi if contiguous else x)
        ctx.sca = (c, p, factors)
        ctx.used = False
        return o2

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gout: torch.Tensor):
        (phi,) = ctx.saved_tensors
        c, p, factors = ctx.sca
        if p.factor == "eigh":
            return factors * (gout[0] + gout[1]), None
        x = phi.detach().contiguous()
        if ctx.used:
            # a repeated backward (retain_graph): the FP64 blocked path has
            # inverted the factors in place, so factorise again
            c.factorize(p, x, factors)
        ctx.used = True
        g = c.grad_from_factors(p, x, factors)
        return g * (gout[0] + gout[1]), None


def potential(p: Params, phi: torch.Tensor) -> torch.Tensor:
    """Differentiable (Omega, Omega~) at phi (float64 CUDA tensor of N)."""
    return SCAPotential.apply(phi, p)
