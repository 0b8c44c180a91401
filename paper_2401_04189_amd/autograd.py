"""E_x as a differentiable function of the orbitals.

`ExchangeEnergy.apply(psi, system, ctx, compute)` returns E_x (a 0-d float64
tensor).  Its forward runs the energy-only path (pair densities, projection,
core-space kernel sum, pair energies; no back-projection) and saves only psi.
Its backward is the exchange action itself, recomputed from psi: the
derivative of E_x = -1/2 sum_ij <psi_i psi_j, phi_ij>_W with respect to the
grid values of psi_i is 2 w(r) (Vx psi_i)(r) (the functional derivative of
the exact-exchange term, with w = q0 q1 q2 the grid weights), which the
library writes directly, scaled by the incoming gradient, through its
out_scale / out_weighted epilogue.  No pair data is kept between forward and
backward.
"""
from __future__ import annotations

import torch

from . import txe


class ExchangeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, psi, sysm, ctx, compute="f64"):
        psi_c = psi.contiguous()
        _, ex, _ = txe.apply(ctx, sysm, psi_c, compute=compute, symmetric=True, want_vx=False)
        fctx.save_for_backward(psi_c)
        fctx.sysm = sysm
        fctx.txe_ctx = ctx
        fctx.compute = compute
        return ex

    @staticmethod
    def backward(fctx, g):
        (psi,) = fctx.saved_tensors
        scale = (2.0 * g).to(dtype=torch.float64, device=psi.device).reshape(()).contiguous()
        grad, _, _ = txe.apply(fctx.txe_ctx, fctx.sysm, psi, compute=fctx.compute, symmetric=True,
                               want_vx=True, out_scale=scale, out_weighted=True)
        return grad, None, None, None


def exchange_energy(psi, sysm, ctx, compute="f64"):
    """E_x(psi) with autograd support (symmetric mode over all orbitals)."""
    return ExchangeEnergy.apply(psi, sysm, ctx, compute)
