"""torch.autograd.Function wrappers whose backward passes are the library's
hand-written adjoint kernels (forces, virial, loss gradient)."""
from __future__ import annotations

import torch

from .model import Batch, Potential


def _set_theta(P: Potential, c, xi):
    P.set_params(c.detach().double().cpu().numpy(), xi.detach().double().cpu().numpy())


class MTPEnergy(torch.autograd.Function):
    """E_k(positions, c, xi) for every configuration of a batch.

    forward(pos [N,3] FP64 on the device, c [n_c], xi [m], P, batch) -> E [K].
    backward: dE/dpos = -F (mtp_eval's adjoint), dE/dxi = b (descriptors),
    dE/dc from mtp_loss_grad with the energy weight only."""

    @staticmethod
    def forward(ctx, pos, c, xi, P: Potential, batch: Batch, precision="fp64"):
        _set_theta(P, c, xi)
        b = Batch(batch.atom_offsets, pos.detach().contiguous(), batch.species, batch.cell, batch.pbc)
        out = P.eval(b, precision=precision, forces=True, virial=False, b=True)
        ctx.P, ctx.batch, ctx.precision = P, b, precision
        ctx.save_for_backward(out["forces"], out["b"], out["energy"], c.detach(), xi.detach())
        return out["energy"]

    @staticmethod
    def backward(ctx, gE):
        F, bdesc, E, c, xi = ctx.saved_tensors
        _set_theta(ctx.P, c, xi)   # the parameters of this forward pass
        gE = gE.to(torch.float64)
        atoms_cfg = torch.repeat_interleave(torch.arange(len(gE), device=gE.device),
                                            ctx.batch.atom_offsets.diff())
        g_pos = -F * gE[atoms_cfg][:, None]
        g_xi = gE @ bdesc
        # sum_k gE_k dE_k/dc: the loss sum_k (E_k - E_t,k)^2 with E_t = E - gE / 2
        # has gradient sum_k gE_k dE_k/dtheta
        N, K = ctx.batch.n_atoms, ctx.batch.n_configs
        dev = gE.device
        _, grad = ctx.P.loss_grad(ctx.batch, E - gE / 2, torch.zeros((N, 3), dtype=torch.float64, device=dev),
                                  torch.zeros((K, 3, 3), dtype=torch.float64, device=dev), w_e=1.0, w_f=0.0,
                                  w_s=0.0, scaling="molecules", precision=ctx.precision)
        g_c = grad[ctx.P.m:]
        return g_pos, g_c, g_xi, None, None, None


class MTPLoss(torch.autograd.Function):
    """L(c, xi) of eq. Fitting over a batch with fixed targets; backward is
    mtp_loss_grad."""

    @staticmethod
    def forward(ctx, c, xi, P: Potential, batch: Batch, E_t, F_t, W_t, w_e=1.0, w_f=0.01, w_s=0.001,
                scaling="vibrations", precision="fp64"):
        _set_theta(P, c, xi)
        loss, grad = P.loss_grad(batch, E_t, F_t, W_t, w_e=w_e, w_f=w_f, w_s=w_s, scaling=scaling,
                                 precision=precision)
        ctx.m = P.m
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, gL):
        (grad,) = ctx.saved_tensors
        g = grad * gL.to(torch.float64)
        return g[ctx.m:], g[:ctx.m], None, None, None, None, None, None, None, None, None, None


class MTPLossPositions(torch.autograd.Function):
    """L(positions, c, xi) of eq. Fitting with fixed targets; backward is
    mtp_loss_grad with its position gradient (dL/dx, dL/dc, dL/dxi).

    forward(pos [N,3] FP64 on the device, c [n_c], xi [m], P, batch, E_t, F_t,
    W_t, ...) -> L."""

    @staticmethod
    def forward(ctx, pos, c, xi, P: Potential, batch: Batch, E_t, F_t, W_t, w_e=1.0, w_f=0.01, w_s=0.001,
                scaling="vibrations", precision="fp64"):
        _set_theta(P, c, xi)
        b = Batch(batch.atom_offsets, pos.detach().contiguous(), batch.species, batch.cell, batch.pbc)
        loss, grad, gpos = P.loss_grad(b, E_t, F_t, W_t, w_e=w_e, w_f=w_f, w_s=w_s, scaling=scaling,
                                       precision=precision, pos=True)
        ctx.m = P.m
        ctx.save_for_backward(grad, gpos)
        return loss[0]

    @staticmethod
    def backward(ctx, gL):
        grad, gpos = ctx.saved_tensors
        gL = gL.to(torch.float64)
        g = grad * gL
        return gpos * gL, g[ctx.m:], g[:ctx.m], None, None, None, None, None, None, None, None, None, None
