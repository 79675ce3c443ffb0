"""torch.autograd glue: the free energy as a function of H and S values, and
the Slater-Koster map from positions to H and S values.

    H, S = SKFn.apply(pos, ctx)          # pattern fixed by ctx.sk_build
    A = EnergyFn.apply(H, S, ctx, opts)  # Mermin free energy, eV
    A.backward()                         # pos.grad = dA/dR, forces = -pos.grad

EnergyFn.backward returns dA/dH = gA rho and dA/dS = -gA pi (pi the
energy-density matrix), computed on the device by the library's pass 2 with
the Krylov columns recomputed (memory-saving workflow) or read back (store
workflow): the density-matrix reading of the forces (Eq. 2 and the force
paragraph after Eq. 1).  SKFn.backward contracts them with the analytic
Slater-Koster derivatives on the device.  Gradients come back as tensors on
the device and dtype of the inputs, whatever the context's output kind.
"""
from __future__ import annotations

import torch


def _as_tensor(x, like):
    if isinstance(x, torch.Tensor):
        return x.to(device=like.device, dtype=like.dtype)
    return torch.as_tensor(x, dtype=like.dtype, device=like.device)


class EnergyFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, H, S, mctx, opts: dict):
        mctx.update_values(H.detach(), S.detach())
        _, _, A = mctx.solve(**opts)
        fctx.mctx = mctx
        fctx.save_for_backward(H)
        return torch.tensor(A, dtype=H.dtype, device=H.device)

    @staticmethod
    def backward(fctx, gA):
        (H,) = fctx.saved_tensors
        dH, dS = fctx.mctx.backward(float(gA))
        return _as_tensor(dH, H), _as_tensor(dS, H), None, None


class SKFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, pos, mctx):
        H, S = mctx.sk_values(pos.detach())
        fctx.mctx = mctx
        fctx.save_for_backward(pos)
        return _as_tensor(H, pos), _as_tensor(S, pos)

    @staticmethod
    def backward(fctx, gH, gS):
        (pos,) = fctx.saved_tensors
        z = torch.zeros_like
        gH = z(gH) if gH is None else gH
        gS = z(gS) if gS is None else gS
        grad = fctx.mctx.sk_vjp(pos.detach(), gH.contiguous(), gS.contiguous())
        return _as_tensor(grad, pos), None
