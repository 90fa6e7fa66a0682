"""torch.autograd wrappers whose backward passes call the hand-written adjoints.

  Transform.apply(L, C, nvec, nocc, sel, prec)  -> (Bsel, Bvo)        Eq. (transformation)
  QPSolve.apply(Bsel, Bvo, eps, meta)           -> omega (nsel,)      Eqs. (qpapp)/(iter)

QPSolve's backward differentiates the converged Newton fixed point implicitly:
d(w*)/d(theta) = P d(e_q + Sigma_qq(w*; theta))/d(theta) with P = 1/(1 - Sigma'(w*)), computed by
cds_qp_adjoint.  That formula holds only at a fixed point, so the backward raises for any
target whose forward solve did not converge (status MAX_ITER or NONFINITE).  Transform's
backward is C_bar = sum_K L^K C (Bbar^K + Bbar^K^T) by cds_transform_adjoint.  FP64 and FP32 blocks are differentiable (the split-bf16 planes are not).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import _lib as A
from . import core


@dataclasses.dataclass
class SolveMeta:
    nvec: int
    ldk: int
    nmo: int
    nocc: int
    sel: np.ndarray
    prec: int
    conv: float = 1e-12
    max_iter: int = 100
    mode: str = "residues"
    result: core.QPResult | None = None   # the last forward's result (for inspection only)


def _blocks(Bsel, Bvo, meta: SolveMeta) -> core.BBlocks:
    return core.BBlocks(meta.prec, Bsel, Bvo, meta.nvec, meta.ldk, meta.nmo, meta.nocc, meta.sel)


class QPSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Bsel, Bvo, eps, meta: SolveMeta):
        if meta.prec == A.PREC_BF16X3:
            raise ValueError("QPSolve differentiates FP64 or FP32 blocks only")
        B = _blocks(Bsel.detach(), Bvo.detach(), meta)
        r = core.qp_solve(B, eps.detach(), conv=meta.conv, max_iter=meta.max_iter, mode=meta.mode)
        meta.result = r
        # the backward uses this forward's own energies and statuses (meta may be reused)
        ctx.meta = meta
        ctx.omega = r.omega.copy()
        ctx.status = r.status.copy()
        ctx.save_for_backward(Bsel, Bvo, eps)
        return torch.tensor(r.omega, dtype=torch.float64, device=eps.device)

    @staticmethod
    def backward(ctx, gomega):
        Bsel, Bvo, eps = ctx.saved_tensors
        meta = ctx.meta
        bad = np.flatnonzero(ctx.status != A.QP_CONVERGED)
        if bad.size:
            raise RuntimeError(f"QPSolve.backward: targets {meta.sel[bad].tolist()} did not converge "
                               f"(status {ctx.status[bad].tolist()}); the implicit gradient needs the fixed point")
        B = _blocks(Bsel.detach(), Bvo.detach(), meta)
        gs, gv, ge = core.qp_adjoint(B, eps.detach(), ctx.omega, gomega.detach().double().cpu().numpy())
        return gs.to(Bsel.dtype).reshape(Bsel.shape), gv.to(Bvo.dtype).reshape(Bvo.shape), ge, None


class Transform(torch.autograd.Function):
    @staticmethod
    def forward(ctx, L, C, nvec: int, nocc: int, sel, prec="fp64", ldk=None):
        prec_i = core._prec(prec)
        if prec_i == A.PREC_BF16X3:
            raise ValueError("Transform differentiates FP64 or FP32 outputs only")
        B = core.transform(L.detach(), nvec, C.detach(), nocc, sel, prec_i, ldk=ldk)
        ctx.save_for_backward(L, C)
        ctx.info = (nvec, nocc, np.asarray(sel, dtype=np.int32), B.ldk)
        return B.Bsel, B.Bvo

    @staticmethod
    def backward(ctx, gBsel, gBvo):
        L, C = ctx.saved_tensors
        nvec, nocc, sel, ldk = ctx.info
        if gBsel is None:
            gBsel = torch.zeros((len(sel) * C.shape[1], ldk), dtype=torch.float64, device=C.device)
        if gBvo is None:
            gBvo = torch.zeros(((C.shape[1] - nocc) * nocc, ldk), dtype=torch.float64, device=C.device)
        dt = torch.float64 if gBsel.dtype == torch.float64 else torch.float32
        Cbar = core.transform_adjoint(L.detach(), nvec, C.detach(), nocc, sel, gBsel.to(dt).contiguous(),
                                      gBvo.to(dt).contiguous(), ldk)
        return None, Cbar, None, None, None, None, None


def quasiparticle_energies(L, nvec: int, C, eps, nocc: int, sel, prec="fp64", conv=1e-12, mode="residues"):
    """omega(C, eps) through the transform and the solve, differentiable in C and eps."""
    Bsel, Bvo = Transform.apply(L, C, nvec, nocc, sel, prec)
    ldk = Bsel.shape[-1]
    meta = SolveMeta(nvec, ldk, C.shape[1], nocc, np.asarray(sel, dtype=np.int32), core._prec(prec),
                     conv=conv, mode=mode)
    return QPSolve.apply(Bsel, Bvo, eps, meta)
