"""Upload of oracle-layout B blocks into the library's block layout (test infrastructure).

The oracle's blocks Bsel (M, nsel, nmo) and Bvo (M, nvirt, nocc) are written K-contiguous and
padded to ldk, in the storage each precision's kernels read: double, float, or the split-bf16
pair of planes (hi = x rounded to bf16, lo = the FP32 remainder rounded to bf16), the same
split the library's transform writes.  Only the tests use this; the product path forms its
blocks on the device.
"""
from __future__ import annotations

import numpy as np
import torch

import paper_0912_1459_amd.core as C
from paper_0912_1459_amd import _lib as A


def blocks_from_numpy(Bsel: np.ndarray, Bvo: np.ndarray, nocc: int, sel, prec="fp64", *, ldk=None,
                      device="cuda") -> C.BBlocks:
    prec = C._prec(prec)
    M, nsel, nmo = Bsel.shape
    ldk = ldk or C.round_up(M, 64)
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))

    def pack(x, rows):
        y = np.zeros((rows, ldk))
        y[:, :M] = x.reshape(M, rows).T
        t = torch.from_numpy(y).to(device)
        if prec == A.PREC_FP64:
            return t.contiguous()
        if prec == A.PREC_FP32:
            return t.to(torch.float32).contiguous()
        f = t.to(torch.float32)
        hi = f.to(torch.bfloat16)
        lo = (f - hi.to(torch.float32)).to(torch.bfloat16)
        return torch.stack([hi, lo]).contiguous()
    return C.BBlocks(prec, pack(Bsel, nsel * nmo), pack(Bvo, Bvo.shape[1] * nocc), M, ldk, nmo, nocc, sel)


def as_float64(B: C.BBlocks):
    """(Bsel (nsel, nmo, nvec), Bvo (nvirt, nocc, nvec)) in FP64: the values the kernels use
    (hi + lo for split-bf16 planes)."""
    def f(t, rows):
        if B.prec == A.PREC_BF16X3:
            x = t[0].to(torch.float64) + t[1].to(torch.float64)
        else:
            x = t.to(torch.float64)
        return x.reshape(rows, B.ldk)[:, : B.nvec]
    bs = f(B.Bsel, B.nsel * B.nmo).reshape(B.nsel, B.nmo, B.nvec)
    bv = f(B.Bvo, B.nvirt * B.nocc).reshape(B.nvirt, B.nocc, B.nvec)
    return bs, bv
