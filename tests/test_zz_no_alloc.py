"""The allocation-free self-energy entry point against cds_sigma2.

cds_sigma2_noalloc keeps every device buffer in one static array per GPU (no hipMalloc); it
must give cds_sigma2's results bit for bit (same kernels, same summation order).  Two calls in a
row through the C ABI, the second smaller (fewer targets, fewer trial energies, so the array
holds the first call's larger contents), each against cds_sigma2 and against the oracle's
Eq. (SE), in FP64 and FP32; the context's workspace stays empty throughout.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import selfenergy as SE
from tests._blocks import blocks_from_numpy
from tests._cases import log, oracle_blocks, workload

pytestmark = pytest.mark.gpu


def _dev(x, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


def _call(ctx, name, B, eps, nsel, om):
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    om = np.ascontiguousarray(om[:nsel], dtype=np.float64)
    T = om.shape[1]
    s = np.zeros((nsel, T))
    ds = np.zeros((nsel, T))
    sel = np.ascontiguousarray(B.sel[:nsel], dtype=np.int32)
    rc = getattr(ctx.lib, name)(ctx.h, B.prec, B.nvec, B.ldk, B.nmo, B.nocc, nsel, vp(sel),
                                ctypes.c_void_p(B.Bsel.data_ptr()), ctypes.c_void_p(B.Bvo.data_ptr()),
                                ctypes.c_void_p(eps.data_ptr()), T, vp(om), vp(s), vp(ds))
    ctx.check(rc)
    return s, ds


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sigma2_noalloc_matches_sigma2(prec):
    import paper_0912_1459_amd.core as C
    w = workload("c60")
    Bs, Bv = oracle_blocks("c60", 1e-6)
    B = blocks_from_numpy(Bs, Bv, w.nocc, w.targets, prec)
    eps = _dev(w.eps)
    om = w.trial_energies()
    ctx = C.Context(0)
    assert ctx.workspace_bytes() == 0
    for nsel, T in ((len(w.targets), om.shape[1]), (5, 2)):
        log(f"allocation-free sigma2 {prec}: {nsel} targets x {T} trial energies")
        got = _call(ctx, "cds_sigma2_noalloc", B, eps, nsel, om[:, :T])
        assert ctx.workspace_bytes() == 0
        ref = _call(C.Context(0), "cds_sigma2", B, eps, nsel, om[:, :T])
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        if prec == "fp64":
            for k in range(nsel):
                x, y = SE.xy_from_B(Bs[:, k, :], Bv, w.nocc)
                rs, rds = SE.sigma(x, y, w.eps, w.nocc, om[k, T - 1])
                assert abs(got[0][k, T - 1] - rs) <= 1e-10
                assert abs(got[1][k, T - 1] - rds) <= 1e-10 * max(1.0, abs(rds))


def test_sigma2_noalloc_rejects_oversize():
    # the most trial energies on c60 fit; a shape whose partial sums exceed the array is an
    # argument error before any device work (the blocks are never read)
    import paper_0912_1459_amd.core as C
    import paper_0912_1459_amd._lib as A
    w = workload("c60")
    Bs, Bv = oracle_blocks("c60", 1e-6)
    B = blocks_from_numpy(Bs, Bv, w.nocc, w.targets, "fp64")
    ctx = C.Context(0)
    om = np.repeat(w.trial_energies(), 2, axis=1)                      # T = 16
    s, ds = _call(ctx, "cds_sigma2_noalloc", B, _dev(w.eps), len(w.targets), om)
    ref = _call(C.Context(0), "cds_sigma2", B, _dev(w.eps), len(w.targets), om)
    assert np.array_equal(s, ref[0]) and np.array_equal(ds, ref[1])
    # nocc = 8, nvirt = 2048: 8 x 136 + 2048 tasks per target; 100 targets x 16 trial energies
    # need 80 MB of partial sums
    nocc, nmo, nsel, ldk = 8, 2056, 100, 64
    Z = C.BBlocks(A.PREC_FP64, torch.zeros((nsel * nmo, ldk), dtype=torch.float64, device="cuda"),
                  torch.zeros(((nmo - nocc) * nocc, ldk), dtype=torch.float64, device="cuda"), 64, ldk, nmo,
                  nocc, np.arange(nsel, dtype=np.int32))
    eps = _dev(np.concatenate([np.linspace(-1.5, -0.3, nocc), np.linspace(0.1, 3.0, nmo - nocc)]))
    with pytest.raises(C.CdsError) as e:
        _call(ctx, "cds_sigma2_noalloc", Z, eps, nsel, np.zeros((nsel, 16)))
    assert e.value.code == A.CDS_EINVAL and "scratch" in str(e.value)
    assert ctx.workspace_bytes() == 0
