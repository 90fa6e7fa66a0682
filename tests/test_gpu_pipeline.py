"""GPU tests of the decomposition with the transform overlapped (cds_cholesky_transform_sgauss).

Its results must equal the decomposition followed by the transform of its vectors, bit for
bit, in every precision (each vector's blocks do not depend on how the vectors are batched);
the FP64 blocks also match the oracle's transform (Eq. (transformation)) of the oracle's
vectors.  A capped run transforms the vectors it made; bad arguments write nothing.  Blocks
re-strided in place (cds_restride_blocks, which the binding applies when the row stride is at
least twice the entries used) keep every entry they keep bit for bit.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_0912_1459_amd._lib as A
from tests._blocks import as_float64
from tests._cases import log, oracle_blocks, workload

pytestmark = pytest.mark.gpu


def _dev(x, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


@pytest.fixture(scope="module")
def C():
    import paper_0912_1459_amd.core as C
    return C


def _bits(t: torch.Tensor) -> torch.Tensor:
    """The stored bits (so that -0.0 and 0.0 differ)."""
    return t.contiguous().view({torch.float64: torch.int64, torch.float32: torch.int32,
                                torch.bfloat16: torch.int16}[t.dtype])


def _inputs(name):
    w = workload(name)
    return w, _dev(w.centres), _dev(w.alpha), _dev(w.C)


@pytest.mark.parametrize("name,delta,prec", [("plain", 1e-6, "fp64"), ("small_cage", 1e-6, "fp32"),
                                             ("c60", 1e-6, "fp64"), ("c60", 1e-6, "bf16x3"),
                                             ("c60", 1e-4, "fp32"), ("c60", 1e-4, "bf16x3")])
def test_fused_equals_separate_calls(C, name, delta, prec):
    w, centres, alpha, Cm = _inputs(name)
    log(f"fused decomposition + transform {name} delta={delta} {prec}")
    max_vec = min(C.npairs(w.nbf), 12 * w.nbf)
    cd, B = C.cholesky_transform(delta, centres=centres, alpha=alpha, C=Cm, nocc=w.nocc, sel=w.targets, prec=prec,
                                 max_vec=max_vec)
    ref = C.cholesky(delta, centres=centres, alpha=alpha, max_vec=max_vec, grow=False)
    assert cd.status == ref.status == A.CD_CONVERGED
    assert cd.nvec == ref.nvec
    assert torch.equal(cd.piv[: cd.nvec], ref.piv[: ref.nvec])
    assert torch.equal(_bits(cd.L), _bits(ref.L))
    assert torch.equal(_bits(cd.D), _bits(ref.D))
    Bref = C.transform(ref.Lbuf, ref.nvec, Cm, w.nocc, w.targets, prec, ldk=B.ldk)
    # the fused call writes entries K < nvec rounded up to 64 (the rest of ldk is never read)
    kz = min(B.ldk, C.round_up(cd.nvec, 64))
    assert torch.equal(_bits(B.Bsel)[..., :kz], _bits(Bref.Bsel)[..., :kz])
    assert torch.equal(_bits(B.Bvo)[..., :kz], _bits(Bref.Bvo)[..., :kz])


@pytest.mark.parametrize("name,delta", [("plain", 1e-6), ("c60", 1e-6)])
def test_fused_fp64_matches_oracle(C, name, delta):
    w, centres, alpha, Cm = _inputs(name)
    log(f"fused fp64 vs oracle {name} delta={delta}")
    cd, B = C.cholesky_transform(delta, centres=centres, alpha=alpha, C=Cm, nocc=w.nocc, sel=w.targets,
                                 prec="fp64", max_vec=min(C.npairs(w.nbf), 12 * w.nbf))
    refs, refv = oracle_blocks(name, delta)
    assert cd.nvec == refs.shape[0]
    gs, gv = (x.cpu().numpy() for x in as_float64(B))
    # vectors of the two decompositions agree to rounding (same pivots); B follows them
    scale = max(np.abs(refs).max(), np.abs(refv).max())
    assert np.abs(gs - refs.transpose(1, 2, 0)).max() <= 1e-9 * scale
    assert np.abs(gv - refv.transpose(1, 2, 0)).max() <= 1e-9 * scale
    kz = min(B.ldk, C.round_up(cd.nvec, 64))
    assert torch.all(B.Bsel.reshape(-1, B.ldk)[:, cd.nvec:kz] == 0)
    assert torch.all(B.Bvo.reshape(-1, B.ldk)[:, cd.nvec:kz] == 0)


def _fused_raw(C, w, centres, alpha, Cm, delta, max_vec, ldk, prec=A.PREC_FP64):
    ctx = C.context(0)
    np_ = C.npairs(w.nbf)
    ldl = C.round_up(np_, 64)
    L = torch.zeros((max_vec, ldl), dtype=torch.float64, device="cuda")
    piv = torch.zeros(max_vec, dtype=torch.int64, device="cuda")
    D = torch.zeros(np_, dtype=torch.float64, device="cuda")
    nmo = Cm.shape[1]
    sel = np.ascontiguousarray(np.asarray(w.targets, dtype=np.int32))
    Bsel = torch.full((sel.shape[0] * nmo, ldk), 7.0, dtype=torch.float64, device="cuda")
    Bvo = torch.full(((nmo - w.nocc) * w.nocc, ldk), 7.0, dtype=torch.float64, device="cuda")
    nvec, dmax, status = ctypes.c_int64(-1), ctypes.c_double(), ctypes.c_int32(-9)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = ctx.lib.cds_cholesky_transform_sgauss(
        ctx.h, w.nbf, p(centres), p(alpha), delta, -1.0, -1.0, max_vec, p(L), ldl, p(piv), p(D), prec, p(Cm), nmo,
        w.nocc, sel.shape[0], sel.ctypes.data_as(ctypes.c_void_p), ldk, p(Bsel), p(Bvo), ctypes.byref(nvec),
        ctypes.byref(dmax), ctypes.byref(status))
    torch.cuda.synchronize()
    return rc, int(nvec.value), int(status.value), L, Bsel, Bvo


def test_fused_cap_transforms_the_vectors_made(C):
    w, centres, alpha, Cm = _inputs("c60")
    log("fused decomposition + transform, capped at 300 vectors")
    rc, nvec, status, L, Bsel, Bvo = _fused_raw(C, w, centres, alpha, Cm, 1e-6, 300, 320)
    assert rc == A.CDS_ECAP and status == A.CD_CAP and nvec == 300
    Bref = C.transform(L, nvec, Cm, w.nocc, w.targets, "fp64", ldk=320)
    assert torch.equal(_bits(Bsel), _bits(Bref.Bsel))
    assert torch.equal(_bits(Bvo), _bits(Bref.Bvo))


def test_fused_rejects_short_ldk(C):
    w, centres, alpha, Cm = _inputs("plain")
    log("fused decomposition + transform, ldk < max_vec")
    rc, nvec, status, L, Bsel, Bvo = _fused_raw(C, w, centres, alpha, Cm, 1e-6, 256, 192)
    assert rc == A.CDS_EINVAL
    assert nvec == -1 and status == -9
    assert torch.all(Bsel == 7.0) and torch.all(Bvo == 7.0) and torch.all(L == 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("rows,ldk,ldk_new", [(3001, 640, 64), (1000, 640, 320), (257, 2880, 768), (1, 128, 64)])
def test_restride_keeps_entries(C, prec, rows, ldk, ldk_new):
    log(f"restride {prec} rows={rows} ldk={ldk} -> {ldk_new}")
    g = torch.Generator(device="cuda").manual_seed(rows + ldk)
    shape = (2, rows, ldk) if prec == "bf16x3" else (rows, ldk)
    dt = {"fp64": torch.float64, "fp32": torch.float32, "bf16x3": torch.bfloat16}[prec]
    B = torch.randn(shape, generator=g, device="cuda", dtype=torch.float32).to(dt)
    want = _bits(B[..., :ldk_new]).clone()
    out = C.restride_blocks(B, prec, ldk_new)
    torch.cuda.synchronize()
    assert out.shape == want.shape and out.data_ptr() == B.data_ptr()
    assert torch.equal(_bits(out), want)


def test_restride_rejects_bad_strides(C):
    ctx = C.context(0)
    B = torch.full((100, 640), 7.0, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(B.data_ptr())
    log("restride: stride not halved, rows not 16-byte multiples, misaligned buffer")
    assert ctx.lib.cds_restride_blocks(ctx.h, A.PREC_FP64, 100, 640, 321 + 63, p) == A.CDS_EINVAL
    assert ctx.lib.cds_restride_blocks(ctx.h, A.PREC_FP64, 100, 640, 63, p) == A.CDS_EINVAL
    assert ctx.lib.cds_restride_blocks(ctx.h, A.PREC_FP32, 100, 640, 2, p) == A.CDS_EINVAL
    q = ctypes.c_void_p(B.data_ptr() + 8)
    assert ctx.lib.cds_restride_blocks(ctx.h, A.PREC_FP64, 99, 640, 64, q) == A.CDS_EINVAL
    torch.cuda.synchronize()
    assert torch.all(B == 7.0)
