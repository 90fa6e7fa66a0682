"""GPU parity of the transform, the self-energy and the quasi-particle solves.

FP64 paths: B within 1e-12 of max|B|, Sigma/Sigma'/w/P within 1e-10 Eh of the
oracle, identical Newton statuses.  FP32 and split-bf16 (3-term) paths: every
quasi-particle energy within 1 meV of the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from oracle import mo, selfenergy as SE
from paper_0912_1459_amd import inputs as I
from tests._blocks import as_float64, blocks_from_numpy
from tests._cases import EV, log, oracle_blocks, oracle_cd, oracle_qp, workload

pytestmark = pytest.mark.gpu

MEV = 1e-3 / EV


def _dev(x, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


@pytest.fixture(scope="module")
def cds():
    import paper_0912_1459_amd.core as C
    return C


def _L_on_device(name, delta):
    r = oracle_cd(name, delta)
    return _dev(r.L.T), r.M


@pytest.mark.parametrize("name,delta", [("plain", 1e-6), ("small_cage", 1e-6), ("c60", 1e-6)])
def test_transform_fp64(cds, name, delta):
    w = workload(name)
    log(f"transform fp64 {name}")
    Ld, M = _L_on_device(name, delta)
    refs, refv = oracle_blocks(name, delta)
    B = cds.transform(Ld, M, _dev(w.C), w.nocc, w.targets, "fp64")
    gs, gv = as_float64(B)
    gs, gv = gs.cpu().numpy(), gv.cpu().numpy()
    scale = max(np.abs(refs).max(), np.abs(refv).max())
    assert np.abs(gs - refs.transpose(1, 2, 0)).max() <= 1e-12 * scale
    assert np.abs(gv - refv.transpose(1, 2, 0)).max() <= 1e-12 * scale
    # padding beyond nvec is zero
    assert torch.all(B.Bsel.reshape(-1, B.ldk)[:, M:] == 0)


# Per-element bound of a reduced-precision transform, relative to (|C|^T |L^K| |C|)_pq (the sum
# of the absolute values of the terms of B^K_pq): two products, each over at most nbf terms with
# FP32 accumulation (nbf * 2^-24 per product); split-bf16 operands hi + lo represent an FP32
# value to 2^-18 relative and the dropped lo*lo term is below 2^-18 of the product, so each
# split product adds 3 * 2^-18.  Doubled for the two stages.
_U = {"fp32": lambda n: 2 * n * 2.0 ** -24, "bf16x3": lambda n: 2 * (n * 2.0 ** -24 + 3 * 2.0 ** -18)}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_transform_reduced(cds, prec):
    name, delta = "c60", 1e-6
    w = workload(name)
    log(f"transform {prec} {name}")
    Ld, M = _L_on_device(name, delta)
    refs, refv = oracle_blocks(name, delta)
    r = oracle_cd(name, delta)
    abss, absv = mo.transform_blocks(np.abs(r.L), np.abs(w.C), w.nocc, w.targets)
    B = cds.transform(Ld, M, _dev(w.C), w.nocc, w.targets, prec)
    gs, gv = as_float64(B)
    u = _U[prec](w.nbf)
    rs = np.abs(gs.cpu().numpy() - refs.transpose(1, 2, 0)) / (u * abss.transpose(1, 2, 0) + 1e-300)
    rv = np.abs(gv.cpu().numpy() - refv.transpose(1, 2, 0)) / (u * absv.transpose(1, 2, 0) + 1e-300)
    scale = max(np.abs(refs).max(), np.abs(refv).max())
    log(f"  max error / per-element bound = {max(rs.max(), rv.max()):.3e}; max error / max |B| = "
        f"{max(np.abs(gs.cpu().numpy() - refs.transpose(1, 2, 0)).max(), np.abs(gv.cpu().numpy() - refv.transpose(1, 2, 0)).max()) / scale:.2e}")
    assert rs.max() <= 1.0 and rv.max() <= 1.0


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-7), ("bf16x3", 2e-5)])
def test_transform_fp64_working_precision(cds, prec, tol):
    # GEMMs in FP64, only the output rounded: per element within one rounding of the output
    # format (FP32: 2^-24; split bf16 from the FP32 value: about 2^-17) relative to the largest B
    name, delta = "c60", 1e-6
    w = workload(name)
    log(f"transform {prec} output, FP64 working precision, {name}")
    Ld, M = _L_on_device(name, delta)
    refs, refv = oracle_blocks(name, delta)
    ctx = cds.Context(0)
    ctx.set_transform_fp64(True)
    B = cds.transform(Ld, M, _dev(w.C), w.nocc, w.targets, prec, ctx=ctx)
    gs, gv = as_float64(B)
    scale = max(np.abs(refs).max(), np.abs(refv).max())
    es = np.abs(gs.cpu().numpy() - refs.transpose(1, 2, 0)).max() / scale
    ev = np.abs(gv.cpu().numpy() - refv.transpose(1, 2, 0)).max() / scale
    log(f"  max error / max |B|: {max(es, ev):.2e}")
    assert es <= tol and ev <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_transform_scattered_selection(cds, prec):
    # targets out of order, repeated, occupied and virtual mixed: each selected orbital's block
    # must still be its own row of B^K (the transform shares the occupied rows and groups runs)
    name, delta = "small_cage", 1e-6
    w = workload(name)
    nmo = w.C.shape[1]
    sel = np.array([w.nocc + 3, 2, w.nocc + 3, w.nocc - 1, w.nocc, 0, nmo - 1, w.nocc + 1], dtype=np.int32)
    log(f"transform {prec} {name} selection {sel.tolist()}")
    Ld, M = _L_on_device(name, delta)
    r = oracle_cd(name, delta)
    refs, refv = mo.transform_blocks(r.L, w.C, w.nocc, sel)
    abss, absv = mo.transform_blocks(np.abs(r.L), np.abs(w.C), w.nocc, sel)
    B = cds.transform(Ld, M, _dev(w.C), w.nocc, sel, prec)
    gs, gv = (x.cpu().numpy() for x in as_float64(B))
    u = 1e-12 * max(np.abs(refs).max(), np.abs(refv).max()) if prec == "fp64" else None
    if u is not None:
        assert np.abs(gs - refs.transpose(1, 2, 0)).max() <= u
        assert np.abs(gv - refv.transpose(1, 2, 0)).max() <= u
    else:
        b = _U[prec](w.nbf)
        assert (np.abs(gs - refs.transpose(1, 2, 0)) <= b * abss.transpose(1, 2, 0) + 1e-300).all()
        assert (np.abs(gv - refv.transpose(1, 2, 0)) <= b * absv.transpose(1, 2, 0) + 1e-300).all()
    # the repeated target's two blocks are the same bits
    bs = B.Bsel.reshape(*B.Bsel.shape[:-2], len(sel), nmo, B.ldk)
    assert torch.equal(bs[..., 0, :, :M], bs[..., 2, :, :M])


@pytest.mark.parametrize("name", ["plain", "c60"])
def test_sigma2_fp64_trial_energies(cds, name):
    w = workload(name)
    log(f"sigma2 fp64 {name}")
    Bs, Bv = oracle_blocks(name, 1e-6)
    B = blocks_from_numpy(Bs, Bv, w.nocc, w.targets, "fp64")
    eps = _dev(w.eps)
    om = w.trial_energies() if w.n_trial > 1 else np.stack([w.eps[w.targets], w.eps[w.targets] + 0.03], 1)
    s, ds = cds.sigma2(B, eps, om)
    for k, q in enumerate(w.targets):
        x, y = SE.xy_from_B(Bs[:, k, :], Bv, w.nocc)
        for t in range(om.shape[1]):
            rs, rds = SE.sigma(x, y, w.eps, w.nocc, om[k, t])
            assert abs(s[k, t] - rs) <= 1e-10
            assert abs(ds[k, t] - rds) <= 1e-10 * max(1.0, abs(rds))


@pytest.mark.parametrize("name,mode", [("plain", "residues"), ("plain", "recompute"),
                                       ("c60", "residues"), ("c60", "recompute")])
def test_qp_solve_fp64(cds, name, mode):
    w = workload(name)
    log(f"qp_solve fp64 {name} {mode}")
    Bs, Bv = oracle_blocks(name, 1e-6)
    ref = oracle_qp(name, 1e-6, 1e-12)
    B = blocks_from_numpy(Bs, Bv, w.nocc, w.targets, "fp64")
    got = cds.qp_solve(B, _dev(w.eps), conv=1e-12, max_iter=50, mode=mode)
    assert list(got.status) == [r.status for r in ref]
    om = np.array([r.omega for r in ref])
    po = np.array([r.pole for r in ref])
    assert np.abs(got.omega - om).max() <= 1e-10
    assert np.abs(got.pole - po).max() <= 1e-10
    assert np.all((got.pole > 0) & (got.pole <= 1))


def test_end_to_end_fp64_c60(cds):
    # the whole path on the GPU: on-demand CD -> transform -> Newton
    w = workload("c60")
    log("end-to-end fp64 c60")
    cd = cds.cholesky(1e-6, centres=_dev(w.centres), alpha=_dev(w.alpha))
    ref_cd = oracle_cd("c60", 1e-6)
    assert np.array_equal(cd.piv[: cd.nvec].cpu().numpy(), ref_cd.piv)
    B = cds.transform(cd.Lbuf, cd.nvec, _dev(w.C), w.nocc, w.targets, "fp64")
    got = cds.qp_solve(B, _dev(w.eps), conv=1e-12)
    ref = oracle_qp("c60", 1e-6, 1e-12)
    assert np.abs(got.omega - np.array([r.omega for r in ref])).max() <= 1e-10
    assert np.abs(got.pole - np.array([r.pole for r in ref])).max() <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_reduced_precision_within_one_mev(cds, prec):
    w = workload("c60")
    log(f"precision {prec} c60")
    cd = cds.cholesky(1e-6, centres=_dev(w.centres), alpha=_dev(w.alpha))
    B = cds.transform(cd.Lbuf, cd.nvec, _dev(w.C), w.nocc, w.targets, prec)
    got = cds.qp_solve(B, _dev(w.eps), conv=1e-10)
    ref = oracle_qp("c60", 1e-6, 1e-12)
    err = np.abs(got.omega - np.array([r.omega for r in ref]))
    log(f"  max |dw| = {err.max() * EV * 1e3:.4f} meV")
    assert np.all(got.status == 0)
    assert err.max() <= MEV


def test_qp_statuses_forced(cds):
    w = workload("plain")
    Bs, Bv = oracle_blocks("plain", 1e-6)
    B = blocks_from_numpy(Bs, Bv, w.nocc, w.targets, "fp64")
    got = cds.qp_solve(B, _dev(w.eps), conv=1e-14, max_iter=1)
    assert np.all(got.status == 1)
    # start on a pole of the 2h1p family of target HOMO
    q = w.nocc - 1
    om0 = w.eps[w.targets].copy()
    s = list(w.targets).index(q)
    om0[s] = 2 * w.eps[0] - w.eps[w.nocc]
    got = cds.qp_solve(B, _dev(w.eps), omega0=om0, conv=1e-12)
    x, y = SE.xy_from_B(Bs[:, s, :], Bv, w.nocc)
    ref = SE.newton(x, y, w.eps, w.nocc, q, omega0=om0[s], conv=1e-12)
    assert ref.status == SE.STATUS_NON_FINITE and got.status[s] == 2


def test_ragged_random_blocks(cds):
    # sizes that are not multiples of any tile: nocc=7, nvirt=13, M=37, 3 targets
    nocc, nvirt, M = 7, 13, 37
    n = nocc + nvirt
    Bfull = I.random_factor(n, M, 5, scale=0.15)
    eps = I.random_energies(nocc, nvirt, 5)
    sel = np.array([nocc - 2, nocc - 1, nocc])
    Bs = np.ascontiguousarray(Bfull[:, sel, :])
    Bv = np.ascontiguousarray(Bfull[:, nocc:, :nocc])
    ref = SE.solve_targets(Bs, Bv, eps, nocc, sel, conv=1e-12)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-5), ("bf16x3", 1e-4)):
        B = blocks_from_numpy(Bs, Bv, nocc, sel, prec)
        got = cds.qp_solve(B, _dev(eps), conv=1e-12)
        assert np.abs(got.omega - np.array([r.omega for r in ref])).max() <= tol, prec


def test_unfused_fallback_matches_oracle(cds):
    # blocks whose row length does not suit the fused kernel's 16-byte K stages (ldk = M = 37)
    # take the path that stores the integrals; same sizes as the ragged case above
    nocc, nvirt, M = 7, 13, 37
    n = nocc + nvirt
    Bfull = I.random_factor(n, M, 5, scale=0.15)
    eps = I.random_energies(nocc, nvirt, 5)
    sel = np.array([nocc - 2, nocc - 1, nocc])
    Bs = np.ascontiguousarray(Bfull[:, sel, :])
    Bv = np.ascontiguousarray(Bfull[:, nocc:, :nocc])
    ref = SE.solve_targets(Bs, Bv, eps, nocc, sel, conv=1e-12)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-5)):
        B = blocks_from_numpy(Bs, Bv, nocc, sel, prec, ldk=M)
        for mode in ("residues", "recompute"):
            got = cds.qp_solve(B, _dev(eps), conv=1e-12, mode=mode)
            assert np.abs(got.omega - np.array([r.omega for r in ref])).max() <= tol, (prec, mode)
