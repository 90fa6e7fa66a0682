"""GPU parity of the hand-written adjoint (implicit differentiation of the
Newton fixed point) against the oracle gradient, and of the transform adjoint.
"""
import numpy as np
import pytest
import torch

from oracle import selfenergy as SE
from tests._blocks import blocks_from_numpy
from tests._cases import log, oracle_blocks, oracle_cd, workload

pytestmark = pytest.mark.gpu


def _dev(x, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


@pytest.fixture(scope="module")
def cds():
    import paper_0912_1459_amd.core as C
    return C


def _oracle_grads(name, sel_idx, wbar, conv=1e-14):
    w = workload(name)
    Bs, Bv = oracle_blocks(name, 1e-6)
    gBs = np.zeros_like(Bs)
    gBv = np.zeros_like(Bv)
    ge = np.zeros(w.nmo)
    oms = []
    for k, s in enumerate(sel_idx):
        q = int(w.targets[s])
        x, y = SE.xy_from_B(Bs[:, s, :], Bv, w.nocc)
        om = SE.newton(x, y, w.eps, w.nocc, q, conv=conv, max_iter=100).omega
        oms.append(om)
        g = SE.qp_gradient(Bs[:, s, :], Bv, w.eps, w.nocc, q, om)
        gBs[:, s, :] += wbar[k] * g.Bsel_q
        gBv += wbar[k] * g.Bvo
        ge += wbar[k] * g.eps
    return np.array(oms), gBs, gBv, ge


@pytest.mark.parametrize("name", ["plain", "c60"])
def test_qp_adjoint_fp64(cds, name):
    w = workload(name)
    log(f"adjoint fp64 {name}")
    Bs, Bv = oracle_blocks(name, 1e-6)
    sel_idx = [list(w.targets).index(w.nocc - 1), list(w.targets).index(w.nocc)]
    sel = w.targets[sel_idx]
    wbar = np.array([1.0, -0.5])
    oms, gBs, gBv, ge = _oracle_grads(name, sel_idx, wbar)
    B = blocks_from_numpy(Bs[:, sel_idx, :], Bv, w.nocc, sel, "fp64")
    gs, gv, gE = cds.qp_adjoint(B, _dev(w.eps), oms, wbar)
    M = Bs.shape[0]
    gs = gs.cpu().numpy().reshape(len(sel), w.nmo, B.ldk)
    gv = gv.cpu().numpy().reshape(w.nvirt, w.nocc, B.ldk)
    refs = gBs[:, sel_idx, :].transpose(1, 2, 0)
    refv = gBv.transpose(1, 2, 0)
    sc = max(np.abs(refs).max(), np.abs(refv).max())
    assert np.abs(gs[:, :, :M] - refs).max() <= 1e-9 * sc
    assert np.abs(gv[:, :, :M] - refv).max() <= 1e-9 * sc
    assert np.all(gs[:, :, M:] == 0) and np.all(gv[:, :, M:] == 0)
    assert np.abs(gE.cpu().numpy() - ge).max() <= 1e-9 * max(1.0, np.abs(ge).max())


def test_qp_adjoint_fp32_against_fp64_oracle(cds):
    w = workload("c60")
    log("adjoint fp32 c60")
    Bs, Bv = oracle_blocks("c60", 1e-6)
    sel_idx = [list(w.targets).index(w.nocc - 1), list(w.targets).index(w.nocc)]
    wbar = np.array([1.0, 1.0])
    oms, gBs, gBv, ge = _oracle_grads("c60", sel_idx, wbar)
    B = blocks_from_numpy(Bs[:, sel_idx, :], Bv, w.nocc, w.targets[sel_idx], "fp32")
    gs, gv, gE = cds.qp_adjoint(B, _dev(w.eps), oms, wbar)
    M = Bs.shape[0]
    gv = gv.cpu().numpy().reshape(w.nvirt, w.nocc, B.ldk)[:, :, :M]
    gs = gs.cpu().numpy().reshape(len(sel_idx), w.nmo, B.ldk)[:, :, :M]
    refv = gBv.transpose(1, 2, 0)
    refs = gBs[:, sel_idx, :].transpose(1, 2, 0)
    rel = np.linalg.norm(gv - refv) / np.linalg.norm(refv)
    rel_s = np.linalg.norm(gs - refs) / np.linalg.norm(refs)
    log(f"  fp32 Bvo_bar relative error {rel:.2e}, Bsel_bar {rel_s:.2e}")
    assert rel <= 1e-4 and rel_s <= 1e-4
    assert np.abs(gE.cpu().numpy() - ge).max() <= 1e-4 * np.abs(ge).max()


@pytest.mark.parametrize("name", ["plain", "c60"])
def test_transform_adjoint_fp64(cds, name):
    # C-bar = sum_K L^K C (Bbar^K + Bbar^K^T) against the oracle, fed the oracle's own gradient
    # of the HOMO/LUMO energies with respect to the blocks
    w = workload(name)
    log(f"transform adjoint {name}")
    r = oracle_cd(name, 1e-6)
    sel_idx = [list(w.targets).index(w.nocc - 1), list(w.targets).index(w.nocc)]
    wbar = np.array([0.7, -1.3])
    oms, gBs, gBv, ge = _oracle_grads(name, sel_idx, wbar)
    ref = SE.transform_adjoint(r.L, w.C, w.nocc, w.targets, gBs, gBv)
    M = r.M
    ldk = (M + 63) // 64 * 64
    pad = lambda x, rows: np.pad(x.reshape(M, rows).T, ((0, 0), (0, ldk - M)))
    gs = _dev(pad(gBs, len(w.targets) * w.nmo))
    gv = _dev(pad(gBv, w.nvirt * w.nocc))
    Cbar = cds.transform_adjoint(_dev(r.L.T), M, _dev(w.C), w.nocc, w.targets, gs, gv, ldk).cpu().numpy()
    assert np.abs(Cbar - ref).max() <= 1e-10 * np.abs(ref).max()
