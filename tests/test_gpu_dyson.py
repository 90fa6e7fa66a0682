"""GPU parity of the non-diagonal self-energy matrix and the Dyson pole search
(Sec. II.B) against the oracle: matrices at trial energies (FP64 relative 1e-10, FP32
2e-5, bf16x3 2e-4 of the largest element), poles, pole strengths, statuses and
eigenvectors of the FP64 search (1e-9), and the one-orbital limit (the quasi-particle
Newton solve).  Orbitals: HOMO-2 ... LUMO+2 of the c60 cage and 12 of the plain workload.
"""
import numpy as np
import pytest
import torch

from oracle import dyson as DY
from tests._blocks import blocks_from_numpy
from tests._cases import log, oracle_blocks, workload

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-10, "fp32": 2e-5, "bf16x3": 2e-4}


def _dev(x, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


@pytest.fixture(scope="module")
def cds():
    import paper_0912_1459_amd.core as C
    return C


def _case(name):
    w = workload(name)
    Bs, Bv = oracle_blocks(name, 1e-6)
    if name == "c60":
        sel = np.arange(w.nocc - 3, w.nocc + 3)
    else:
        sel = np.arange(w.nocc - 6, w.nocc + 6)
    idx = [list(w.targets).index(q) for q in sel]
    return w, np.ascontiguousarray(Bs[:, idx, :]), Bv, sel


@pytest.mark.parametrize("name", ["plain", "c60"])
def test_sigma_matrix(cds, name):
    w, Bs, Bv, sel = _case(name)
    xs, ys = DY.xys_from_B(Bs, Bv, w.nocc)
    om = np.array([w.eps[sel[0]] - 0.05, 0.5 * (w.eps[w.nocc - 1] + w.eps[w.nocc]), w.eps[sel[-1]] + 0.05])
    ref = [DY.sigma_matrix(xs, ys, w.eps, w.nocc, o) for o in om]
    for prec in ("fp64", "fp32", "bf16x3"):
        B = blocks_from_numpy(Bs, Bv, w.nocc, sel, prec)
        s, ds = cds.sigma2_matrix(B, _dev(w.eps), om)
        for t in range(om.size):
            e1 = np.abs(s[t] - ref[t][0]).max() / np.abs(ref[t][0]).max()
            e2 = np.abs(ds[t] - ref[t][1]).max() / np.abs(ref[t][1]).max()
            assert e1 <= TOL[prec] and e2 <= TOL[prec], (prec, t, e1, e2)
        log(f"sigma matrix {name} {prec}: ok")


@pytest.mark.parametrize("name", ["plain", "c60"])
def test_dyson_roots(cds, name):
    w, Bs, Bv, sel = _case(name)
    xs, ys = DY.xys_from_B(Bs, Bv, w.nocc)
    ref = DY.dyson_roots(xs, ys, w.eps, w.nocc, sel, conv=1e-12)
    B = blocks_from_numpy(Bs, Bv, w.nocc, sel, "fp64")
    got = cds.dyson_solve(B, _dev(w.eps), conv=1e-12)
    for k, r in enumerate(ref):
        assert got.status[k] == r.status
        assert abs(got.omega[k] - r.omega) <= 1e-9 and abs(got.pole[k] - r.pole) <= 1e-8
        assert abs(abs(got.vec[k] @ r.vec) - 1.0) <= 1e-8
    log(f"dyson {name}: {sel.size} roots, max iterations {got.iters.max()}")
    # one orbital: the quasi-particle Newton solve of Eq. (iter)
    for k in (0, sel.size - 1):
        B1 = blocks_from_numpy(np.ascontiguousarray(Bs[:, k:k + 1, :]), Bv, w.nocc, sel[k:k + 1], "fp64")
        d1 = cds.dyson_solve(B1, _dev(w.eps), conv=1e-12)
        q1 = cds.qp_solve(B1, _dev(w.eps), conv=1e-12)
        assert abs(d1.omega[0] - q1.omega[0]) <= 1e-11 and abs(d1.pole[0] - q1.pole[0]) <= 1e-10
