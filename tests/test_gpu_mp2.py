"""GPU parity of the MP2 correlation energy (Eq. (MP2)) against the oracle.

FP64 to rounding (relative 1e-11); FP32 and split-bf16 contractions to the error of their
integrals (FP32: 24-bit products, relative 2e-6; bf16x3: the dropped lo*lo term and the
two-plane split, about 2^-16 per product, relative 5e-5).  Cases: the plain and c60
workloads from oracle blocks, the whole device path (CD -> transform -> MP2) on c60, and
random blocks whose sizes match no tile and force several chunks of virtuals.
"""
import numpy as np
import pytest
import torch

from oracle import mp2 as MP
from paper_0912_1459_amd import inputs as I
from tests._blocks import blocks_from_numpy
from tests._cases import log, oracle_blocks, workload

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 2e-6, "bf16x3": 5e-5}


def _dev(x, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


@pytest.fixture(scope="module")
def cds():
    import paper_0912_1459_amd.core as C
    return C


@pytest.mark.parametrize("name", ["plain", "c60"])
def test_mp2_from_oracle_blocks(cds, name):
    w = workload(name)
    Bs, Bv = oracle_blocks(name, 1e-6)
    ref = MP.mp2_from_B(Bv, w.eps, w.nocc)
    log(f"mp2 {name}: oracle E = {ref:.12f}")
    for prec in ("fp64", "fp32", "bf16x3"):
        B = blocks_from_numpy(Bs, Bv, w.nocc, w.targets, prec)
        got = cds.mp2_energy(B, _dev(w.eps))
        rel = abs(got - ref) / abs(ref)
        log(f"  {prec}: rel {rel:.2e}")
        assert rel <= TOL[prec], prec


def test_mp2_device_path_c60(cds):
    # Cholesky, transform and MP2 all on the device, against the oracle's chain
    w = workload("c60")
    Bs, Bv = oracle_blocks("c60", 1e-6)
    ref = MP.mp2_from_B(Bv, w.eps, w.nocc)
    cd = cds.cholesky(1e-6, centres=_dev(w.centres), alpha=_dev(w.alpha))
    for prec in ("fp64", "bf16x3"):
        B = cds.transform(cd.Lbuf, cd.nvec, _dev(w.C), w.nocc, w.targets, prec)
        got = cds.mp2_energy(B, _dev(w.eps))
        rel = abs(got - ref) / abs(ref)
        log(f"mp2 c60 device path {prec}: rel {rel:.2e}")
        assert rel <= (1e-10 if prec == "fp64" else TOL[prec])


@pytest.mark.parametrize("nocc,nvirt,M", [(37, 53, 91), (5, 3, 7), (1, 17, 64)])
def test_mp2_ragged_random_blocks(cds, nocc, nvirt, M):
    n = nocc + nvirt
    Bfull = I.random_factor(n, M, 400 + nocc, scale=0.15)
    eps = I.random_energies(nocc, nvirt, 400 + nocc)
    Bv = np.ascontiguousarray(Bfull[:, nocc:, :nocc])
    Bs = np.ascontiguousarray(Bfull[:, :1, :])
    ref = MP.mp2_from_B(Bv, eps, nocc)
    for prec in ("fp64", "fp32", "bf16x3"):
        B = blocks_from_numpy(Bs, Bv, nocc, [0], prec)
        got = cds.mp2_energy(B, _dev(eps))
        assert abs(got - ref) <= TOL[prec] * abs(ref), (prec, got, ref)


def test_mp2_deterministic_and_invalid(cds):
    w = workload("plain")
    Bs, Bv = oracle_blocks("plain", 1e-6)
    B = blocks_from_numpy(Bs, Bv, w.nocc, w.targets, "fp32")
    eps = _dev(w.eps)
    e1 = cds.mp2_energy(B, eps)
    e2 = cds.mp2_energy(B, eps)
    assert e1 == e2
    bad = cds.BBlocks(B.prec, B.Bsel, B.Bvo, B.nvec, B.ldk, B.nmo, B.nmo, B.sel)   # nocc == nmo
    with pytest.raises(cds.CdsError):
        cds.mp2_energy(bad, eps)
