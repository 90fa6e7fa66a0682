"""Pins of the MP2 oracle, Eq. (MP2) of Sec. II.A.

* The spin-adapted closed-shell sum equals the textbook spin-orbital MP2
  energy with antisymmetrised integrals, 1/4 sum |<IJ||AB>|^2 / (e_I+e_J-e_A-e_B),
  evaluated by brute force on tiny systems: pins the exchange term, the factor
  2 and every index.
* One occupied and one virtual orbital: E = K^2 / (2 (e_0 - e_1)) with K = (10|10).
* At full Cholesky rank the energy from B equals the one from exact integrals
  (quarter transform of the dense ERI matrix), and it converges as delta shrinks.
"""
import numpy as np
import pytest

from oracle import eri_cd as E
from oracle import mo
from oracle import mp2 as MP
from paper_0912_1459_amd import inputs as I


def _eri_from_B(B):
    return np.einsum("kpq,krs->pqrs", B, B)


def _mp2_spin_orbital(eri, eps, nocc):
    n = eps.shape[0]
    so = [(p, s) for p in range(n) for s in (0, 1)]

    def phys(P, Q, R, S):                # <PQ|RS> = (pr|qs) with spin delta functions
        if P[1] != R[1] or Q[1] != S[1]:
            return 0.0
        return eri[P[0], R[0], Q[0], S[0]]

    occ = [P for P in so if P[0] < nocc]
    vir = [P for P in so if P[0] >= nocc]
    tot = 0.0
    for Iq in occ:
        for J in occ:
            for A in vir:
                for Bq in vir:
                    v = phys(Iq, J, A, Bq) - phys(Iq, J, Bq, A)
                    tot += 0.25 * v * v / (eps[Iq[0]] + eps[J[0]] - eps[A[0]] - eps[Bq[0]])
    return tot


@pytest.mark.parametrize("nocc,nvirt,seed", [(2, 3, 0), (3, 2, 1), (2, 2, 2), (1, 4, 3)])
def test_mp2_matches_spin_orbital_brute_force(nocc, nvirt, seed):
    n = nocc + nvirt
    B = I.random_factor(n, 6, 200 + seed, scale=0.3)
    eps = I.random_energies(nocc, nvirt, 200 + seed)
    ref = _mp2_spin_orbital(_eri_from_B(B), eps, nocc)
    Bvo = np.ascontiguousarray(B[:, nocc:, :nocc])
    got = MP.mp2_from_B(Bvo, eps, nocc)
    assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))
    assert got < 0.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mp2_two_orbitals_closed_form(seed):
    B = I.random_factor(2, 4, 300 + seed, scale=0.3)
    eps = I.random_energies(1, 1, 300 + seed)
    K = float(_eri_from_B(B)[1, 0, 1, 0])
    got = MP.mp2_from_B(np.ascontiguousarray(B[:, 1:, :1]), eps, 1)
    assert abs(got - K * K / (2.0 * (eps[0] - eps[1]))) <= 1e-15 * max(1.0, K * K)


def test_mp2_per_virtual_equals_full_tensor():
    n, nocc = 9, 4
    B = I.random_factor(n, 7, 310, scale=0.2)
    eps = I.random_energies(nocc, n - nocc, 310)
    Bvo = np.ascontiguousarray(B[:, nocc:, :nocc])
    X = np.einsum("kai,kbj->aibj", Bvo, Bvo)
    assert abs(MP.mp2_from_B(Bvo, eps, nocc) - MP.mp2_from_X(X, eps, nocc)) <= 1e-14


@pytest.fixture(scope="module")
def plain():
    w = I.make_plain()
    V = E.eri_matrix(w.centres, w.alpha)
    return w, V


def test_mp2_full_rank_equals_exact_and_converges(plain):
    w, V = plain
    exact = MP.mp2_exact(V, w.C, w.nocc, w.eps)
    assert exact < 0.0
    sel = np.array([0])
    errs = []
    for d in [1e-3, 1e-5, 1e-8, 1e-13]:
        r = E.pivoted_cd(d, V=V)
        _, Bvo = mo.transform_blocks(r.L, w.C, w.nocc, sel)
        errs.append(abs(MP.mp2_from_B(Bvo, w.eps, w.nocc) - exact))
    assert errs[-1] <= 1e-12 * abs(exact)
    assert errs[-1] < errs[2] < errs[0]
