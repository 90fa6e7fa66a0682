"""Pins of the atomic-CD oracle (Sec. II.A, Eqs. (int_approx), (error_approx)).

* The restricted pivoted CD reproduces the V-approximation written out with a dense
  solve (two formulations of the same inner projection).
* Rows of the chosen products are reproduced exactly and V - V~ is PSD.
* Identical atoms select the same products whether decomposed once or one by one.
* Unlike the full CD, the aCD error reaches a plateau as delta shrinks.
"""
import numpy as np
import pytest

from oracle import acd as AC
from oracle import eri_cd as E
from paper_0912_1459_amd import inputs as I


@pytest.fixture(scope="module")
def cage():
    w = I.make_small_cage()
    return w, E.eri_matrix(w.centres, w.alpha)


@pytest.fixture(scope="module")
def plain():
    w = I.make_plain()
    return w, E.eri_matrix(w.centres, w.alpha)


@pytest.mark.parametrize("which", ["plain", "cage"])
def test_restricted_cd_equals_v_approximation(which, plain, cage):
    w, V = plain if which == "plain" else cage
    A, r = AC.acd_vectors(w.centres, w.alpha, 1e-6)
    assert np.array_equal(np.sort(r.piv), A)                 # every product used once
    vmax = np.diag(V).max()
    # rows checked: all on the plain workload; the products plus a seeded sample on the cage
    rows = np.arange(V.shape[0])
    if which == "cage":
        g = np.random.default_rng(I.SEED_ROOT + 17)
        rows = np.union1d(A, g.choice(V.shape[0], 400, replace=False))
    L = np.ascontiguousarray(r.L)
    LLt = L[rows] @ L.T
    VA = V[:, A]
    Vt = VA[rows] @ np.linalg.solve(V[np.ix_(A, A)], VA.T)    # Eq. (int_approx) written out
    assert np.abs(LLt - Vt).max() <= 1e-10 * vmax
    # rows of the chosen products are exact; the residual is PSD (eigenvalues on the plain
    # workload, diagonal and Schwarz bound on the cage sample)
    inA = np.isin(rows, A)
    assert np.abs(LLt[inA] - V[rows[inA]]).max() <= 1e-12 * vmax
    R = V[rows] - LLt
    if which == "plain":
        assert np.linalg.eigvalsh(R).min() >= -1e-12 * vmax
    else:
        dall = np.einsum("ij,ij->i", L, L)
        dall = np.diag(V) - dall
        d = dall[rows]
        assert dall.min() >= -1e-12 * vmax
        bound = np.sqrt(np.outer(np.maximum(d, 0), np.maximum(dall, 0)))
        assert np.all(np.abs(R) <= bound + 1e-12 * vmax)


def test_products_are_one_centre_and_shared(cage):
    w, _ = cage
    A = AC.atomic_products(w.centres, w.alpha, 1e-6)
    cid = AC.centre_ids(w.centres)
    for I_ in A:
        a, b = AC.pair_functions(int(I_))
        assert cid[a] == cid[b]
    assert np.array_equal(A, AC.atomic_products(w.centres, w.alpha, 1e-6, shared=False))
    assert A.size % (cid.max() + 1) == 0                      # the same count on every atom


def test_acd_error_plateau(cage):
    # largest residual diagonal D_II (the Eq. (stricterr) bound) over all pairs
    w, V = cage
    errs = []
    for d in (1e-4, 1e-6, 1e-8):
        A, r = AC.acd_vectors(w.centres, w.alpha, d)
        errs.append(r.D.max())
    full = E.pivoted_cd(1e-8, V=V).D.max()
    assert full <= 1e-8 < errs[-1]
    assert errs[-1] > 0.2 * errs[0]                           # no longer improves with delta
