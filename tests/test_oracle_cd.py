"""Pins of the oracle's pivoted incomplete Cholesky decomposition.

Sec. II.A of the paper fixes: the error bound D_IJ <= delta (Eq. (stricterr)),
exactness of integrals among pivot pairs, a positive semidefinite residual
(Eq. (error_approx) and the Schwarz bound), the stopping rule on the residual
diagonal, and continuity as delta -> 0.  LAPACK's pivoted Cholesky (dpstrf)
is an independent implementation of the same greedy algorithm.
"""
import numpy as np
import pytest
from scipy.linalg import lapack

from oracle import eri_cd as E
from paper_0912_1459_amd import inputs as I

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def plain():
    w = I.make("plain")
    return w, E.eri_matrix(w.centres, w.alpha)


@pytest.fixture(scope="module")
def cage1():
    # 60 equivalent centres, one exponent: exact symmetric ties on the diagonal
    w = I.make_small_cage(exps=[0.8], nocc=20)
    return w, E.eri_matrix(w.centres, w.alpha)


@pytest.mark.parametrize("delta", [1e-4, 1e-6, 1e-8])
def test_matches_lapack_dpstrf(plain, delta):
    w, V = plain
    r = E.pivoted_cd(delta, V=V, tau=0.0)
    U, perm, rank, info = lapack.dpstrf(V.copy(), tol=delta, lower=0)
    perm = perm - 1
    assert rank == r.M
    assert np.array_equal(perm[:rank], r.piv)
    # first `rank` rows of U are the Cholesky vectors in permuted order
    Ut = np.triu(U[:rank, :])
    mine = r.L[perm, :].T
    # rounding in a residual column (~k eps max V) is divided by sqrt(D_p) of its pivot
    vmax = np.diag(V).max()
    lpp = r.L[r.piv, np.arange(r.M)]
    tol = 64 * EPS * vmax * np.sqrt(np.arange(1, r.M + 1)) / lpp
    assert np.all(np.abs(Ut - mine).max(axis=1) <= tol)


def _check_invariants(V, r, delta):
    R = V - r.L @ r.L.T
    vmax = np.diag(V).max()
    assert r.status == E.STATUS_CONVERGED
    assert r.dmax <= delta
    # Eq. (stricterr): every element of the residual within delta
    assert np.abs(R).max() <= delta * (1 + 1e-9)
    # residual diagonal as tracked equals the recomputed one, pivots exactly zero
    assert np.abs(np.diag(R) - r.D).max() < 1e3 * EPS * vmax
    assert np.all(r.D[r.piv] == 0.0)
    # integrals among pivot pairs are exact to rounding
    assert np.abs(R[np.ix_(r.piv, r.piv)]).max() <= 64 * EPS * vmax
    # lower-trapezoidal: vector k vanishes on earlier pivots, equals sqrt(D_p) on its own
    for k in range(r.M):
        assert np.all(r.L[r.piv[:k], k] == 0.0)
    # residual is positive semidefinite (Eq. (error_approx)) ...
    assert np.linalg.eigvalsh(R).min() >= -1e3 * EPS * vmax
    # ... hence Schwarz: |D_IJ| <= sqrt(D_II D_JJ)
    d = np.sqrt(np.clip(np.diag(R), 0, None))
    assert np.all(np.abs(R) <= np.outer(d, d) + 1e3 * EPS * vmax)


@pytest.mark.parametrize("delta", [1e-4, 1e-6, 1e-8])
def test_invariants_plain(plain, delta):
    w, V = plain
    _check_invariants(V, E.pivoted_cd(delta, V=V), delta)


@pytest.mark.parametrize("delta", [1e-4, 1e-6])
def test_invariants_cage_with_ties(cage1, delta):
    w, V = cage1
    r = E.pivoted_cd(delta, V=V)
    _check_invariants(V, r, delta)
    # symmetric ties: the first pivot is the lowest index among the 60 equal diagonals
    diag = np.diag(V)
    assert r.piv[0] == np.flatnonzero(diag >= diag.max() - E.default_tau(diag.max()))[0]


def test_on_demand_equals_dense(cage1):
    w, V = cage1
    a = E.pivoted_cd(1e-6, V=V)
    b = E.pivoted_cd(1e-6, centres=w.centres, alpha=w.alpha)
    assert np.array_equal(a.piv, b.piv)
    assert np.array_equal(a.L, b.L)


def test_prefix_and_resume(plain):
    w, V = plain
    r4 = E.pivoted_cd(1e-4, V=V)
    r6 = E.pivoted_cd(1e-6, V=V)
    # pivots at a looser threshold are a prefix of those at a tighter one
    assert np.array_equal(r6.piv[: r4.M], r4.piv)
    assert np.array_equal(r6.L[:, : r4.M], r4.L)
    # resuming to the tighter threshold reproduces the direct run bit for bit
    rr = E.pivoted_cd(1e-6, V=V, resume=E.pivoted_cd(1e-4, V=V))
    assert np.array_equal(rr.piv, r6.piv)
    assert np.array_equal(rr.L, r6.L)
    assert np.array_equal(rr.D, r6.D)


def test_cap_then_resume(plain):
    w, V = plain
    full = E.pivoted_cd(1e-6, V=V)
    cap = E.pivoted_cd(1e-6, V=V, max_vec=50)
    assert cap.status == E.STATUS_CAP and cap.M == 50
    assert cap.dmax > 1e-6
    done = E.pivoted_cd(1e-6, V=V, resume=cap, max_vec=full.M + 10)
    assert np.array_equal(done.piv, full.piv) and np.array_equal(done.L, full.L)


def test_continuity_delta_to_zero(plain):
    # Sec. II.A: the approximation improves monotonically and is exact to
    # rounding by delta = 1e-10
    w, V = plain
    errs = []
    for d in [1e-3, 1e-4, 1e-6, 1e-8, 1e-10]:
        r = E.pivoted_cd(d, V=V)
        errs.append(np.abs(V - r.L @ r.L.T).max())
    assert all(errs[i + 1] <= errs[i] for i in range(len(errs) - 1))
    assert errs[-1] <= 1e-10


def test_not_psd_is_reported():
    g = np.random.default_rng(1)
    X = g.standard_normal((30, 30))
    V = X @ X.T
    V[7, 7] -= 0.9 * (V[7, 7])          # no longer PSD: forces a negative residual diagonal
    ev = np.linalg.eigvalsh(V)
    assert ev.min() < 0
    r = E.pivoted_cd(1e-12, V=V)
    assert r.status == E.STATUS_NOT_PSD


def test_full_rank_status():
    g = np.random.default_rng(2)
    X = g.standard_normal((12, 12))
    V = X @ X.T + np.eye(12)
    r = E.pivoted_cd(1e-30, V=V, tau=0.0)
    assert r.status == E.STATUS_FULL_RANK and r.M == 12
    assert np.abs(V - r.L @ r.L.T).max() < 1e-12 * np.abs(V).max()
