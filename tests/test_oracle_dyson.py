"""Pins of the non-diagonal self-energy and Dyson pole-search oracle (Sec. II.B).

* Sigma_pq against the brute-force spin-orbital second-order self-energy with
  antisymmetrised integrals (all indices, exchange terms, signs); its diagonal equals
  Eq. (SE) and the matrix is symmetric.
* Sigma' against central differences.
* With one selected orbital the Dyson search is the quasi-particle Newton solve.
* At every converged pole det(w - e - Sigma(w)) vanishes and the eigenvalue fixed point
  equals a bracketing root (brentq) of lambda(w) - w.
"""
import numpy as np
import pytest
from scipy import optimize

from oracle import dyson as DY
from oracle import selfenergy as SE
from paper_0912_1459_amd import inputs as I


def _eri_from_B(B):
    return np.einsum("kpq,krs->pqrs", B, B)


def _sigma_so(eri, eps, nocc, p, q, omega):
    n = eps.shape[0]
    so = [(r, s) for r in range(n) for s in (0, 1)]

    def phys(P, Q, R, S):
        if P[1] != R[1] or Q[1] != S[1]:
            return 0.0
        return eri[P[0], R[0], Q[0], S[0]]

    def anti(P, Q, R, S):
        return phys(P, Q, R, S) - phys(P, Q, S, R)
    occ = [P for P in so if P[0] < nocc]
    vir = [P for P in so if P[0] >= nocc]
    P0, Q0 = (p, 0), (q, 0)
    tot = 0.0
    for Iq in occ:
        for A in vir:
            for Bq in vir:
                tot += 0.5 * anti(P0, Iq, A, Bq) * anti(Q0, Iq, A, Bq) / (omega + eps[Iq[0]] - eps[A[0]] - eps[Bq[0]])
    for Iq in occ:
        for J in occ:
            for A in vir:
                tot += 0.5 * anti(P0, A, Iq, J) * anti(Q0, A, Iq, J) / (omega + eps[A[0]] - eps[Iq[0]] - eps[J[0]])
    return tot


def _setup(n, nocc, seed, m=6, scale=0.3):
    B = I.random_factor(n, m, 500 + seed, scale=scale)
    eps = I.random_energies(nocc, n - nocc, 500 + seed)
    sel = np.arange(n)
    xs, ys = DY.xys_from_B(np.ascontiguousarray(B[:, sel, :]), np.ascontiguousarray(B[:, nocc:, :nocc]), nocc)
    return B, eps, sel, xs, ys


@pytest.mark.parametrize("n,nocc,seed", [(5, 2, 0), (4, 3, 1)])
def test_sigma_matrix_matches_spin_orbital(n, nocc, seed):
    B, eps, sel, xs, ys = _setup(n, nocc, seed)
    eri = _eri_from_B(B)
    for omega in (eps[0] - 0.1, 0.05, eps[-1] + 0.2):
        S, _ = DY.sigma_matrix(xs, ys, eps, nocc, omega)
        for p in range(n):
            for q in range(n):
                ref = _sigma_so(eri, eps, nocc, p, q, omega)
                assert abs(S[p, q] - ref) <= 1e-13 * max(1.0, abs(ref))
        assert np.abs(S - S.T).max() <= 1e-13
        for p in range(n):
            assert abs(S[p, p] - SE.sigma(xs[p], ys[p], eps, nocc, omega)[0]) <= 1e-14


def test_sigma_matrix_derivative():
    B, eps, sel, xs, ys = _setup(6, 3, 2, m=8, scale=0.2)
    w0, h = 0.07, 1e-5
    fd = (DY.sigma_matrix(xs, ys, eps, 3, w0 + h)[0] - DY.sigma_matrix(xs, ys, eps, 3, w0 - h)[0]) / (2 * h)
    assert np.abs(DY.sigma_matrix(xs, ys, eps, 3, w0)[1] - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_single_orbital_is_quasiparticle_newton():
    B, eps, sel, xs, ys = _setup(6, 3, 3, m=8, scale=0.2)
    for q in range(6):
        r = DY.dyson_roots([xs[q]], [ys[q]], eps, 3, [q], conv=1e-12)[0]
        ref = SE.newton(xs[q], ys[q], eps, 3, q, conv=1e-12)
        assert r.status == ref.status == SE.STATUS_CONVERGED
        assert abs(r.omega - ref.omega) <= 1e-13 and abs(r.pole - ref.pole) <= 1e-12


def test_converged_poles_solve_the_dyson_equation():
    B, eps, sel, xs, ys = _setup(6, 3, 4, m=8, scale=0.2)
    roots = DY.dyson_roots(xs, ys, eps, 3, sel, conv=1e-12)
    for k, r in enumerate(roots):
        assert r.status == SE.STATUS_CONVERGED and 0.0 < r.pole <= 1.0
        S, _ = DY.sigma_matrix(xs, ys, eps, 3, r.omega)
        M = r.omega * np.eye(6) - np.diag(eps) - S
        assert np.linalg.svd(M, compute_uv=False).min() <= 1e-10 * np.abs(M).max()

        # the tracked eigenvalue crosses w at the root: brentq on lambda_j(w) - w nearby
        def f(w, j=None):
            lam, U = np.linalg.eigh(np.diag(eps) + DY.sigma_matrix(xs, ys, eps, 3, w)[0])
            jj = int(np.argmax(np.abs(U.T @ r.vec)))
            return lam[jj] - w
        a, b = r.omega - 1e-4, r.omega + 1e-4
        assert f(a) * f(b) < 0
        assert abs(optimize.brentq(f, a, b, xtol=1e-15) - r.omega) <= 1e-10
