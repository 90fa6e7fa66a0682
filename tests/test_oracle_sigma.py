"""Pins of the oracle's transform, self-energy, Newton solve and gradient.

* Eq. (SE) is the closed-shell, spin-adapted form of the textbook
  spin-orbital second-order self-energy with antisymmetrised integrals; a
  brute-force spin-orbital evaluation on tiny systems pins every index,
  exchange term and sign.
* With one occupied and one virtual orbital, Eq. (qpapp) becomes a cubic
  polynomial whose roots numpy finds independently of Newton's method.
* Newton's fixed point equals a bracketing root (brentq) of w - e_q - Sigma(w).
* dSigma/dw, the quasi-particle gradient and the transform adjoint are
  checked against central finite differences.
* At full Cholesky rank, Eq. (aomo)/(transformation) reproduce exact MO
  integrals from a quarter transform of the dense ERI matrix.
"""
import numpy as np
import pytest
from scipy import optimize

from oracle import eri_cd as E
from oracle import mo
from oracle import selfenergy as SE
from paper_0912_1459_amd import inputs as I


def _eri_from_B(B):
    """(pq|rs) = sum_K B^K_pq B^K_rs for full symmetric B (M, n, n)."""
    return np.einsum("kpq,krs->pqrs", B, B)


def _sigma_spin_orbital(eri, eps, nocc, q, omega):
    """Brute-force spin-orbital Sigma^(2)_qq with antisymmetrised integrals.

    Spin orbital P = (p, s): spatial p, spin s.  <PQ|RS> = (pr|qs) d(sP,sR) d(sQ,sS),
    <PQ||RS> = <PQ|RS> - <PQ|SR>.  Target Q0 = (q, alpha).
    Sigma = 1/2 sum_{I occ, A,B virt} |<Q0 I||A B>|^2 / (w + e_I - e_A - e_B)
          + 1/2 sum_{I,J occ, A virt} |<Q0 A||I J>|^2 / (w + e_A - e_I - e_J)
    """
    n = eps.shape[0]
    so = [(p, s) for p in range(n) for s in (0, 1)]

    def phys(P, Q, R, S):
        (p, sp), (qq, sq), (r, sr), (s_, ss) = P, Q, R, S
        if sp != sr or sq != ss:
            return 0.0
        return eri[p, r, qq, s_]

    def anti(P, Q, R, S):
        return phys(P, Q, R, S) - phys(P, Q, S, R)
    occ = [P for P in so if P[0] < nocc]
    vir = [P for P in so if P[0] >= nocc]
    Q0 = (q, 0)
    tot = 0.0
    for Iq in occ:
        for A in vir:
            for Bq in vir:
                v = anti(Q0, Iq, A, Bq)
                tot += 0.5 * v * v / (omega + eps[Iq[0]] - eps[A[0]] - eps[Bq[0]])
    for Iq in occ:
        for J in occ:
            for A in vir:
                v = anti(Q0, A, Iq, J)
                tot += 0.5 * v * v / (omega + eps[A[0]] - eps[Iq[0]] - eps[J[0]])
    return tot


def _blocks_from_full(B, nocc, sel):
    Bsel = B[:, sel, :]
    Bvo = B[:, nocc:, :nocc]
    return np.ascontiguousarray(Bsel), np.ascontiguousarray(Bvo)


@pytest.mark.parametrize("nocc,nvirt,seed", [(2, 3, 0), (3, 2, 1), (2, 2, 2)])
def test_sigma_matches_spin_orbital_brute_force(nocc, nvirt, seed):
    n = nocc + nvirt
    B = I.random_factor(n, 6, seed, scale=0.3)
    eps = I.random_energies(nocc, nvirt, seed)
    eri = _eri_from_B(B)
    sel = np.arange(n)
    Bsel, Bvo = _blocks_from_full(B, nocc, sel)
    for s, q in enumerate(sel):
        x, y = SE.xy_from_B(Bsel[:, s, :], Bvo, nocc)
        for omega in (eps[q], eps[q] + 0.13, -0.05):
            got, _ = SE.sigma(x, y, eps, nocc, omega)
            ref = _sigma_spin_orbital(eri, eps, nocc, q, omega)
            assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))


def test_derivative_against_central_difference():
    n, nocc = 7, 3
    B = I.random_factor(n, 9, 11, scale=0.2)
    eps = I.random_energies(nocc, n - nocc, 11)
    Bsel, Bvo = _blocks_from_full(B, nocc, np.arange(n))
    for q in range(n):
        x, y = SE.xy_from_B(Bsel[:, q, :], Bvo, nocc)
        w0 = eps[q] + 0.02
        h = 1e-5
        fd = (SE.sigma(x, y, eps, nocc, w0 + h)[0] - SE.sigma(x, y, eps, nocc, w0 - h)[0]) / (2 * h)
        _, ds = SE.sigma(x, y, eps, nocc, w0)
        assert abs(ds - fd) <= 1e-7 * max(1.0, abs(ds))
        assert ds < 0.0                   # pole strength in (0, 1]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_two_orbital_cubic(seed):
    # one occupied (0) and one virtual (1) orbital: Eq. (SE) has one pole per
    # family, so Eq. (qpapp) is  (w - e0)(w - p1)(w - p2) - A (w - p2) - B (w - p1) = 0
    B = I.random_factor(2, 4, 100 + seed, scale=0.3)
    eps = I.random_energies(1, 1, 100 + seed)
    eri = _eri_from_B(B)
    for q in (0, 1):
        A_ = eri[q, 0, 1, 0] ** 2          # 2h1p: i = j = 0, a = 1
        B_ = eri[q, 1, 0, 1] ** 2          # 2p1h: i = 0, a = b = 1
        p1 = 2 * eps[0] - eps[1]           # pole of the 2h1p term
        p2 = 2 * eps[1] - eps[0]           # pole of the 2p1h term
        cubic = np.polysub(np.polymul(np.polymul([1, -eps[q]], [1, -p1]), [1, -p2]),
                           np.polyadd(np.polymul([A_], [1, -p2]), np.polymul([B_], [1, -p1])))
        roots = np.roots(cubic)
        roots = np.sort(roots[np.abs(roots.imag) < 1e-12].real)
        Bsel, Bvo = _blocks_from_full(B, 1, np.array([0, 1]))
        x, y = SE.xy_from_B(Bsel[:, q, :], Bvo, 1)
        r = SE.newton(x, y, eps, 1, q, conv=1e-14)
        assert r.status == SE.STATUS_CONVERGED
        assert np.min(np.abs(roots - r.omega)) < 1e-12
        # the quasi-particle root is the one between the two poles
        assert p1 < r.omega < p2
        # pole strength from the analytic derivative of the two-pole Sigma
        dsig = -A_ / (r.omega - p1) ** 2 - B_ / (r.omega - p2) ** 2
        assert abs(r.pole - 1 / (1 - dsig)) < 1e-9
        assert 0.0 < r.pole <= 1.0


@pytest.fixture(scope="module")
def plain_cd():
    w = I.make("plain")
    V = E.eri_matrix(w.centres, w.alpha)
    r = E.pivoted_cd(1e-6, V=V)
    Bsel, Bvo = mo.transform_blocks(r.L, w.C, w.nocc, w.targets)
    return w, V, r, Bsel, Bvo


def test_newton_equals_bracketing_root(plain_cd):
    w, V, r, Bsel, Bvo = plain_cd
    nocc = w.nocc
    eo, ev = w.eps[:nocc], w.eps[nocc:]
    poles = np.sort(np.concatenate([(eo[:, None] + eo[None, :] - ev[:, None, None]).ravel(),
                                    (ev[:, None] + ev[None, :] - eo[:, None, None]).ravel()]))
    for q in (nocc - 2, nocc - 1, nocc, nocc + 1):     # near-gap orbitals
        s = list(w.targets).index(q)
        x, y = SE.xy_from_B(Bsel[:, s, :], Bvo, nocc)
        res = SE.newton(x, y, w.eps, nocc, q, conv=1e-13)
        assert res.status == SE.STATUS_CONVERGED
        lo = poles[poles < res.omega].max()
        hi = poles[poles > res.omega].min()
        f = lambda om: om - w.eps[q] - SE.sigma(x, y, w.eps, nocc, om)[0]
        a, b = lo + 1e-9, hi - 1e-9
        root = optimize.brentq(f, a, b, xtol=1e-15, rtol=4 * np.finfo(float).eps)
        assert abs(root - res.omega) < 1e-12
        assert 0.0 < res.pole <= 1.0


def test_newton_statuses(plain_cd):
    w, V, r, Bsel, Bvo = plain_cd
    q = w.nocc - 1
    x, y = SE.xy_from_B(Bsel[:, q, :], Bvo, w.nocc)
    assert SE.newton(x, y, w.eps, w.nocc, q, max_iter=1, conv=1e-14).status == SE.STATUS_MAX_ITER
    # start exactly on a pole of the 2h1p family: w + e_a - e_i - e_j = 0
    pole = w.eps[0] + w.eps[0] - w.eps[w.nocc]
    assert SE.newton(x, y, w.eps, w.nocc, q, omega0=pole).status == SE.STATUS_NON_FINITE


def test_transform_full_rank_reproduces_exact_integrals(plain_cd):
    w, V, r, _, _ = plain_cd
    full = E.pivoted_cd(1e-13, V=V)
    Bsel, Bvo = mo.transform_blocks(full.L, w.C, w.nocc, w.targets)
    Zc = mo.Z_from_B(Bsel, Bvo)
    Zx = mo.exact_mo_blocks(V, w.C, w.nocc, w.targets)
    cscale = np.abs(w.C).sum(axis=0).max() ** 4
    assert np.abs(Zc - Zx).max() <= 1e-13 * cscale
    # and the MO integrals have the (pq|rs) = (qp|rs) symmetry of Eq. (integral)
    B = mo.full_B(full.L, w.C)
    assert np.abs(B - B.transpose(0, 2, 1)).max() < 1e-12 * np.abs(B).max()


def test_delta_convergence_of_quasiparticle_energies(plain_cd):
    # Sec. II.A continuity and the Results section: the CD error in IPs/EAs
    # shrinks as delta decreases and vanishes in the limit
    w, V, _, _, _ = plain_cd
    sel = np.array([w.nocc - 1, w.nocc])
    Zx = mo.exact_mo_blocks(V, w.C, w.nocc, sel)
    exact = [r.omega for r in SE.solve_targets_Z(Zx, w.eps, w.nocc, sel, conv=1e-13)]
    errs = []
    for d in [1e-3, 1e-4, 1e-6, 1e-8, 1e-10]:
        r = E.pivoted_cd(d, V=V)
        Bsel, Bvo = mo.transform_blocks(r.L, w.C, w.nocc, sel)
        om = [q.omega for q in SE.solve_targets(Bsel, Bvo, w.eps, w.nocc, sel, conv=1e-13)]
        errs.append(max(abs(a - b) for a, b in zip(om, exact)))
    assert errs[-1] < 1e-9
    assert errs[-1] < errs[2] < errs[0]


def _omega(Bsel_q, Bvo, eps, nocc, q):
    x, y = SE.xy_from_B(Bsel_q, Bvo, nocc)
    return SE.newton(x, y, eps, nocc, q, conv=1e-14, max_iter=100).omega


@pytest.mark.parametrize("q", [9, 10])
def test_gradient_against_central_differences(plain_cd, q):
    w, V, r, Bsel, Bvo = plain_cd
    s = list(w.targets).index(q)
    Bq = Bsel[:, s, :].copy()
    w0 = _omega(Bq, Bvo, w.eps, w.nocc, q)
    g = SE.qp_gradient(Bq, Bvo, w.eps, w.nocc, q, w0)
    h = 1e-5
    rng = np.random.default_rng(5)
    for _ in range(6):
        dq = rng.standard_normal(Bq.shape)
        dv = rng.standard_normal(Bvo.shape)
        de = rng.standard_normal(w.eps.shape)
        nrm = np.sqrt((dq ** 2).sum() + (dv ** 2).sum() + (de ** 2).sum())
        dq, dv, de = dq / nrm, dv / nrm, de / nrm
        fp = _omega(Bq + h * dq, Bvo + h * dv, w.eps + h * de, w.nocc, q)
        fm = _omega(Bq - h * dq, Bvo - h * dv, w.eps - h * de, w.nocc, q)
        fd = (fp - fm) / (2 * h)
        an = (g.Bsel_q * dq).sum() + (g.Bvo * dv).sum() + (g.eps * de).sum()
        gn = np.sqrt((g.Bsel_q ** 2).sum() + (g.Bvo ** 2).sum() + (g.eps ** 2).sum())
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-3 * gn)


def test_transform_adjoint_against_central_differences(plain_cd):
    w, V, r, _, _ = plain_cd
    sel = np.array([w.nocc - 1, w.nocc])
    nocc = w.nocc

    def omegas(C):
        Bsel, Bvo = mo.transform_blocks(r.L, C, nocc, sel)
        return np.array([_omega(Bsel[:, s, :], Bvo, w.eps, nocc, q) for s, q in enumerate(sel)])

    Bsel, Bvo = mo.transform_blocks(r.L, w.C, nocc, sel)
    wbar = np.array([0.7, -1.3])           # an arbitrary cotangent on the two energies
    gBsel = np.zeros_like(Bsel)
    gBvo = np.zeros_like(Bvo)
    for s, q in enumerate(sel):
        om = _omega(Bsel[:, s, :], Bvo, w.eps, nocc, q)
        g = SE.qp_gradient(Bsel[:, s, :], Bvo, w.eps, nocc, q, om)
        gBsel[:, s, :] += wbar[s] * g.Bsel_q
        gBvo += wbar[s] * g.Bvo
    Cbar = SE.transform_adjoint(r.L, w.C, nocc, sel, gBsel, gBvo)
    h = 1e-5
    rng = np.random.default_rng(9)
    for _ in range(4):
        d = rng.standard_normal(w.C.shape)
        d /= np.linalg.norm(d)
        fd = (wbar @ omegas(w.C + h * d) - wbar @ omegas(w.C - h * d)) / (2 * h)
        an = (Cbar * d).sum()
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.linalg.norm(Cbar))
