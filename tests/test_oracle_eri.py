"""Pins of the oracle's ERI evaluation to mathematics outside itself.

Eq. (integral) of the paper defines (mu nu|lam sig) as a six-dimensional
Coulomb integral; nothing here re-types the closed form the oracle uses.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import eri_cd as E
from paper_0912_1459_amd import inputs as I


@pytest.mark.parametrize("T", [0.0, 1e-14, 1e-9, 1e-4, 0.1, 1.0, 7.5, 30.0, 400.0])
def test_boys_f0_against_quadrature(T):
    # F0(T) = int_0^1 exp(-T t^2) dt, its definition
    ref, _ = integrate.quad(lambda t: math.exp(-T * t * t), 0.0, 1.0, epsabs=0, epsrel=1.2e-14, limit=200)
    assert abs(E.boys_f0(T) - ref) <= 1e-14 * ref


def test_boys_f0_limits():
    assert E.boys_f0(0.0) == 1.0
    T = 2500.0
    assert abs(E.boys_f0(T) - 0.5 * math.sqrt(math.pi / T)) < 1e-15


@pytest.mark.parametrize("a", [0.05, 0.15, 0.6, 2.4, 9.6, 50.0])
def test_self_coulomb_of_one_gaussian(a):
    # (aa|aa) for a normalized s-Gaussian density is 2 sqrt(a/pi): the Coulomb
    # self-energy of a Gaussian charge exp(-2a r^2) (2a/pi)^(3/2).
    A = np.zeros(3)
    assert abs(E.eri4(A, a, A, a, A, a, A, a) - 2.0 * math.sqrt(a / math.pi)) < 1e-14 * a


def _gauss6(alphas, centres, u2):
    """int int prod_k exp(-a_k |r_(k) - A_k|^2) exp(-u2 |r1 - r2|^2) dr1 dr2.

    The exponent is a quadratic form in x = (r1, r2) in R^6, evaluated with
    the general Gaussian integral pi^(n/2) det(A)^(-1/2) exp(b^T A^-1 b - c).
    Functions 0, 1 act on r1 and 2, 3 on r2.
    """
    A = np.zeros((6, 6))
    b = np.zeros(6)
    c = 0.0
    for k in range(4):
        sl = slice(0, 3) if k < 2 else slice(3, 6)
        A[sl, sl] += alphas[k] * np.eye(3)
        b[sl] += alphas[k] * centres[k]
        c += alphas[k] * centres[k] @ centres[k]
    A[0:3, 0:3] += u2 * np.eye(3)
    A[3:6, 3:6] += u2 * np.eye(3)
    A[0:3, 3:6] -= u2 * np.eye(3)
    A[3:6, 0:3] -= u2 * np.eye(3)
    sol = np.linalg.solve(A, b)
    return math.pi ** 3 / math.sqrt(np.linalg.det(A)) * math.exp(b @ sol - c)


def _eri_by_quadrature(cs, al):
    # 1/r = (2/sqrt(pi)) int_0^inf exp(-u^2 r^2) du ; normalization (2a/pi)^(3/4)
    norm = np.prod([(2 * a / math.pi) ** 0.75 for a in al])
    f = lambda u: _gauss6(al, cs, u * u)
    val, _ = integrate.quad(f, 0.0, np.inf, epsabs=0, epsrel=1e-13, limit=400)
    return norm * 2.0 / math.sqrt(math.pi) * val


def test_eri_against_six_dimensional_integral():
    g = np.random.default_rng(7)
    for _ in range(12):
        cs = g.uniform(-2.0, 2.0, (4, 3))
        al = np.exp(g.uniform(math.log(0.1), math.log(10.0), 4))
        if g.uniform() < 0.3:
            cs[1] = cs[0]
        ref = _eri_by_quadrature(cs, al)
        got = E.eri4(cs[0], al[0], cs[1], al[1], cs[2], al[2], cs[3], al[3])
        assert abs(got - ref) <= 1e-11 * abs(ref) + 1e-300


def test_eri_permutational_symmetry():
    g = np.random.default_rng(3)
    for _ in range(20):
        cs = g.uniform(-3, 3, (4, 3))
        al = g.uniform(0.1, 5.0, 4)
        args = [(cs[i], al[i]) for i in range(4)]

        def e(i, j, k, l):
            return E.eri4(*args[i], *args[j], *args[k], *args[l])
        ref = e(0, 1, 2, 3)
        for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]:
            assert abs(e(*perm) - ref) <= 4e-16 * abs(ref) * 8


def test_eri_point_charge_limit():
    # far apart: interaction of two unit-normalised-weight charges -> S_I S_J / R
    a, b = 0.7, 1.3
    A = np.zeros(3)
    R = 60.0
    B = np.array([0.0, 0.0, R])
    # S_I = int chi_a chi_a = 1 for a normalized Gaussian
    got = E.eri4(A, a, A, a, B, b, B, b)
    assert abs(got - 1.0 / R) < 1e-15


def test_eri_matrix_symmetric_psd_plain():
    w = I.make("plain")
    V = E.eri_matrix(w.centres, w.alpha)
    assert np.array_equal(V, V.T)
    ev = np.linalg.eigvalsh(V)
    assert ev.min() >= -64 * np.finfo(float).eps * ev.max()
    assert np.allclose(np.diag(V), E.eri_diagonal(w.centres, w.alpha), rtol=0, atol=0)
    cols = np.array([0, 5, 400, 819])
    assert np.array_equal(E.eri_columns(w.centres, w.alpha, cols), V[:, cols].T)


def test_overlap_metric_of_generated_orbitals():
    for name in ("plain", "c60"):
        w = I.make(name)
        S = I.overlap_s(w.centres, w.alpha)
        assert np.abs(w.C.T @ S @ w.C - np.eye(w.nmo)).max() < 1e-12 / w.s_min
        assert np.all(np.diff(w.eps[: w.nocc]) >= 0) and np.all(np.diff(w.eps[w.nocc:]) >= 0)


def test_cage_geometry():
    c = I.truncated_icosahedron(2.7)
    d = np.linalg.norm(c[:, None] - c[None], axis=-1)
    edges = np.abs(d - 2.7) < 1e-9
    assert edges.sum() // 2 == 90
    assert np.all(edges.sum(axis=1) == 3)
    assert np.allclose(np.linalg.norm(c, axis=1), 6.690650381, atol=1e-8)
    assert d[d > 0].min() > 2.7 - 1e-9
