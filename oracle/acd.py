"""ORACLE (test infrastructure): atomic Cholesky decomposition (aCD), FP64.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.

Paper, Sec. II.A: in the aCD the Cholesky basis holds only one-centre product
densities, chosen for each unique atom/basis pair; every ERI is then taken from
the inner projection onto those products, Eq. (int_approx):
    V ~ V[:, A] V[A, A]^-1 V[A, :]          (the V-approximation),
which reproduces the rows and columns of the chosen products exactly and
leaves a residual V - V~ that is positive semidefinite, Eq. (error_approx).
Readings (the paper cites the aCD without restating it):
  * an atom's products are the pivots of a pivoted CD, to the same threshold
    delta, of the one-centre integrals of that atom's functions alone;
    identical atoms (same exponents) share one atomic decomposition;
  * the molecular vectors come from a pivoted CD of the full ERI matrix whose
    pivots are restricted to the chosen products (rows of all pairs updated),
    run until every chosen product is used or its residual falls below
    fit_delta (default 1e-12 max V_II, which drops only numerically dependent
    products).  Its L L^T equals the V-approximation above.
"""
from __future__ import annotations

import numpy as np
from scipy import linalg

from . import eri_cd as E


def centre_ids(centres: np.ndarray) -> np.ndarray:
    """Index of the centre of every basis function (functions on one centre share coordinates)."""
    return np.unique(np.asarray(centres), axis=0, return_inverse=True)[1].ravel()


def pair_index(a: int, b: int) -> int:
    a, b = min(a, b), max(a, b)
    return b * (b + 1) // 2 + a


def pair_functions(I: int) -> tuple[int, int]:
    """Inverse of pair_index: I -> (a, b), a <= b."""
    b = int((np.sqrt(8.0 * I + 1.0) - 1.0) // 2)
    while b * (b + 1) // 2 > I:
        b -= 1
    while (b + 1) * (b + 2) // 2 <= I:
        b += 1
    return I - b * (b + 1) // 2, b


def atomic_products(centres: np.ndarray, alpha: np.ndarray, delta: float, shared: bool = True) -> np.ndarray:
    """Sorted global pair indices of the aCD basis: per atom, the pivots of the pivoted CD of
    its own one-centre integrals.  shared=False decomposes every atom separately."""
    cid = centre_ids(centres)
    cache = {}
    out = []
    for c in range(int(cid.max()) + 1):
        f = np.flatnonzero(cid == c)
        key = tuple(np.asarray(alpha)[f].tolist()) if shared else c
        if key not in cache:
            cache[key] = E.pivoted_cd(delta, centres=np.asarray(centres)[f], alpha=np.asarray(alpha)[f]).piv
        for lp in cache[key]:
            a, b = pair_functions(int(lp))
            out.append(pair_index(int(f[a]), int(f[b])))
    return np.array(sorted(out), dtype=np.int64)


def default_fit_delta(centres, alpha) -> float:
    return 1e-12 * float(E.eri_diagonal(centres, alpha).max())


def acd_vectors(centres, alpha, delta: float, fit_delta: float | None = None) -> tuple[np.ndarray, E.CDResult]:
    """(products A, restricted pivoted CD) of the aCD at threshold delta."""
    A = atomic_products(centres, alpha, delta)
    allowed = np.zeros(np.asarray(alpha).shape[0] * (np.asarray(alpha).shape[0] + 1) // 2, dtype=bool)
    allowed[A] = True
    fd = default_fit_delta(centres, alpha) if fit_delta is None else fit_delta
    return A, E.pivoted_cd(fd, centres=centres, alpha=alpha, allowed=allowed)


def v_approximation(V: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Eq. (int_approx) written out: V[:, A] V[A, A]^-1 V[A, :] (dense V, small systems)."""
    VA = V[:, A]
    return VA @ linalg.solve(V[np.ix_(A, A)], VA.T, assume_a="pos")
