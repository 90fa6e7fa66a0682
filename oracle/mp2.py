"""ORACLE (test infrastructure): MP2 correlation energy, FP64 numpy.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.

Paper, Sec. II.A, Eq. (MP2): the closed-shell MP2 correlation energy
  E = sum_{i,j occ; a,b virt} (2 (ai|bj) - (aj|bi)) (ai|bj) / (e_i + e_j - e_a - e_b),
all orbitals active.  From the Cholesky-transformed blocks, Eq. (aomo) gives
(ai|bj) = sum_K B^K_ai B^K_bj.  The exact branch takes the same sum over
integrals from a quarter transform of the dense ERI matrix (no Cholesky).
"""
from __future__ import annotations

import numpy as np

from . import mo


def mp2_from_X(X: np.ndarray, eps: np.ndarray, nocc: int) -> float:
    """E from X[a, i, b, j] = (ai|bj) (nvirt, nocc, nvirt, nocc), the plain sum."""
    eo, ev = eps[:nocc], eps[nocc:]
    d = (eo[None, :, None, None] + eo[None, None, None, :]
         - ev[:, None, None, None] - ev[None, None, :, None])
    Xx = X.transpose(0, 3, 2, 1)                   # [a, i, b, j] = X[a, j, b, i] = (aj|bi)
    return float(((2.0 * X - Xx) * X / d).sum())


def mp2_from_B(Bvo: np.ndarray, eps: np.ndarray, nocc: int) -> float:
    """E from Bvo (M, nvirt, nocc), Bvo[K, a, i] = B^K_ai: one virtual a at a time,
    (ai|bj) for all i, b, j by one matrix product over K."""
    M, nvirt, _ = Bvo.shape
    flat = Bvo.reshape(M, nvirt * nocc)
    eo, ev = eps[:nocc], eps[nocc:]
    total = 0.0
    for a in range(nvirt):
        Xa = (Bvo[:, a, :].T @ flat).reshape(nocc, nvirt, nocc)   # [i, b, j] = (ai|bj)
        Xx = Xa.transpose(2, 1, 0)                                 # [i, b, j] = (aj|bi)
        d = eo[:, None, None] + eo[None, None, :] - ev[a] - ev[None, :, None]
        total += float(((2.0 * Xa - Xx) * Xa / d).sum())
    return total


def mp2_exact(V: np.ndarray, C: np.ndarray, nocc: int, eps: np.ndarray) -> float:
    """E from exact (ai|bj) of the dense ERI matrix V (no Cholesky)."""
    nmo = C.shape[1]
    virt = np.arange(nocc, nmo)
    Z = mo.exact_mo_blocks(V, C, nocc, virt)        # Z[a, r, b, j] = (a r|b j)
    X = Z[:, :nocc, :, :]                           # r = i occupied
    return mp2_from_X(X, eps, nocc)
