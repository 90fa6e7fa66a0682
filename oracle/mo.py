"""ORACLE (test infrastructure): AO->MO transform of the Cholesky vectors and
exact MO-basis ERIs by quarter transforms, FP64 numpy.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.

Paper: Eqs. (factorization), (aomo) and (transformation) of Sec. II.A:
(pq|rs) = sum_K B^K_pq B^K_rs with B^K_pq = sum_{mu,nu} C_mu,p L^K_mu,nu C_nu,q.
The sum over (mu, nu) runs over all ordered AO pairs, so the packed vector
L^K (one entry per mu <= nu) is first unpacked to the symmetric N x N matrix.
"""
from __future__ import annotations

import numpy as np


def unpack(lvec: np.ndarray, nbf: int) -> np.ndarray:
    """Packed pair vector (I = nu(nu+1)/2 + mu) -> symmetric (..., N, N) matrix."""
    # packed order enumerates nu outer, mu = 0..nu inner
    nu_of = np.concatenate([np.full(n + 1, n) for n in range(nbf)])
    mu_of = np.concatenate([np.arange(n + 1) for n in range(nbf)])
    out = np.zeros(lvec.shape[:-1] + (nbf, nbf), dtype=lvec.dtype)
    out[..., mu_of, nu_of] = lvec
    out[..., nu_of, mu_of] = lvec
    return out


def transform_blocks(L: np.ndarray, C: np.ndarray, nocc: int, sel, chunk: int = 64, order: str = "right"):
    """B blocks needed by the self-energy, Eq. (transformation).

    L: (npairs, M) Cholesky vectors (column K = L^K packed).
    Returns Bsel (M, nsel, nmo) = B^K[q, :] for q in sel and
    Bvo (M, nvirt, nocc) = B^K[nocc + a, i].
    order "right" forms C_x^T (L^K C_y), "left" (C_x^T L^K) C_y: the same sums associated the
    other way, which measures how much rounding alone moves a result.
    """
    sel = np.asarray(sel, dtype=np.int64)
    nbf, nmo = C.shape
    M = L.shape[1]
    Cocc, Cvir, Csel = C[:, :nocc], C[:, nocc:], C[:, sel]
    Bsel = np.empty((M, sel.shape[0], nmo))
    Bvo = np.empty((M, nmo - nocc, nocc))
    for k0 in range(0, M, chunk):
        k1 = min(M, k0 + chunk)
        Lk = unpack(np.ascontiguousarray(L[:, k0:k1].T), nbf)        # (kc, N, N)
        if order == "right":
            T_occ = Lk @ Cocc                                         # L^K C_occ
            Bvo[k0:k1] = Cvir.T[None] @ T_occ                         # C_vir^T L^K C_occ
            T_sel = Lk @ Csel                                         # L^K C_sel
            Bsel[k0:k1] = T_sel.transpose(0, 2, 1) @ C[None]          # C_sel^T L^K C
        else:
            Bvo[k0:k1] = (Cvir.T[None] @ Lk) @ Cocc[None]
            Bsel[k0:k1] = (Csel.T[None] @ Lk) @ C[None]
    return Bsel, Bvo


def full_B(L: np.ndarray, C: np.ndarray) -> np.ndarray:
    """All of B^K = C^T L^K C, (M, nmo, nmo); small systems only."""
    nbf = C.shape[0]
    Lk = unpack(np.ascontiguousarray(L.T), nbf)
    return C.T[None] @ Lk @ C[None]


def exact_mo_blocks(V: np.ndarray, C: np.ndarray, nocc: int, sel, chunk: int = 256):
    """Exact (no Cholesky) integrals from the dense ERI supermatrix.

    Returns Z (nsel, nmo, nvirt, nocc) with Z[s, r, a, j] = (q r | a j),
    q = sel[s], a virtual (absolute MO nocc + a), j occupied.  These hold both
    families of Eq. (SE): (q i|a j) for r = i occupied and, using the
    symmetry (q a|i b) = (q a|b i), (q a|i b) = Z[s, nocc + a, b, i].
    Quarter transforms: first the ket pair (lam sig) -> (a j), then the bra.
    """
    sel = np.asarray(sel, dtype=np.int64)
    nbf, nmo = C.shape
    npairs = V.shape[0]
    nvirt = nmo - nocc
    Cocc, Cvir = C[:, :nocc], C[:, nocc:]
    ket = np.empty((npairs, nvirt, nocc))
    for i0 in range(0, npairs, chunk):
        i1 = min(npairs, i0 + chunk)
        W = unpack(V[i0:i1], nbf)                                     # (ic, N, N)
        ket[i0:i1] = Cvir.T[None] @ (W @ Cocc[None])
    ket = ket.reshape(npairs, nvirt * nocc)
    Z = np.empty((sel.shape[0], nmo, nvirt, nocc))
    for s, q in enumerate(sel):
        # bra (q r) over packed AO pairs: coefficient C_mu,q C_nu,r + C_nu,q C_mu,r (mu<nu)
        full = np.outer(C[:, q], np.ones(nmo))[:, None, :] * C[None, :, :]   # [mu, nu, r] = C_mu q C_nu r
        coef = full + full.transpose(1, 0, 2)
        nu_of = np.concatenate([np.full(n + 1, n) for n in range(nbf)])
        mu_of = np.concatenate([np.arange(n + 1) for n in range(nbf)])
        cpk = coef[mu_of, nu_of, :]                                   # (npairs, nmo)
        diag = mu_of == nu_of
        cpk[diag] *= 0.5
        Z[s] = (cpk.T @ ket).reshape(nmo, nvirt, nocc)
    return Z


def Z_from_B(Bsel: np.ndarray, Bvo: np.ndarray) -> np.ndarray:
    """(q r|a j) = sum_K B^K_qr B^K_aj, Eq. (aomo); same layout as exact_mo_blocks."""
    M, nsel, nmo = Bsel.shape
    _, nvirt, nocc = Bvo.shape
    return np.einsum("ksr,kx->srx", Bsel, Bvo.reshape(M, nvirt * nocc),
                     optimize=True).reshape(nsel, nmo, nvirt, nocc)
