"""ORACLE (test infrastructure): ERIs and pivoted incomplete Cholesky, FP64.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the HIP product path never does.  All arithmetic lives in the
plain-C file cd_oracle.c; this module marshals numpy arrays.

Follows Sec. II.A of the paper: Eq. (integral) for the ERI supermatrix over
product densities, Eqs. (gs_coulomb) and (CD) for the Cholesky vectors, the
threshold rule below Eq. (gs_coulomb), Eq. (stricterr) for the error bound.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from ._clib import lib

STATUS_CONVERGED = 0   # D_max <= delta
STATUS_CAP = 1         # max_vec vectors made first (state resumable)
STATUS_FULL_RANK = 2   # every pair became a pivot
STATUS_NOT_PSD = -4    # a residual diagonal fell below -psd_tol


def _p(a: np.ndarray):
    return a.ctypes.data


def boys_f0(T: float) -> float:
    return lib().orc_boys_f0(float(T))


def eri4(A, a, B, b, C, c, D, d) -> float:
    """(mu nu|lam sig) for four normalized primitive s-Gaussians."""
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (A, B, C, D)]
    return lib().orc_eri4(_p(arrs[0]), float(a), _p(arrs[1]), float(b),
                          _p(arrs[2]), float(c), _p(arrs[3]), float(d))


def pair_index(mu: int, nu: int) -> int:
    if mu > nu:
        mu, nu = nu, mu
    return nu * (nu + 1) // 2 + mu


def pair_list(nbf: int) -> np.ndarray:
    """(npairs, 2) array of (mu, nu) in packed order."""
    out = []
    for nu in range(nbf):
        for mu in range(nu + 1):
            out.append((mu, nu))
    return np.array(out, dtype=np.int64)


def eri_matrix(centres: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """Dense ERI supermatrix V (npairs x npairs), Eq. (integral)."""
    centres = np.ascontiguousarray(centres, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    nbf = alpha.shape[0]
    np_ = nbf * (nbf + 1) // 2
    V = np.empty((np_, np_), dtype=np.float64)
    lib().orc_eri_matrix(nbf, _p(centres), _p(alpha), _p(V))
    return V


def eri_columns(centres: np.ndarray, alpha: np.ndarray, cols) -> np.ndarray:
    """Columns V[:, cols] as a (len(cols), npairs) array."""
    centres = np.ascontiguousarray(centres, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    nbf = alpha.shape[0]
    np_ = nbf * (nbf + 1) // 2
    out = np.empty((cols.shape[0], np_), dtype=np.float64)
    lib().orc_eri_columns(nbf, _p(centres), _p(alpha), cols.shape[0], _p(cols), _p(out))
    return out


def eri_diagonal(centres: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """Diagonal V_II of the ERI supermatrix (the initial residual diagonal)."""
    centres = np.ascontiguousarray(centres, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    nbf = alpha.shape[0]
    np_ = nbf * (nbf + 1) // 2
    out = np.empty(np_, dtype=np.float64)
    lib().orc_eri_diagonal(nbf, _p(centres), _p(alpha), _p(out))
    return out


@dataclasses.dataclass
class CDResult:
    L: np.ndarray        # (npairs, M) Cholesky vectors, column k = vector k
    piv: np.ndarray      # (M,) pivot pairs in order of selection
    D: np.ndarray        # (npairs,) residual diagonal (0 on pivots)
    dmax: float          # final largest non-pivot residual diagonal
    status: int
    _Lfull: np.ndarray = dataclasses.field(repr=False, default=None)

    @property
    def M(self) -> int:
        return self.piv.shape[0]


def default_tau(diag_max: float) -> float:
    """Tie window for the pivot choice: 1e-10 of the largest ERI diagonal (the C code caps
    it at 1% of the current largest residual diagonal)."""
    return 1e-10 * diag_max


def pivoted_cd(delta: float, *, V: np.ndarray | None = None, centres=None, alpha=None,
               tau: float | None = None, max_vec: int | None = None,
               resume: CDResult | None = None, psd_tol: float | None = None,
               allowed: np.ndarray | None = None, reverse_sums: bool = False) -> CDResult:
    """Diagonal-pivoted incomplete Cholesky of the ERI matrix to threshold delta.

    Either a dense V or the basis (centres, alpha) for on-demand columns.
    ``resume`` continues a previous result to a smaller delta or larger cap.
    ``allowed`` (bool per pair) restricts the pivots (all rows are still updated).
    ``reverse_sums`` sums each residual column over the earlier vectors in reverse order (the same
    decomposition up to rounding; used to measure rounding sensitivity).
    """
    if V is not None:
        V = np.ascontiguousarray(V, dtype=np.float64)
        npairs = V.shape[0]
        diag = np.diag(V)
        nbf = 0
        cptr = aptr = None
    else:
        centres = np.ascontiguousarray(centres, dtype=np.float64)
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        nbf = alpha.shape[0]
        npairs = nbf * (nbf + 1) // 2
        diag = None
        cptr, aptr = _p(centres), _p(alpha)
    grow = max_vec is None
    if grow:
        max_vec = max(64, 12 * (nbf if nbf else int(np.sqrt(2 * npairs))))
        if resume is not None:
            max_vec = max(max_vec, 2 * resume.M)
    max_vec = min(max_vec, npairs)
    if resume is not None and resume._Lfull is not None and resume._Lfull.shape[1] >= max_vec:
        Lfull = resume._Lfull
    else:
        Lfull = np.zeros((npairs, max_vec), dtype=np.float64)
    piv = np.zeros(max_vec, dtype=np.int64)
    D = np.zeros(npairs, dtype=np.float64)
    nvec = np.zeros(1, dtype=np.int64)
    dmax = np.zeros(1, dtype=np.float64)
    if resume is not None:
        m0 = resume.M
        if Lfull is not resume._Lfull:
            Lfull[:, :m0] = resume.L
        piv[:m0] = resume.piv
        D[:] = resume.D
        nvec[0] = m0
    if diag is None:
        diag = eri_diagonal(centres, alpha)
    dmx = float(diag.max())
    if tau is None:
        tau = default_tau(dmx)
    if psd_tol is None:
        psd_tol = 1e3 * np.finfo(np.float64).eps * dmx
    allow_u8 = None if allowed is None else np.ascontiguousarray(np.asarray(allowed, dtype=bool), dtype=np.uint8)
    st = lib().orc_pivoted_cd(npairs, _p(V) if V is not None else None, nbf, cptr, aptr,
                              float(delta), float(tau), float(psd_tol), int(max_vec), int(Lfull.shape[1]),
                              _p(Lfull), _p(piv), _p(D), _p(nvec), _p(dmax),
                              _p(allow_u8) if allow_u8 is not None else None, int(bool(reverse_sums)))
    M = int(nvec[0])
    res = CDResult(Lfull[:, :M], piv[:M].copy(), D, float(dmax[0]), int(st), Lfull)
    if grow and st == STATUS_CAP:
        # no cap requested: continue with twice the room
        return pivoted_cd(delta, V=V, centres=centres, alpha=alpha, tau=tau,
                          max_vec=min(2 * max_vec, npairs), resume=res, psd_tol=psd_tol, allowed=allowed,
                          reverse_sums=reverse_sums)
    return res
