"""ORACLE (test infrastructure): non-diagonal second-order self-energy and the
Dyson pole search in a space of selected orbitals, FP64 numpy.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.

Paper, Sec. II.B, Eqs. (Dyson), (DysonSol), (DysonSol2): the poles of
G(w) = (w - e - Sigma(w))^-1 solve det(w - e - Sigma(w)) = 0; Eq. (qpapp) is its
diagonal (quasi-particle) approximation.  Here Sigma is kept as a full matrix over
a set S of orbitals (the second-order closed-shell form whose diagonal is Eq. (SE)):
  Sigma_pq(w) = sum_{a,i,j} (pi|aj) (2(qi|aj) - (qj|ai)) / (w + e_a - e_i - e_j)
              + sum_{i,a,b} (pa|ib) (2(qa|ib) - (qb|ia)) / (w + e_i - e_a - e_b).
Readings:
  * a pole of the S-block Dyson equation is a fixed point w = lambda_k(w) of an
    eigenvalue of A(w) = diag(e_S) + Sigma_SS(w); its Newton rule (the analogue of
    Eq. (iter), with the eigenvalue slope u^T Sigma'(w) u by Hellmann-Feynman) is
      w <- w + (lambda_k(w) - w) P,   P = 1 / (1 - u^T Sigma'(w) u),
    and P is the pole strength; with |S| = 1 it is Eq. (iter) exactly;
  * one root per orbital of S: start at w_0 = e_q with u = e_q and follow the
    eigenvector of largest overlap with the previous one; stop as Eq. (NR).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import selfenergy as SE


def sigma_matrix(xs, ys, eps, nocc, omega):
    """Sigma_SS(omega) and its derivative from per-target x[a,i,j] = (qi|aj), y[i,a,b] = (qa|ib):
    Sigma_pq = sum_e x_p[e] (2 x_q[e] - x_q[e~]) / d[e] over both families, e~ the element with
    the two occupied (resp. virtual) indices exchanged; one matrix product per family."""
    d_x, d_y = SE._denominators(eps, nocc, omega)
    X = np.stack([x.ravel() for x in xs])                                   # (n, E_x)
    Xe = np.stack([(2.0 * x - x.transpose(0, 2, 1)).ravel() for x in xs])
    Y = np.stack([y.ravel() for y in ys])
    Ye = np.stack([(2.0 * y - y.transpose(0, 2, 1)).ravel() for y in ys])
    S = (X / d_x.ravel()) @ Xe.T + (Y / d_y.ravel()) @ Ye.T
    dS = -(X / d_x.ravel() ** 2) @ Xe.T - (Y / d_y.ravel() ** 2) @ Ye.T
    return S, dS


def xys_from_B(Bsel, Bvo, nocc):
    """Per-target (x, y) for every selected orbital from the blocks (Bsel (M, nsel, nmo))."""
    out = [SE.xy_from_B(Bsel[:, s, :], Bvo, nocc) for s in range(Bsel.shape[1])]
    return [o[0] for o in out], [o[1] for o in out]


@dataclasses.dataclass
class DysonRoot:
    omega: float
    pole: float
    vec: np.ndarray
    iters: int
    status: int


def dyson_roots(xs, ys, eps, nocc, sel, conv=1e-5, max_iter=50):
    sel = np.asarray(sel)
    eS = eps[sel]
    out = []
    for k in range(sel.size):
        w = float(eS[k])
        u = np.zeros(sel.size)
        u[k] = 1.0
        pole = float("nan")
        res = None
        for it in range(1, max_iter + 1):
            S, dS = sigma_matrix(xs, ys, eps, nocc, w)
            lam, U = np.linalg.eigh(np.diag(eS) + S)
            j = int(np.argmax(np.abs(U.T @ u)))
            v = U[:, j] * np.sign(U[:, j] @ u)
            pole = 1.0 / (1.0 - v @ dS @ v)
            w_new = w + (lam[j] - w) * pole
            u = v
            if not np.isfinite(w_new) or not np.isfinite(pole):
                res = DysonRoot(w_new, pole, u, it, SE.STATUS_NON_FINITE)
                break
            if abs(w_new - w) <= conv:
                res = DysonRoot(w_new, pole, u, it, SE.STATUS_CONVERGED)
                break
            w = w_new
        out.append(res if res is not None else DysonRoot(w, pole, u, max_iter, SE.STATUS_MAX_ITER))
    return out
