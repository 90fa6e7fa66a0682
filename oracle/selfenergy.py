"""ORACLE (test infrastructure): second-order self-energy, quasi-particle
Newton solve and its gradient, FP64 numpy.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.

Paper, Sec. II.B:
  * Eq. (SE): closed-shell Sigma^(2)_qq(w) =
      sum_{a,i,j} (2(qi|aj) - (qj|ai)) (qi|aj) / (w + e_a - e_i - e_j)
    + sum_{i,a,b} (2(qa|ib) - (qb|ia)) (qa|ib) / (w + e_i - e_a - e_b),
    i, j occupied and a, b virtual, all orbitals active ("fully correlated").
  * Eq. (qpapp): w = e_q + Sigma_qq(w); Eq. (iter): Newton-Raphson update
    w <- w + (e_q + Sigma(w) - w) P; Eq. (ps): P = (1 - dSigma/dw)^-1;
    Eq. (NR): stop when |w_{n+1} - w_n| <= Delta, starting from w_0 = e_q.
The derivative dSigma/dw follows from Eq. (SE) term by term.  The gradient
(not in the paper) differentiates the converged fixed point implicitly:
dw*/dtheta = P * d(e_q + Sigma_qq(w*; theta))/dtheta.

Integral layout used throughout (one target q):
  x[a, i, j] = (q i|a j)      a virtual, i, j occupied
  y[i, a, b] = (q a|i b)      i occupied, a, b virtual
"""
from __future__ import annotations

import dataclasses

import numpy as np

STATUS_CONVERGED = 0
STATUS_MAX_ITER = 1
STATUS_NON_FINITE = 2

HARTREE_EV = 27.211396   # conversion used in the paper's computational details


def xy_from_Z(Zq: np.ndarray, nocc: int):
    """Split Z[r, a, j] = (q r|a j) into x[a,i,j] = (qi|aj) and y[i,a,b] = (qa|ib)."""
    x = np.ascontiguousarray(Zq[:nocc].transpose(1, 0, 2))        # [a, i, j]
    y = np.ascontiguousarray(Zq[nocc:].transpose(2, 0, 1))        # (qa|b i) -> [i, a, b]
    return x, y


def xy_from_B(Bsel_q: np.ndarray, Bvo: np.ndarray, nocc: int):
    """x, y for one target from B^K: (pq|rs) = sum_K B^K_pq B^K_rs, Eq. (aomo).

    Bsel_q: (M, nmo) = B^K[q, :]; Bvo: (M, nvirt, nocc) = B^K[nocc + a, i].
    """
    M, nvirt, _ = Bvo.shape
    Bq_occ, Bq_vir = Bsel_q[:, :nocc], Bsel_q[:, nocc:]
    flat = Bvo.reshape(M, nvirt * nocc)
    x = (Bq_occ.T @ flat).reshape(nocc, nvirt, nocc).transpose(1, 0, 2)   # (q i|a j)
    yt = (Bq_vir.T @ flat).reshape(nvirt, nvirt, nocc)                     # [a, b, i] = (q a|b i)
    y = yt.transpose(2, 0, 1)                                              # (q a|i b) = (q a|b i)
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def _denominators(eps: np.ndarray, nocc: int, omega: float):
    eo, ev = eps[:nocc], eps[nocc:]
    d_x = omega + ev[:, None, None] - eo[None, :, None] - eo[None, None, :]   # [a, i, j]
    d_y = omega + eo[:, None, None] - ev[None, :, None] - ev[None, None, :]   # [i, a, b]
    return d_x, d_y


def numerators(x: np.ndarray, y: np.ndarray):
    """(2(qi|aj) - (qj|ai)) (qi|aj) and (2(qa|ib) - (qb|ia)) (qa|ib), Eq. (SE)."""
    u = (2.0 * x - x.transpose(0, 2, 1)) * x
    w = (2.0 * y - y.transpose(0, 2, 1)) * y
    return u, w


def sigma(x, y, eps, nocc, omega):
    """Sigma_qq(omega) and dSigma/domega, Eq. (SE)."""
    u, w = numerators(x, y)
    d_x, d_y = _denominators(eps, nocc, omega)
    s = (u / d_x).sum() + (w / d_y).sum()
    ds = -(u / d_x ** 2).sum() - (w / d_y ** 2).sum()
    return float(s), float(ds)


def min_abs_denominator(eps, nocc, omega):
    d_x, d_y = _denominators(eps, nocc, omega)
    return min(np.abs(d_x).min(), np.abs(d_y).min())


@dataclasses.dataclass
class QPResult:
    omega: float
    pole: float
    iters: int
    status: int


def newton(x, y, eps, nocc, q, *, omega0=None, conv=1e-5, max_iter=50) -> QPResult:
    """Quasi-particle solve of Eq. (qpapp) by the Newton-Raphson rule Eq. (iter).

    Starts at w_0 = e_q (or omega0); at each step P_n = 1/(1 - Sigma'(w_n)),
    w_{n+1} = w_n + (e_q + Sigma(w_n) - w_n) P_n; stops when |w_{n+1} - w_n| <= conv
    (Eq. (NR)).  Returns w_{n+1} with P_n.  Non-finite values, or a pole hit
    exactly (|d| < 1e-300), end the iteration with STATUS_NON_FINITE.
    """
    w = float(eps[q]) if omega0 is None else float(omega0)
    pole = float("nan")
    for it in range(1, max_iter + 1):
        if min_abs_denominator(eps, nocc, w) < 1e-300:
            return QPResult(w, pole, it, STATUS_NON_FINITE)
        s, ds = sigma(x, y, eps, nocc, w)
        pole = 1.0 / (1.0 - ds)
        w_new = w + (eps[q] + s - w) * pole
        if not np.isfinite(w_new) or not np.isfinite(pole):
            return QPResult(w_new, pole, it, STATUS_NON_FINITE)
        if abs(w_new - w) <= conv:
            return QPResult(w_new, pole, it, STATUS_CONVERGED)
        w = w_new
    return QPResult(w, pole, max_iter, STATUS_MAX_ITER)


def solve_targets(Bsel, Bvo, eps, nocc, sel, **kw):
    """Newton solve for every target; Bsel (M, nsel, nmo), Bvo (M, nvirt, nocc)."""
    out = []
    for s, q in enumerate(sel):
        x, y = xy_from_B(Bsel[:, s, :], Bvo, nocc)
        out.append(newton(x, y, eps, nocc, int(q), **kw))
    return out


def solve_targets_Z(Z, eps, nocc, sel, **kw):
    """Newton solve for every target from exact integrals Z (nsel, nmo, nvirt, nocc)."""
    out = []
    for s, q in enumerate(sel):
        x, y = xy_from_Z(Z[s], nocc)
        out.append(newton(x, y, eps, nocc, int(q), **kw))
    return out


# ----------------------------------------------------------------------------
# gradient of the converged quasi-particle energy (implicit differentiation)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class QPGrad:
    Bsel_q: np.ndarray   # (M, nmo)   d omega* / d B^K[q, r]
    Bvo: np.ndarray      # (M, nvirt, nocc)  d omega* / d B^K[nocc+a, i]
    eps: np.ndarray      # (nmo,)


def qp_gradient(Bsel_q, Bvo, eps, nocc, q, omega) -> QPGrad:
    """Gradient of the fixed point w* of F(w, theta) = e_q + Sigma_qq(w; theta) - w.

    dw*/dtheta = P * dF/dtheta with P = 1/(1 - Sigma'(w*)).
    dSigma/dx[a,i,j] = (4 x[a,i,j] - 2 x[a,j,i]) / d[a,i,j] (x enters its own
    Coulomb-like term and the exchange term of its transpose partner; d is
    symmetric in i, j), likewise for y.  x[a,i,j] = sum_K Bq[K,i] Bvo[K,a,j] and
    y[i,a,b] = sum_K Bq[K,nocc+a] Bvo[K,b,i] carry the chain to B.
    """
    x, y = xy_from_B(Bsel_q, Bvo, nocc)
    d_x, d_y = _denominators(eps, nocc, omega)
    u, w = numerators(x, y)
    _, ds = sigma(x, y, eps, nocc, omega)
    P = 1.0 / (1.0 - ds)
    gx = (4.0 * x - 2.0 * x.transpose(0, 2, 1)) / d_x          # [a, i, j]
    gy = (4.0 * y - 2.0 * y.transpose(0, 2, 1)) / d_y          # [i, a, b]
    M, nvirt, _ = Bvo.shape
    nmo = Bsel_q.shape[1]
    gBq = np.zeros((M, nmo))
    # x[a,i,j] = sum_K Bq[K,i] Bvo[K,a,j]
    gBq[:, :nocc] += np.einsum("aij,kaj->ki", gx, Bvo, optimize=True)
    gBvo = np.einsum("aij,ki->kaj", gx, Bsel_q[:, :nocc], optimize=True)
    # y[i,a,b] = sum_K Bq[K,nocc+a] Bvo[K,b,i]
    gBq[:, nocc:] += np.einsum("iab,kbi->ka", gy, Bvo, optimize=True)
    gBvo += np.einsum("iab,ka->kbi", gy, Bsel_q[:, nocc:], optimize=True)
    # energies: d Sigma/d e_r = -sum U/d^2 * dd/de_r
    eo = np.zeros(nocc)
    ev = np.zeros(nvirt)
    rx = u / d_x ** 2                                           # d = w + e_a - e_i - e_j
    ev -= rx.sum(axis=(1, 2))
    eo += rx.sum(axis=(0, 2)) + rx.sum(axis=(0, 1))
    ry = w / d_y ** 2                                           # d = w + e_i - e_a - e_b
    eo -= ry.sum(axis=(1, 2))
    ev += ry.sum(axis=(0, 2)) + ry.sum(axis=(0, 1))
    geps = np.concatenate([eo, ev])
    geps[q] += 1.0
    return QPGrad(P * gBq, P * gBvo, P * geps)


def transform_adjoint(L, C, nocc, sel, gBsel, gBvo, chunk: int = 64):
    """C-bar = sum_K L^K C (Bbar^K + Bbar^K^T), the adjoint of Eq. (transformation).

    gBsel: (M, nsel, nmo) gradient w.r.t. B^K[sel[s], r]; gBvo: (M, nvirt, nocc)
    gradient w.r.t. B^K[nocc + a, i].  Both are scattered into full nmo x nmo
    matrices Bbar^K first.
    """
    from .mo import unpack
    nbf, nmo = C.shape
    M = L.shape[1]
    sel = np.asarray(sel, dtype=np.int64)
    Cbar = np.zeros_like(C)
    for k0 in range(0, M, chunk):
        k1 = min(M, k0 + chunk)
        Bb = np.zeros((k1 - k0, nmo, nmo))
        for s, q in enumerate(sel):
            Bb[:, q, :] += gBsel[k0:k1, s, :]
        Bb[:, nocc:, :nocc] += gBvo[k0:k1]
        Lk = unpack(np.ascontiguousarray(L[:, k0:k1].T), nbf)
        Cbar += ((Lk @ C[None]) @ (Bb + Bb.transpose(0, 2, 1))).sum(axis=0)
    return Cbar
