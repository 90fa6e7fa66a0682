"""ORACLE (test infrastructure): spectral-window delta sweep, FP64 numpy/scipy.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.

Results section of the paper (Tables III-IV, Figs. 2-5 and S1): every orbital
whose energy lies in a window is a target; its quasi-particle pole (Newton
from e_q, Eqs. (qpapp)/(iter)) is computed with the integrals of a Cholesky
decomposition at several thresholds delta, and each spectrum is compared
with the one at a small reference threshold ("CD-10"):
  * RMAX = max |w_delta - w_ref|, RMS = sqrt(mean (w_delta - w_ref)^2);
  * a least-squares line w_delta = slope w_ref + intercept with correlation
    coefficient R (the paper finds R = 1.00000, i.e. a uniform shift);
  * the mean and spread of the differences (uniform shift: spread << |mean|).
Only quasi-particle poles enter: converged solves with pole strength P at
least `min_pole` in every spectrum (reading: P >= 0.5 by default).
The thresholds share one decomposition: a pivoted CD to a smaller delta
continues the one to a larger delta (prefix property, Sec. II.A).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy import stats as _st

from . import eri_cd as E
from . import mo
from . import selfenergy as SE


def window(eps: np.ndarray, lo_ev: float, hi_ev: float) -> np.ndarray:
    """Orbitals with lo <= e_q (in eV) <= hi."""
    e = np.asarray(eps) * SE.HARTREE_EV
    return np.nonzero((e >= lo_ev) & (e <= hi_ev))[0].astype(np.int32)


def spectrum_stats(w: np.ndarray, w_ref: np.ndarray) -> dict:
    """RMAX, RMS, mean and spread of w - w_ref; linear regression of w on w_ref."""
    d = np.asarray(w) - np.asarray(w_ref)
    lr = _st.linregress(w_ref, w)
    return {"n": int(d.size), "rmax": float(np.abs(d).max()), "rms": float(np.sqrt(np.mean(d * d))),
            "mean": float(d.mean()), "spread": float(d.std()), "slope": float(lr.slope),
            "intercept": float(lr.intercept), "r": float(lr.rvalue)}


@dataclasses.dataclass
class Spectrum:
    delta: float
    M: int
    omega: np.ndarray
    pole: np.ndarray
    status: np.ndarray


def spectra(centres, alpha, C, eps, nocc, sel, deltas, conv=1e-5, max_iter=50):
    """One spectrum per delta (decreasing order), each CD continuing the previous one."""
    out = []
    r = None
    for d in sorted(deltas, reverse=True):
        r = E.pivoted_cd(d, centres=centres, alpha=alpha, resume=r)
        Bsel, Bvo = mo.transform_blocks(r.L, C, nocc, sel)
        res = SE.solve_targets(Bsel, Bvo, eps, nocc, sel, conv=conv, max_iter=max_iter)
        out.append(Spectrum(d, r.M, np.array([q.omega for q in res]), np.array([q.pole for q in res]),
                            np.array([q.status for q in res])))
    return out


def sweep_stats(specs: list[Spectrum], min_pole: float = 0.5) -> dict:
    """Statistics of every spectrum against the one at the smallest delta."""
    ref = min(specs, key=lambda s: s.delta)
    keep = np.ones(ref.omega.shape[0], dtype=bool)
    for s in specs:
        keep &= (s.status == SE.STATUS_CONVERGED) & (s.pole >= min_pole)
    return {s.delta: spectrum_stats(s.omega[keep], ref.omega[keep]) for s in specs if s is not ref}
