"""Write stored expected values for the large workload; calls only oracle/ and the input draws.

Run from the repository root:  python tests/golden/make_golden_large.py
(about 5-10 minutes on 8 cores, ~10 GB of memory).

Output: tests/golden/large_oracle.json -- for the large workload (truncated-icosahedron
cage, 16 s-Gaussians per centre, N = 960, 461,280 pairs, delta = 1e-4):
  * the pivoted incomplete Cholesky decomposition with on-demand ERI columns (Sec. II.A,
    Eqs. (gs_coulomb), (CD); tie window 1e-10 max V_II): vector count, pivot order, final
    largest residual diagonal and status;
  * the FP64 quasi-particle energies, pole strengths, iteration counts and statuses of the
    16 target orbitals (MOs 112..127) from Eq. (transformation), Eq. (SE) and the Newton
    rule Eq. (iter), threshold 1e-12;
  * each energy's sensitivity to rounding alone: the same decomposition with every residual
    column summed over the earlier vectors in reverse order, and the same transform associated
    the other way ((C^T L^K) C instead of C^T (L^K C)), move Sigma at the converged energy by
    dSigma, hence the energy by P dSigma to first order (Eq. (iter)), and the pole strength by
    P^2 dSigma' (Eq. (ps));
  * |Sigma''| at the converged energy (central difference of Sigma' with step 1e-7 Eh): the pole
    strength returned is P_n at the last iterate w_n, which two evaluations reach only within the
    Newton threshold of each other, so P can differ by P^2 |Sigma''| times that threshold.  The MO coefficients of this workload
    are ill-conditioned (C = S^-1/2 Q, smallest overlap eigenvalue ~2e-7), so two correct FP64
    evaluations of the path can differ by more than 1e-10 Eh; this is their measured spread.
These are the expected values the GPU path is compared with at its full size.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import eri_cd as E, mo, selfenergy as SE  # noqa: E402
from paper_0912_1459_amd import inputs as I  # noqa: E402

CONV = 1e-12
MAX_VEC = 1200      # room for the decomposition (it converges well below this)


def main():
    w = I.make("large")
    t0 = time.time()
    r = E.pivoted_cd(w.delta, centres=w.centres, alpha=w.alpha, max_vec=MAX_VEC)
    t1 = time.time()
    assert r.status == E.STATUS_CONVERGED, r.status
    print(f"CD: M={r.M} dmax={r.dmax:.6e} in {t1 - t0:.1f} s", flush=True)
    Bsel, Bvo = mo.transform_blocks(r.L, w.C, w.nocc, w.targets)
    del r._Lfull
    r2 = E.pivoted_cd(w.delta, centres=w.centres, alpha=w.alpha, max_vec=MAX_VEC, reverse_sums=True)
    assert r2.M == r.M and np.array_equal(r2.piv, r.piv), "rounding changed the pivot order"
    Bsel2, Bvo2 = mo.transform_blocks(r2.L, w.C, w.nocc, w.targets, order="left")
    del r2
    t2 = time.time()
    print(f"transform in {t2 - t1:.1f} s", flush=True)
    res, noise, pnoise, curv = [], [], [], []
    for s, q in enumerate(w.targets):
        x, y = SE.xy_from_B(Bsel[:, s, :], Bvo, w.nocc)
        res.append(SE.newton(x, y, w.eps, w.nocc, int(q), conv=CONV))
        s1, d1 = SE.sigma(x, y, w.eps, w.nocc, res[-1].omega)
        h = 1e-7
        d2p = (SE.sigma(x, y, w.eps, w.nocc, res[-1].omega + h)[1]
               - SE.sigma(x, y, w.eps, w.nocc, res[-1].omega - h)[1]) / (2 * h)
        curv.append(abs(d2p))
        del x, y
        x, y = SE.xy_from_B(Bsel2[:, s, :], Bvo2, w.nocc)
        s2, d2 = SE.sigma(x, y, w.eps, w.nocc, res[-1].omega)
        del x, y
        noise.append(abs(res[-1].pole * (s2 - s1)))
        pnoise.append(abs(res[-1].pole ** 2 * (d2 - d1)))
        print(f"target {int(q)}: omega={res[-1].omega:.12f} P={res[-1].pole:.6f} "
              f"iters={res[-1].iters} status={res[-1].status} rounding spread {noise[-1]:.2e}", flush=True)
    t3 = time.time()
    out = {"workload": "large", "delta": w.delta, "conv": CONV, "max_iter": 50,
           "source": ("oracle/ (on-demand ERI columns, pivoted CD, Eq. (transformation), Eq. (SE), "
                      "Eq. (iter)); written by tests/golden/make_golden_large.py"),
           "nvec": int(r.M), "pivots": [int(p) for p in r.piv], "dmax": float(r.dmax),
           "cd_status": int(r.status), "targets": [int(q) for q in w.targets],
           "omega": [float(x.omega) for x in res], "pole": [float(x.pole) for x in res],
           "iters": [int(x.iters) for x in res], "status": [int(x.status) for x in res],
           "omega_rounding_spread": [float(x) for x in noise],
           "pole_rounding_spread": [float(x) for x in pnoise],
           "sigma_second_derivative": [float(x) for x in curv],
           "seconds": {"cd": round(t1 - t0, 1), "transform": round(t2 - t1, 1),
                       "newton": round(t3 - t2, 1)}}
    with open(os.path.join(HERE, "large_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
