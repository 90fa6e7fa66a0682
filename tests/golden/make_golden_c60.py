"""Write stored expected values for the C60-shaped workload; calls only oracle/ and the input draws.

Run from the repository root:  python tests/golden/make_golden_c60.py
(a few minutes on 8 cores, ~15 GB of memory: the dense ERI supermatrix is 6.7 GB).

Output: tests/golden/c60_oracle.json -- for the c60 workload (truncated-icosahedron cage,
4 s-Gaussians per centre, N = 240, 28,920 pairs; the 20 targets HOMO-9 ... LUMO+9):
  * per threshold delta in {1e-4, 1e-6, 1e-8}: the vector count and pivot order of the
    pivoted incomplete Cholesky decomposition with on-demand ERI columns (Sec. II.A), and
    the FP64 quasi-particle energies / pole strengths / statuses from Eq. (transformation),
    Eq. (SE) and the Newton rule Eq. (iter) at threshold 1e-12;
  * the same solves from the exact MO integrals (dense ERI supermatrix, quarter transforms,
    no Cholesky step), so that the error the decomposition alone causes,
    e_delta(q) = |w_q(CD at delta) - w_q(exact)|, can be stated beside any other error
    (the convergence to the exact result as delta -> 0 is the point of Sec. II.A).
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


def main():
    w = I.make("c60")
    out = {"workload": "c60", "conv": CONV, "max_iter": 50, "targets": [int(q) for q in w.targets],
           "source": ("oracle/ (ERI closed form, pivoted CD with on-demand columns, dense-V quarter "
                      "transforms, Eq. (transformation), Eq. (SE), Eq. (iter)); written by "
                      "tests/golden/make_golden_c60.py"),
           "cd": {}}
    for d in (1e-4, 1e-6, 1e-8):
        t0 = time.time()
        r = E.pivoted_cd(d, centres=w.centres, alpha=w.alpha)
        Bsel, Bvo = mo.transform_blocks(r.L, w.C, w.nocc, w.targets)
        res = SE.solve_targets(Bsel, Bvo, w.eps, w.nocc, w.targets, conv=CONV)
        out["cd"][f"{d:g}"] = {"delta": d, "nvec": int(r.M), "pivots": [int(p) for p in r.piv],
                               "dmax": float(r.dmax), "cd_status": int(r.status),
                               "omega": [float(x.omega) for x in res], "pole": [float(x.pole) for x in res],
                               "iters": [int(x.iters) for x in res], "status": [int(x.status) for x in res]}
        print(f"delta {d:g}: M={r.M} in {time.time() - t0:.1f} s", flush=True)
        del r, Bsel, Bvo
    t0 = time.time()
    V = E.eri_matrix(w.centres, w.alpha)
    Z = mo.exact_mo_blocks(V, w.C, w.nocc, w.targets)
    del V
    res = SE.solve_targets_Z(Z, w.eps, w.nocc, w.targets, conv=CONV)
    out["exact"] = {"omega": [float(x.omega) for x in res], "pole": [float(x.pole) for x in res],
                    "iters": [int(x.iters) for x in res], "status": [int(x.status) for x in res]}
    print(f"exact integrals in {time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "c60_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
