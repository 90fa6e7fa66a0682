"""Write stored expected values for the plain workload; calls only oracle/.

Run from the repository root:  python tests/golden/make_golden.py
Output: tests/golden/plain_oracle.json (pivot order, vector counts and
quasi-particle energies / pole strengths of all 40 orbitals at delta=1e-6,
Newton threshold 1e-12), used as a regression pin of the oracle itself.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import eri_cd as E, mo, selfenergy as SE  # noqa: E402
from paper_0912_1459_amd import inputs as I  # noqa: E402


def main():
    w = I.make("plain")
    V = E.eri_matrix(w.centres, w.alpha)
    out = {"workload": "plain", "delta": 1e-6, "conv": 1e-12,
           "source": "oracle/ (ERI closed form, pivoted CD, Eq. (transformation), Eq. (SE), Eq. (iter))"}
    ms = {}
    for d in (1e-4, 1e-6, 1e-8):
        ms[str(d)] = E.pivoted_cd(d, V=V).M
    out["nvec"] = ms
    r = E.pivoted_cd(1e-6, V=V)
    out["pivots"] = [int(p) for p in r.piv]
    Bsel, Bvo = mo.transform_blocks(r.L, w.C, w.nocc, w.targets)
    res = SE.solve_targets(Bsel, Bvo, w.eps, w.nocc, w.targets, conv=1e-12)
    out["omega"] = [float(x.omega) for x in res]
    out["pole"] = [float(x.pole) for x in res]
    out["status"] = [int(x.status) for x in res]
    with open(os.path.join(HERE, "plain_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
