"""Pins of the spectral-window sweep oracle (Results section of the paper).

* The statistics on hand-computed values and on an exact uniform shift (RMAX = RMS =
  |shift|, zero spread, slope 1, R = 1), which is the paper's reading of its regression.
* The window picks exactly the orbitals whose energies (eV) lie inside it.
* On the plain workload the sweep's errors fall with delta and RMAX >= RMS >= |mean|.
"""
import numpy as np
import pytest

from oracle import selfenergy as SE
from oracle import sweep as S
from paper_0912_1459_amd import inputs as I


def test_stats_hand_values():
    st = S.spectrum_stats(np.array([0.0, 1.0, 2.0, 4.0]), np.array([0.0, 1.0, 2.0, 3.0]))
    assert st["n"] == 4
    assert st["rmax"] == 1.0 and abs(st["rms"] - 0.5) < 1e-15 and abs(st["mean"] - 0.25) < 1e-15
    assert abs(st["spread"] - np.sqrt(0.25 - 0.0625)) < 1e-15
    assert abs(st["slope"] - 1.3) < 1e-14 and abs(st["intercept"] + 0.2) < 1e-14
    assert abs(st["r"] - 6.5 / np.sqrt(5.0 * 8.75)) < 1e-14


def test_stats_uniform_shift():
    ref = np.linspace(-0.6, 0.3, 17)
    st = S.spectrum_stats(ref + 2.5e-4, ref)
    assert abs(st["rmax"] - 2.5e-4) < 1e-15 and abs(st["rms"] - 2.5e-4) < 1e-15
    assert st["spread"] < 1e-15 and abs(st["slope"] - 1.0) < 1e-12 and abs(st["r"] - 1.0) < 1e-12


def test_window():
    eps = np.array([-1.0, -0.52, -0.3, 0.05, 0.2, 0.4])
    got = S.window(eps, -14.303, 9.903)           # -0.5256 .. 0.3639 Eh
    assert got.tolist() == [1, 2, 3, 4]


def test_sweep_plain_errors_fall_with_delta():
    w = I.make_plain()
    sel = S.window(w.eps, -14.303, 9.903)
    assert sel.size >= 5
    specs = S.spectra(w.centres, w.alpha, w.C, w.eps, w.nocc, sel, [1e-3, 1e-4, 1e-6, 1e-10], conv=1e-12)
    Ms = [s.M for s in specs]
    assert Ms == sorted(Ms)
    st = S.sweep_stats(specs)
    r = [st[d]["rmax"] for d in (1e-3, 1e-4, 1e-6)]
    assert r[2] < r[1] < r[0]
    for d, v in st.items():
        assert v["rmax"] >= v["rms"] >= abs(v["mean"]) - 1e-18
    assert all(s.status.max() == SE.STATUS_CONVERGED for s in specs)
