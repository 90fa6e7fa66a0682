"""Seeded synthetic workloads for the Cholesky/Sigma(2) quasi-particle path.

This module only *draws inputs*: basis-function centres and exponents, MO
coefficients, orbital energies, target lists, trial energies and finite-
difference directions.  It holds none of the method's arithmetic (no ERI, no
Cholesky step, no transform, no self-energy); both the HIP library and the
CPU oracle consume exactly the arrays produced here.

The paper (Sec. "Computational details") works on C60 with cc-pVDZ/TZ
basis sets and SCF orbitals, which are not available; these synthetic
stand-ins keep its shape: 60 equivalent centres on a truncated icosahedron
with a carbon-carbon edge of 2.7 bohr, all-electron closed-shell occupations,
and thresholds delta = 1e-4 ... 1e-8 (the "low"/"medium" Cholesky ranges of
the Results section).

Workloads
---------
``plain``  N=40 normalized s-Gaussians, 2 per centre on 20 seeded centres in a
           6-bohr cube, exponents log-uniform in [0.1, 10]; 820 pairs;
           delta=1e-6; nocc=10; Newton on all 40 orbitals.
``c60``    60 truncated-icosahedron centres (edge 2.7 bohr), exponents
           {0.15, 0.6, 2.4, 9.6} per centre; N=240, 28,920 pairs; nocc=nvirt=120;
           targets HOMO-9 ... LUMO+9 (MOs 110..129); 8 trial energies per target.
``large``  same cage, 16 exponents per centre 0.05*1000**(k/15); N=960,
           461,280 pairs; delta=1e-4; nocc=120, nvirt=840; targets MOs 112..127.

Orderings: function mu = n_exp*centre + exponent index; the cage centres are
sorted lexicographically by (x, y, z).  The MO coefficients are the Loewdin
orthonormalised basis rotated by a Haar-random orthogonal matrix,
C = S^{-1/2} Q, so that C^T S C = 1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_ROOT = 9121459

# seed streams inside one workload
STREAM_CENTRES = 0
STREAM_EXPONENTS = 1
STREAM_Q = 2
STREAM_EPS_OCC = 3
STREAM_EPS_VIRT = 4
STREAM_DIRECTIONS = 5

WORKLOAD_IDS = {"plain": 0, "c60": 1, "precision": 2, "gradient": 3, "large": 4}


def rng(workload_id: int, stream: int) -> np.random.Generator:
    """Generator for one (workload, stream) pair."""
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, workload_id, stream]))


def truncated_icosahedron(edge: float = 2.7) -> np.ndarray:
    """60 vertices of a truncated icosahedron with the given edge, sorted by (x,y,z).

    Vertices of the unit-edge-2 solid are the even (cyclic) permutations of
    (0, +-1, +-3phi), (+-1, +-(2+phi), +-2phi) and (+-phi, +-2, +-(2phi+1)).
    """
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    bases = [(0.0, 1.0, 3 * phi), (1.0, 2 + phi, 2 * phi), (phi, 2.0, 2 * phi + 1)]
    pts = set()
    for b in bases:
        for sx in (-1, 1):
            for sy in (-1, 1):
                for sz in (-1, 1):
                    v = (sx * b[0], sy * b[1], sz * b[2])
                    for r in range(3):  # cyclic permutations are the even ones
                        w = (v[r % 3], v[(r + 1) % 3], v[(r + 2) % 3])
                        pts.add(tuple(0.0 if x == 0 else x for x in w))
    arr = np.array(sorted(pts), dtype=np.float64)
    assert arr.shape == (60, 3)
    arr *= edge / 2.0
    order = np.lexsort((arr[:, 2], arr[:, 1], arr[:, 0]))
    return np.ascontiguousarray(arr[order])


def overlap_s(centres_bf: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """Overlap matrix of normalized primitive s-Gaussians (used only to build C)."""
    a = alpha[:, None]
    b = alpha[None, :]
    p = a + b
    r2 = ((centres_bf[:, None, :] - centres_bf[None, :, :]) ** 2).sum(-1)
    return (4.0 * a * b / p ** 2) ** 0.75 * np.exp(-a * b * r2 / p)


def haar_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    """Haar-random orthogonal matrix via sign-fixed QR of a Gaussian matrix."""
    z = g.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))[None, :]


@dataclasses.dataclass
class Workload:
    name: str
    wid: int
    centres: np.ndarray      # (nbf, 3) centre of each basis function, bohr
    alpha: np.ndarray        # (nbf,) exponents
    C: np.ndarray            # (nbf, nmo) MO coefficients, column p = MO p
    eps: np.ndarray          # (nmo,) orbital energies, occupied first, each block sorted
    nocc: int
    targets: np.ndarray      # (nsel,) int32 MO indices
    deltas: tuple            # thresholds used with this workload
    delta: float             # the headline threshold
    n_trial: int             # trial energies per target per launch
    s_min: float             # smallest overlap eigenvalue (conditioning of C)

    @property
    def nbf(self) -> int:
        return self.alpha.shape[0]

    @property
    def nmo(self) -> int:
        return self.C.shape[1]

    @property
    def nvirt(self) -> int:
        return self.nmo - self.nocc

    @property
    def npairs(self) -> int:
        return self.nbf * (self.nbf + 1) // 2

    def trial_energies(self) -> np.ndarray:
        """(nsel, T) trial energies: eps_q + 0.01*(t - (T-1)/2) Eh."""
        t = np.arange(self.n_trial, dtype=np.float64) - (self.n_trial - 1) / 2.0
        return self.eps[self.targets][:, None] + 0.01 * t[None, :]

    def directions(self, n: int, size: int, wid: int | None = None) -> np.ndarray:
        """n unit-norm N(0,1) directions of the given size (finite-difference probes)."""
        g = rng(self.wid if wid is None else wid, STREAM_DIRECTIONS)
        d = g.standard_normal((n, size))
        return d / np.linalg.norm(d, axis=1, keepdims=True)


def _orbitals(wid: int, centres_bf: np.ndarray, alpha: np.ndarray, nocc: int):
    nbf = alpha.shape[0]
    S = overlap_s(centres_bf, alpha)
    s, U = np.linalg.eigh(S)
    s_half_inv = (U / np.sqrt(s)[None, :]) @ U.T
    Q = haar_orthogonal(nbf, rng(wid, STREAM_Q))
    C = np.ascontiguousarray(s_half_inv @ Q)
    nvirt = nbf - nocc
    e_occ = np.sort(rng(wid, STREAM_EPS_OCC).uniform(-1.5, -0.3, nocc))
    e_vir = np.sort(rng(wid, STREAM_EPS_VIRT).uniform(0.1, 3.0, nvirt))
    eps = np.concatenate([e_occ, e_vir])
    return C, eps, float(s[0])


def make_plain() -> Workload:
    wid = WORKLOAD_IDS["plain"]
    ncent, nexp = 20, 2
    cent = rng(wid, STREAM_CENTRES).uniform(0.0, 6.0, (ncent, 3))
    lo, hi = math.log(0.1), math.log(10.0)
    expo = np.exp(rng(wid, STREAM_EXPONENTS).uniform(lo, hi, (ncent, nexp)))
    centres_bf = np.repeat(cent, nexp, axis=0)
    alpha = expo.reshape(-1).copy()
    nocc = 10
    C, eps, smin = _orbitals(wid, centres_bf, alpha, nocc)
    return Workload("plain", wid, np.ascontiguousarray(centres_bf), alpha, C, eps, nocc,
                    np.arange(alpha.shape[0], dtype=np.int32), (1e-6,), 1e-6, 1, smin)


def _cage(wid: int, exps: np.ndarray, nocc: int, targets: np.ndarray, deltas, delta, n_trial, name):
    cent = truncated_icosahedron(2.7)
    nexp = exps.shape[0]
    centres_bf = np.ascontiguousarray(np.repeat(cent, nexp, axis=0))
    alpha = np.tile(exps, cent.shape[0]).astype(np.float64)
    C, eps, smin = _orbitals(wid, centres_bf, alpha, nocc)
    return Workload(name, wid, centres_bf, alpha, C, eps, nocc, targets.astype(np.int32),
                    tuple(deltas), delta, n_trial, smin)


def make_c60() -> Workload:
    exps = np.array([0.15, 0.6, 2.4, 9.6])
    return _cage(WORKLOAD_IDS["c60"], exps, 120, np.arange(110, 130), (1e-4, 1e-6, 1e-8), 1e-6, 8, "c60")


def make_large() -> Workload:
    exps = 0.05 * 1000.0 ** (np.arange(16) / 15.0)
    return _cage(WORKLOAD_IDS["large"], exps, 120, np.arange(112, 128), (1e-4,), 1e-4, 8, "large")


def make_small_cage(nexp: int = 2, nocc: int = 30, exps=None) -> Workload:
    """A cut-down cage (60 centres, fewer exponents) for fast multi-tile tests."""
    if exps is None:
        exps = np.array([0.3, 2.0])[:nexp]
    nbf = 60 * len(exps)
    lo = max(nocc - 4, 0)
    tg = np.arange(lo, min(nocc + 4, nbf))
    return _cage(WORKLOAD_IDS["c60"], np.asarray(exps, dtype=np.float64), nocc, tg, (1e-6,), 1e-6, 8,
                 "small_cage")


def make(name: str) -> Workload:
    if name == "plain":
        return make_plain()
    if name in ("c60", "precision", "gradient"):
        return make_c60()
    if name == "large":
        return make_large()
    if name == "small_cage":
        return make_small_cage()
    raise KeyError(name)


def random_factor(n: int, m: int, seed: int, scale: float = 0.05) -> np.ndarray:
    """Seeded (m, n, n) symmetric matrices, a stand-in for transformed vectors B^K."""
    g = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 99, seed]))
    a = g.standard_normal((m, n, n)) * scale
    return 0.5 * (a + a.transpose(0, 2, 1))


def random_energies(nocc: int, nvirt: int, seed: int) -> np.ndarray:
    g = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 98, seed]))
    return np.concatenate([np.sort(g.uniform(-1.5, -0.3, nocc)), np.sort(g.uniform(0.1, 3.0, nvirt))])
