"""Atomic Cholesky decomposition (aCD) on the device (Sec. II.A of the paper).

The aCD basis holds one-centre product densities only, chosen for each unique atom/basis
pair: here the pivots of a pivoted CD (to the same threshold delta) of the one-centre
integrals of one atom's functions alone, shared by all atoms with the same exponents.  The
molecular integral tables are the inner projection of Eq. (int_approx) onto those products,
V ~ V[:, A] V[A, A]^-1 V[A, :], computed as a pivoted CD of the full ERI matrix whose pivots
are restricted to A (every row updated; cds_cholesky_sgauss_subset), run until every product
is used or its residual is below fit_delta (default 1e-12 of the largest one-centre
diagonal: only numerically dependent products are dropped).

Host work is bookkeeping only: grouping functions by centre and mapping an atom's local pair
indices to global ones.  Every decomposition runs in the library's kernels.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import core


def _pair_index(a: int, b: int) -> int:
    a, b = min(a, b), max(a, b)
    return b * (b + 1) // 2 + a


def _pair_functions(I: int) -> tuple[int, int]:
    b = int((np.sqrt(8.0 * I + 1.0) - 1.0) // 2)
    while b * (b + 1) // 2 > I:
        b -= 1
    while (b + 1) * (b + 2) // 2 <= I:
        b += 1
    return I - b * (b + 1) // 2, b


@dataclasses.dataclass
class ACDResult:
    products: np.ndarray        # global pair indices of the aCD basis (sorted)
    per_atom: int               # products of the first atom
    cd: core.CDResult           # restricted decomposition (the integral tables)
    fit_delta: float


def atomic_products(centres: torch.Tensor, alpha: torch.Tensor, delta: float,
                    ctx: core.Context | None = None) -> np.ndarray:
    c_h = centres.detach().cpu().numpy()
    a_h = alpha.detach().cpu().numpy()
    cid = np.unique(c_h, axis=0, return_inverse=True)[1].ravel()
    cache = {}
    out = []
    for c in range(int(cid.max()) + 1):
        f = np.flatnonzero(cid == c)
        key = tuple(a_h[f].tolist())
        if key not in cache:
            idx = torch.as_tensor(f, device=centres.device)
            r = core.cholesky(delta, centres=centres[idx].contiguous(), alpha=alpha[idx].contiguous(), ctx=ctx)
            cache[key] = r.piv[: r.nvec].cpu().numpy()
        for lp in cache[key]:
            a, b = _pair_functions(int(lp))
            out.append(_pair_index(int(f[a]), int(f[b])))
    return np.array(sorted(out), dtype=np.int64)


def acd(centres: torch.Tensor, alpha: torch.Tensor, delta: float, fit_delta: float | None = None,
        ctx: core.Context | None = None) -> ACDResult:
    A = atomic_products(centres, alpha, delta, ctx=ctx)
    nbf = alpha.shape[0]
    np_ = nbf * (nbf + 1) // 2
    dev = alpha.device
    if fit_delta is None:
        # largest diagonal among the products (the largest ERI diagonal is a one-centre one)
        cols = torch.as_tensor(A, device=dev)
        Vc = core.eri_columns(centres, alpha, cols, ctx=ctx)
        vmax = float(Vc[torch.arange(A.size, device=dev), cols].max())
        fit_delta = 1e-12 * vmax
    allowed = torch.zeros(np_, dtype=torch.uint8, device=dev)
    allowed[torch.as_tensor(A, device=dev)] = 1
    cd = core.cholesky(fit_delta, centres=centres, alpha=alpha, allowed=allowed, max_vec=int(A.size), ctx=ctx)
    cid = np.unique(centres.detach().cpu().numpy(), axis=0, return_inverse=True)[1].ravel()
    a0, b0 = zip(*[_pair_functions(int(I)) for I in A])
    per_atom = int(sum(1 for a in a0 if cid[a] == cid[0]))
    return ACDResult(A, per_atom, cd, fit_delta)
