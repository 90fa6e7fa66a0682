"""Python binding of the cdsigma HIP library: argument marshalling only.

Every step of the path runs in the HIP kernels behind the C ABI; PyTorch
supplies device memory and the stream.  Functions mirror the C calls:

  cholesky(...)        pivoted incomplete Cholesky of the ERI supermatrix (Sec. II.A)
  transform(...)       B^K = C^T L^K C blocks, Eq. (transformation)
  sigma2(...)          Sigma_qq and dSigma/dw at trial energies, Eq. (SE)
  qp_solve(...)        Newton solve of Eq. (qpapp) with pole strengths, Eqs. (iter)/(ps)/(NR)
  qp_adjoint(...)      implicit-differentiation adjoint of the solve
  transform_adjoint(...)  C-bar of the transform
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib as A

PREC = {"fp64": A.PREC_FP64, "fp32": A.PREC_FP32, "bf16x3": A.PREC_BF16X3}


class CdsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cdsigma {A.ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _prec(p) -> int:
    if isinstance(p, str):
        return PREC[p]
    return int(p)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """One library context bound to a device and a HIP stream (torch's current one by default)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.lib = A.load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.cds_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise CdsError(rc, "cds_create failed")
        self.h = h

    def check(self, rc: int, ok=(0,)):
        if rc not in ok:
            raise CdsError(rc, self.lib.cds_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.cds_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def stats(self) -> dict:
        s = A.Stats()
        self.check(self.lib.cds_get_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in A.Stats._fields_}

    def reset_stats(self):
        self.check(self.lib.cds_reset_stats(self.h))

    def set_kernel_timing(self, on: bool):
        self.check(self.lib.cds_set_kernel_timing(self.h, int(bool(on))))

    def set_cd_lookahead(self, block_steps: int):
        """Cholesky look-ahead block length (0: plain one-vector-per-step streaming)."""
        self.check(self.lib.cds_set_cd_lookahead(self.h, int(block_steps)))

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t(0)
        self.check(self.lib.cds_workspace_bytes(self.h, ctypes.byref(n)))
        return int(n.value)

    def set_transform_fp64(self, on: bool):
        """FP32/bf16x3 transforms computed in FP64 with only the output rounded (True)."""
        self.check(self.lib.cds_set_transform_fp64(self.h, int(bool(on))))

    def set_target_chunk(self, n: int):
        """At most n targets per contraction launch (0: as many as memory allows)."""
        self.check(self.lib.cds_set_target_chunk(self.h, int(n)))

    def set_cd_speculate(self, on: bool):
        """Speculative look-ahead blocks in the Cholesky decomposition (default on)."""
        self.check(self.lib.cds_set_cd_speculate(self.h, int(bool(on))))

    def set_cd_mailbox(self, on: bool):
        """Speculative blocks report each commit through a word in pinned host memory (True,
        default), or the host reads the device state after every four blocks (False)."""
        self.check(self.lib.cds_set_cd_mailbox(self.h, int(bool(on))))

    def set_cd_large_path(self, on: bool):
        """Cholesky code path of large pair counts (hierarchical pivot search, four tiles per
        step block) at any size (True), or chosen by size (False)."""
        self.check(self.lib.cds_set_cd_large_path(self.h, int(bool(on))))


_default = {}


def context(device: int = 0) -> Context:
    """A per-device context on torch's current stream (recreated if the stream changed)."""
    s = torch.cuda.current_stream(device)
    c = _default.get(device)
    if c is None or c.stream != s:
        c = Context(device, s)
        _default[device] = c
    return c


def npairs(nbf: int) -> int:
    return nbf * (nbf + 1) // 2


def round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


# ---------------------------------------------------------------------------
# ERIs and the pivoted Cholesky decomposition
# ---------------------------------------------------------------------------

def eri_columns(centres: torch.Tensor, alpha: torch.Tensor, cols: torch.Tensor, ctx: Context | None = None):
    ctx = ctx or context(centres.device.index or 0)
    _dev(centres, torch.float64, "centres")
    _dev(alpha, torch.float64, "alpha")
    _dev(cols, torch.int64, "cols")
    nbf = alpha.shape[0]
    out = torch.empty((cols.shape[0], npairs(nbf)), dtype=torch.float64, device=centres.device)
    ctx.check(ctx.lib.cds_eri_columns(ctx.h, nbf, _ptr(centres), _ptr(alpha), cols.shape[0], _ptr(cols),
                                      _ptr(out)))
    return out


@dataclasses.dataclass
class CDResult:
    Lbuf: torch.Tensor      # (max_vec, ldl) vector-major Cholesky vectors
    piv: torch.Tensor       # (max_vec,) int64 pivots
    D: torch.Tensor         # (npairs,) residual diagonal
    nvec: int
    dmax: float
    status: int
    npairs: int

    @property
    def L(self) -> torch.Tensor:
        """(nvec, npairs) view: row k = vector k."""
        return self.Lbuf[: self.nvec, : self.npairs]

    @property
    def ldl(self) -> int:
        return self.Lbuf.shape[1]


def cholesky(delta: float, *, centres: torch.Tensor | None = None, alpha: torch.Tensor | None = None,
             V: torch.Tensor | None = None, tau: float = -1.0, psd_tol: float = -1.0,
             max_vec: int | None = None, resume: CDResult | None = None, ctx: Context | None = None,
             grow: bool | None = None, allowed: torch.Tensor | None = None) -> CDResult:
    """Pivoted incomplete Cholesky to threshold delta, on demand (basis) or of a dense V.

    With max_vec None the buffer starts at 12 vectors per basis function and grows
    (by resuming into a larger buffer) until the decomposition finishes.  `allowed`
    (device uint8 per pair, basis form only) restricts the pivots to the flagged pairs.
    """
    dense = V is not None
    if dense:
        _dev(V, torch.float64, "V")
        np_ = V.shape[0]
        dev = V.device
        nbf = 0
    else:
        _dev(centres, torch.float64, "centres")
        _dev(alpha, torch.float64, "alpha")
        nbf = alpha.shape[0]
        np_ = npairs(nbf)
        dev = alpha.device
    ctx = ctx or context(dev.index or 0)
    if grow is None:
        grow = max_vec is None
    if max_vec is None:
        max_vec = max(64, 12 * (nbf if nbf else int(np.sqrt(2 * np_))))
    max_vec = int(min(max_vec, np_))
    ldl = round_up(np_, 64)
    nvec_in = 0
    if resume is not None:
        nvec_in = resume.nvec
        if resume.Lbuf.shape[0] >= max_vec and resume.ldl == ldl:
            Lbuf, piv = resume.Lbuf, resume.piv
        else:
            Lbuf = torch.zeros((max_vec, ldl), dtype=torch.float64, device=dev)
            piv = torch.zeros(max_vec, dtype=torch.int64, device=dev)
            Lbuf[:nvec_in, : resume.npairs] = resume.Lbuf[:nvec_in, : resume.npairs]
            piv[:nvec_in] = resume.piv[:nvec_in]
        D = resume.D.clone()
    else:
        # every entry the library reads is written first (vectors < nvec, rows < npairs)
        Lbuf = torch.empty((max_vec, ldl), dtype=torch.float64, device=dev)
        piv = torch.zeros(max_vec, dtype=torch.int64, device=dev)
        D = torch.empty(np_, dtype=torch.float64, device=dev)
    nvec = ctypes.c_int64()
    dmax = ctypes.c_double()
    status = ctypes.c_int32()
    if dense:
        rc = ctx.lib.cds_cholesky_dense(ctx.h, np_, _ptr(V), V.stride(0), float(delta), float(tau),
                                        float(psd_tol), max_vec, _ptr(Lbuf), ldl, _ptr(piv), _ptr(D),
                                        nvec_in, ctypes.byref(nvec), ctypes.byref(dmax), ctypes.byref(status))
    elif allowed is not None:
        _dev(allowed, torch.uint8, "allowed")
        if allowed.numel() != np_:
            raise ValueError("allowed needs one flag per pair")
        rc = ctx.lib.cds_cholesky_sgauss_subset(ctx.h, nbf, _ptr(centres), _ptr(alpha), _ptr(allowed),
                                                float(delta), float(tau), float(psd_tol), max_vec, _ptr(Lbuf),
                                                ldl, _ptr(piv), _ptr(D), nvec_in, ctypes.byref(nvec),
                                                ctypes.byref(dmax), ctypes.byref(status))
    else:
        rc = ctx.lib.cds_cholesky_sgauss(ctx.h, nbf, _ptr(centres), _ptr(alpha), float(delta), float(tau),
                                         float(psd_tol), max_vec, _ptr(Lbuf), ldl, _ptr(piv), _ptr(D),
                                         nvec_in, ctypes.byref(nvec), ctypes.byref(dmax), ctypes.byref(status))
    ctx.check(rc, ok=(A.CDS_OK, A.CDS_ECAP, A.CDS_ENOTPSD))
    res = CDResult(Lbuf, piv, D, int(nvec.value), float(dmax.value), int(status.value), np_)
    if grow and res.status == A.CD_CAP and max_vec < np_:
        return cholesky(delta, centres=centres, alpha=alpha, V=V, tau=tau, psd_tol=psd_tol,
                        max_vec=min(2 * max_vec, np_), resume=res, ctx=ctx, grow=True, allowed=allowed)
    return res


# ---------------------------------------------------------------------------
# transform, self-energy, quasi-particle solve
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class BBlocks:
    """B^K blocks in the contraction layout (K contiguous, padded to ldk).

    fp64: double [rows][ldk]; fp32: float [rows][ldk]; bf16x3: bfloat16 hi plane
    [rows][ldk] followed by the lo plane (tensor shape (2, rows, ldk)).
    """
    prec: int
    Bsel: torch.Tensor
    Bvo: torch.Tensor
    nvec: int
    ldk: int
    nmo: int
    nocc: int
    sel: np.ndarray

    @property
    def nsel(self) -> int:
        return int(self.sel.shape[0])

    @property
    def nvirt(self) -> int:
        return self.nmo - self.nocc


def _alloc_B(prec: int, rows: int, ldk: int, dev):
    if prec == A.PREC_FP64:
        return torch.empty((rows, ldk), dtype=torch.float64, device=dev)
    if prec == A.PREC_FP32:
        return torch.empty((rows, ldk), dtype=torch.float32, device=dev)
    return torch.empty((2, rows, ldk), dtype=torch.bfloat16, device=dev)


def transform(L: torch.Tensor, nvec: int, C: torch.Tensor, nocc: int, sel, prec="fp64", *,
              ldk: int | None = None, ctx: Context | None = None) -> BBlocks:
    """B blocks from Cholesky vectors L (rows = vectors, row stride ldl) and C (nbf x nmo)."""
    prec = _prec(prec)
    if not (L.is_cuda and L.dtype == torch.float64 and L.stride(1) == 1):
        raise TypeError("L must be a float64 device tensor with unit column stride")
    _dev(C, torch.float64, "C")
    ctx = ctx or context(L.device.index or 0)
    nbf, nmo = C.shape
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))
    ldk = ldk or round_up(nvec, 64)
    nvirt = nmo - nocc
    Bsel = _alloc_B(prec, sel.shape[0] * nmo, ldk, L.device)
    Bvo = _alloc_B(prec, nvirt * nocc, ldk, L.device)
    ctx.check(ctx.lib.cds_transform(ctx.h, prec, nbf, nvec, _ptr(L), L.stride(0), _ptr(C), nmo, nocc,
                                    sel.shape[0], sel.ctypes.data_as(ctypes.c_void_p), ldk, _ptr(Bsel),
                                    _ptr(Bvo)))
    return BBlocks(prec, Bsel, Bvo, nvec, ldk, nmo, nocc, sel)


def cholesky_transform(delta: float, *, centres: torch.Tensor, alpha: torch.Tensor, C: torch.Tensor, nocc: int,
                       sel, prec="fp64", tau: float = -1.0, psd_tol: float = -1.0, max_vec: int | None = None,
                       ctx: Context | None = None) -> tuple[CDResult, BBlocks]:
    """cholesky() from a fresh start and transform() of its vectors in one library call.

    The transform of the vectors made so far runs on a second stream while the decomposition
    goes on; the results equal the two calls with ldk = round_up(max_vec, 64).  max_vec must
    be large enough (there is no growth): CDS_ECAP raises.  When round_up(nvec, 64) is at most
    half of that ldk, the blocks are re-strided in place to ldk = round_up(nvec, 64)
    (cds_restride_blocks), the row stride the contraction reads fastest.
    """
    prec = _prec(prec)
    _dev(centres, torch.float64, "centres")
    _dev(alpha, torch.float64, "alpha")
    _dev(C, torch.float64, "C")
    nbf = alpha.shape[0]
    np_ = npairs(nbf)
    dev = alpha.device
    ctx = ctx or context(dev.index or 0)
    if max_vec is None:
        max_vec = max(64, 12 * nbf)
    max_vec = int(min(max_vec, np_))
    ldl = round_up(np_, 64)
    Lbuf = torch.empty((max_vec, ldl), dtype=torch.float64, device=dev)
    piv = torch.zeros(max_vec, dtype=torch.int64, device=dev)
    D = torch.empty(np_, dtype=torch.float64, device=dev)
    nmo = C.shape[1]
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))
    ldk = round_up(max_vec, 64)
    Bsel = _alloc_B(prec, sel.shape[0] * nmo, ldk, dev)
    Bvo = _alloc_B(prec, (nmo - nocc) * nocc, ldk, dev)
    nvec = ctypes.c_int64()
    dmax = ctypes.c_double()
    status = ctypes.c_int32()
    rc = ctx.lib.cds_cholesky_transform_sgauss(
        ctx.h, nbf, _ptr(centres), _ptr(alpha), float(delta), float(tau), float(psd_tol), max_vec, _ptr(Lbuf), ldl,
        _ptr(piv), _ptr(D), prec, _ptr(C), nmo, nocc, sel.shape[0], sel.ctypes.data_as(ctypes.c_void_p), ldk,
        _ptr(Bsel), _ptr(Bvo), ctypes.byref(nvec), ctypes.byref(dmax), ctypes.byref(status))
    ctx.check(rc, ok=(A.CDS_OK, A.CDS_ENOTPSD))
    cd = CDResult(Lbuf, piv, D, int(nvec.value), float(dmax.value), int(status.value), np_)
    ldk_new = round_up(max(cd.nvec, 1), 64)
    if 2 * ldk_new <= ldk:
        Bsel = restride_blocks(Bsel, prec, ldk_new, ctx)
        Bvo = restride_blocks(Bvo, prec, ldk_new, ctx)
        ldk = ldk_new
    return cd, BBlocks(prec, Bsel, Bvo, cd.nvec, ldk, nmo, nocc, sel)


def restride_blocks(B: torch.Tensor, prec, ldk_new: int, ctx: Context | None = None) -> torch.Tensor:
    """Rows of B (as _alloc_B lays them out) cut to their first ldk_new entries, in place
    (cds_restride_blocks); returns the view of B's storage in the new layout."""
    prec = _prec(prec)
    ldk = B.shape[-1]
    rows = B.shape[-2]
    if not (B.is_cuda and B.is_contiguous()):
        raise ValueError("B must be a contiguous device tensor")
    ctx = ctx or context(B.device.index or 0)
    ctx.check(ctx.lib.cds_restride_blocks(ctx.h, prec, rows, ldk, ldk_new, _ptr(B)))
    n = B.shape[0] * rows * ldk_new if prec == A.PREC_BF16X3 else rows * ldk_new
    shape = (2, rows, ldk_new) if prec == A.PREC_BF16X3 else (rows, ldk_new)
    return B.view(-1)[:n].view(shape)


def sigma2(B: BBlocks, eps: torch.Tensor, omega: np.ndarray, ctx: Context | None = None):
    """Sigma and dSigma/dw at omega (nsel, T) trial energies; returns numpy (nsel, T) x 2."""
    _dev(eps, torch.float64, "eps")
    ctx = ctx or context(eps.device.index or 0)
    omega = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(B.nsel, -1))
    T = omega.shape[1]
    s = np.zeros_like(omega)
    ds = np.zeros_like(omega)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    ctx.check(ctx.lib.cds_sigma2(ctx.h, B.prec, B.nvec, B.ldk, B.nmo, B.nocc, B.nsel, vp(B.sel), _ptr(B.Bsel),
                                 _ptr(B.Bvo), _ptr(eps), T, vp(omega), vp(s), vp(ds)))
    return s, ds


def mp2_energy(B: BBlocks, eps: torch.Tensor, ctx: Context | None = None) -> float:
    """MP2 correlation energy, Eq. (MP2), from the Bvo block of B (its precision)."""
    _dev(eps, torch.float64, "eps")
    ctx = ctx or context(eps.device.index or 0)
    out = ctypes.c_double(0.0)
    ctx.check(ctx.lib.cds_mp2(ctx.h, B.prec, B.nvec, B.ldk, B.nmo, B.nocc, _ptr(B.Bvo), _ptr(eps),
                              ctypes.byref(out)))
    return float(out.value)


def sigma2_matrix(B: BBlocks, eps: torch.Tensor, omega, ctx: Context | None = None):
    """Sigma_SS and dSigma_SS/dw over the selected orbitals at trial energies omega (T,);
    returns numpy (T, nsel, nsel) x 2."""
    _dev(eps, torch.float64, "eps")
    ctx = ctx or context(eps.device.index or 0)
    om = np.ascontiguousarray(np.atleast_1d(np.asarray(omega, dtype=np.float64)))
    T, n = om.shape[0], B.nsel
    s = np.zeros((T, n, n))
    ds = np.zeros((T, n, n))
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    ctx.check(ctx.lib.cds_sigma2_matrix(ctx.h, B.prec, B.nvec, B.ldk, B.nmo, B.nocc, n, vp(B.sel), _ptr(B.Bsel),
                                        _ptr(B.Bvo), _ptr(eps), T, vp(om), vp(s), vp(ds)))
    return s, ds


@dataclasses.dataclass
class DysonResult:
    omega: np.ndarray
    pole: np.ndarray
    vec: np.ndarray       # (nsel, nsel): row k = eigenvector of root k over the selected orbitals
    iters: np.ndarray
    status: np.ndarray


def dyson_solve(B: BBlocks, eps: torch.Tensor, *, conv: float = 1e-5, max_iter: int = 50,
                ctx: Context | None = None) -> DysonResult:
    """One pole of the Dyson equation over the selected orbitals per orbital (Eq. (DysonSol2))."""
    _dev(eps, torch.float64, "eps")
    ctx = ctx or context(eps.device.index or 0)
    n = B.nsel
    om, pole = np.zeros(n), np.zeros(n)
    vec = np.zeros((n, n))
    iters = np.zeros(n, dtype=np.int32)
    st = np.zeros(n, dtype=np.int32)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    ctx.check(ctx.lib.cds_dyson_solve(ctx.h, B.prec, B.nvec, B.ldk, B.nmo, B.nocc, n, vp(B.sel), _ptr(B.Bsel),
                                      _ptr(B.Bvo), _ptr(eps), float(conv), int(max_iter), vp(om), vp(pole),
                                      vp(vec), vp(iters), vp(st)))
    return DysonResult(om, pole, vec, iters, st)


@dataclasses.dataclass
class QPResult:
    omega: np.ndarray
    pole: np.ndarray
    iters: np.ndarray
    status: np.ndarray


def qp_solve(B: BBlocks, eps: torch.Tensor, *, omega0=None, conv: float = 1e-5, max_iter: int = 50,
             mode: str = "residues", ctx: Context | None = None) -> QPResult:
    _dev(eps, torch.float64, "eps")
    ctx = ctx or context(eps.device.index or 0)
    n = B.nsel
    om = np.zeros(n)
    pole = np.zeros(n)
    iters = np.zeros(n, dtype=np.int32)
    st = np.zeros(n, dtype=np.int32)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    o0 = None if omega0 is None else vp(np.ascontiguousarray(omega0, dtype=np.float64))
    m = {"recompute": A.QP_RECOMPUTE, "residues": A.QP_RESIDUES}[mode]
    ctx.check(ctx.lib.cds_qp_solve(ctx.h, B.prec, B.nvec, B.ldk, B.nmo, B.nocc, n, vp(B.sel), _ptr(B.Bsel),
                                   _ptr(B.Bvo), _ptr(eps), o0, float(conv), int(max_iter), m, vp(om), vp(pole),
                                   vp(iters), vp(st)))
    return QPResult(om, pole, iters, st)


def qp_adjoint(B: BBlocks, eps: torch.Tensor, omega: np.ndarray, omega_bar: np.ndarray,
               ctx: Context | None = None):
    """Returns (Bsel_bar, Bvo_bar, eps_bar) for cotangents omega_bar on the converged energies.

    Bsel_bar/Bvo_bar: float64 for fp64 blocks, float32 (rows, ldk) otherwise.
    """
    _dev(eps, torch.float64, "eps")
    ctx = ctx or context(eps.device.index or 0)
    dt = torch.float64 if B.prec == A.PREC_FP64 else torch.float32
    dev = eps.device
    gs = torch.empty((B.nsel * B.nmo, B.ldk), dtype=dt, device=dev)
    gv = torch.empty((B.nvirt * B.nocc, B.ldk), dtype=dt, device=dev)
    ge = torch.empty(B.nmo, dtype=torch.float64, device=dev)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    ob = np.ascontiguousarray(omega_bar, dtype=np.float64)
    ctx.check(ctx.lib.cds_qp_adjoint(ctx.h, B.prec, B.nvec, B.ldk, B.nmo, B.nocc, B.nsel, vp(B.sel), _ptr(B.Bsel),
                                     _ptr(B.Bvo), _ptr(eps), vp(om), vp(ob), _ptr(gs), _ptr(gv), _ptr(ge)))
    return gs, gv, ge


def transform_adjoint(L: torch.Tensor, nvec: int, C: torch.Tensor, nocc: int, sel, Bsel_bar: torch.Tensor,
                      Bvo_bar: torch.Tensor, ldk: int, ctx: Context | None = None) -> torch.Tensor:
    """C_bar = sum_K L^K C (Bbar^K + Bbar^K^T); Bbar blocks float64 or float32 (rows, ldk)."""
    _dev(C, torch.float64, "C")
    ctx = ctx or context(C.device.index or 0)
    nbf, nmo = C.shape
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))
    prec = A.PREC_FP64 if Bsel_bar.dtype == torch.float64 else A.PREC_FP32
    Cbar = torch.empty_like(C)
    ctx.check(ctx.lib.cds_transform_adjoint(ctx.h, prec, nbf, nvec, _ptr(L), L.stride(0), _ptr(C), nmo, nocc,
                                            sel.shape[0], sel.ctypes.data_as(ctypes.c_void_p), ldk,
                                            _ptr(Bsel_bar.contiguous()), _ptr(Bvo_bar.contiguous()), _ptr(Cbar)))
    return Cbar
