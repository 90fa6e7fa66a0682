/*
 * cdsigma — C ABI of the MI355X (gfx950) Cholesky-decomposition Sigma(2)
 * quasi-particle path.
 *
 * Method: Vysotskiy & Cederbaum, "On the Cholesky Decomposition for electron
 * propagator methods: General aspects and application on C60"
 * (arXiv:0912.1459).  The calls follow the paper's problem statement:
 *   ERI supermatrix + threshold delta  ->  Cholesky vectors L^K  (Sec. II.A)
 *   vectors + MO coefficients + orbital energies
 *        ->  quasi-particle energies and pole strengths          (Sec. II.B)
 *
 * Conventions shared by every call
 *   - Every function returns an int status: CDS_OK (0) or a negative CDS_E*
 *     code.  No function throws, aborts or exits.  On CDS_EINVAL nothing has
 *     been written or enqueued.  cds_last_error() returns a text for the last
 *     failure on that context.
 *   - Array arguments are DEVICE pointers to caller-owned memory unless their
 *     name starts with h_ (HOST memory).  The library never frees or keeps
 *     caller memory beyond the call.  It owns internal device workspace,
 *     allocated on first need and grown on demand, released by cds_destroy().
 *   - All device work is enqueued on the stream given to cds_create().  Calls
 *     that return host results (h_* outputs) synchronize that stream before
 *     returning; others return once the work is enqueued.
 *   - Indices are 0-based.  Basis functions are normalized primitive
 *     s-Gaussians chi_mu(r) = (2a/pi)^(3/4) exp(-a |r - A_mu|^2).  The pair
 *     (product density) index is I(mu,nu) = nu(nu+1)/2 + mu for mu <= nu, so
 *     npairs = nbf(nbf+1)/2 (Sec. II.A, product-density set).
 *   - Floating point is IEEE FP64 unless a `prec` argument says otherwise.
 *   - Calls on one context are not thread-safe; use one context per thread.
 */
#ifndef CDSIGMA_H
#define CDSIGMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define CDS_OK        0
#define CDS_EINVAL   -1   /* invalid argument (nothing written)                */
#define CDS_ENOMEM   -2   /* device workspace allocation failed               */
#define CDS_EDEVICE  -3   /* a HIP runtime call failed                        */
#define CDS_ENOTPSD  -4   /* a residual diagonal fell below -psd_tol          */
#define CDS_ECAP     -5   /* max_vec vectors made before D_max <= delta;
                             outputs are a valid, resumable state             */
#define CDS_ESTATE   -6   /* call out of order (e.g. context already broken)  */

/* ---- precision of the transform / contraction --------------------------- */
#define CDS_PREC_FP64   0 /* FP64 operands, FP64 MFMA                         */
#define CDS_PREC_FP32   1 /* FP32 operands, FP32 MFMA, FP32 accumulation      */
#define CDS_PREC_BF16X3 2 /* FP32 operands split x = hi + lo (bf16 each);
                             a*b ~ hi*hi + hi*lo + lo*hi on bf16 MFMA with
                             FP32 accumulation                                */

/* ---- Cholesky termination detail (h_status of the CD calls) ------------- */
#define CDS_CD_CONVERGED 0 /* largest residual diagonal <= delta              */
#define CDS_CD_CAP       1 /* max_vec reached first (return code CDS_ECAP)    */
#define CDS_CD_FULLRANK  2 /* every pair became a pivot                       */
#define CDS_CD_NOTPSD   -4 /* return code CDS_ENOTPSD                         */

/* ---- quasi-particle solve status per target ----------------------------- */
#define CDS_QP_CONVERGED 0 /* |w_{n+1} - w_n| <= conv                         */
#define CDS_QP_MAX_ITER  1 /* max_iter Newton steps without convergence       */
#define CDS_QP_NONFINITE 2 /* a pole was hit or a value became non-finite     */

/* ---- Newton evaluation mode --------------------------------------------- */
#define CDS_QP_RECOMPUTE 0 /* every Newton step recomputes the MO integrals
                              from B by the contraction GEMM (the paper's
                              scheme, Sec. "Computational details")           */
#define CDS_QP_RESIDUES  1 /* one contraction forms the pair-symmetrised pole
                              residues; each Newton step then sums them over
                              the energy denominators (same formula)          */

typedef struct cds_ctx cds_ctx;

/* Per-context accumulated device times (HIP events on the context stream),
 * algorithmic bytes and flops.  Reset by cds_reset_stats(). */
typedef struct cds_stats {
    double t_cd_ms;          /* pivoted Cholesky: the whole decomposition     */
    double t_cd_kernel_ms;   /* Cholesky step-kernel time (with kernel timing on) */
    double t_transform_ms;   /* AO->MO transform                              */
    double t_contract_ms;    /* contraction GEMM launches                     */
    double t_epilogue_ms;    /* denominator sums / residue forming            */
    double t_newton_ms;      /* whole quasi-particle solves                   */
    double t_adjoint_ms;     /* adjoint calls                                 */
    double bytes_cd;         /* algorithmic CD bytes: sum_k 8 npairs k + 64 npairs */
    double flops_contract;   /* 2 M nsel nmo nocc nvirt per contraction       */
    int64_t n_cd_steps;
    int64_t n_contract;
    int64_t n_newton_iter;
    double t_cd_pass_ms;     /* look-ahead pass kernels (with kernel timing on) */
    double bytes_cd_pass;    /* bytes those passes read/write: 8 npairs (k0 + ncol),
                                ncol = 64 candidates, or on the large path (128
                                candidates) the block's speculated steps rounded
                                up to 16 */
    int64_t n_cd_pass;       /* look-ahead passes that did work               */
    int64_t n_cd_miss;       /* steps whose pivot was not a look-ahead candidate */
    double flops_cd_pass;    /* nominal pass flops: 2 npairs k0 ncol          */
    double bytes_cd_step;    /* algorithmic bytes of the step kernels: per step and
                                pair row 8 per vector subtracted + 26 (D, mask,
                                L_k) + 8 (column from R or V) or 40 (pair data) */
    int64_t n_cd_step_launch; /* step-kernel launches (a few past the last step
                                 return at once)                                */
    int64_t n_cd_pass_launch; /* look-ahead pass launches                       */
    double t_mp2_ms;         /* MP2 energies (contraction + reduction)        */
    double flops_mp2;        /* 2 nvec x rows x columns of the MP2 contractions */
    double t_dyson_ms;       /* self-energy matrices and Dyson pole searches  */
    double t_cd_spec_ms;     /* speculative blocks (with kernel timing on)    */
    int64_t n_cd_spec;       /* Cholesky steps committed by speculative blocks */
    int64_t n_cd_spec_block; /* speculative blocks tried                      */
    int64_t n_cd_state_read; /* Cholesky state reads that waited for the stream
                                to drain (speculative path)                   */
    double flops_cd_pass_method;  /* the plain algorithm's products that the
                                     look-ahead passes stand in for: 2 npairs k0
                                     per step kept by a block starting at k0   */
    double flops_cd_block_method; /* the rest of those products, made inside the
                                     speculative blocks: 2 npairs (k - k0) per
                                     step k kept                               */
} cds_stats;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the context. */
int cds_create(int device, void *hip_stream, cds_ctx **out);
/* Release the context and all its workspace (synchronizes its stream). */
void cds_destroy(cds_ctx *ctx);
/* Text of the last error on ctx ("" if none).  Valid until the next call. */
const char *cds_last_error(const cds_ctx *ctx);
int cds_get_stats(const cds_ctx *ctx, cds_stats *out);
int cds_reset_stats(cds_ctx *ctx);
/* 1: time the step kernels (one HIP event pair per run of consecutive step
 * launches) and every look-ahead pass of the Cholesky decomposition
 * (cds_stats.t_cd_kernel_ms, t_cd_pass_ms); 0 (default): off. */
int cds_set_kernel_timing(cds_ctx *ctx, int32_t on);
/* Look-ahead of the pivoted Cholesky: every block_steps steps one pass over L
 * forms the residual columns of up to 64 candidate pivots (the next pivot and
 * the largest residual diagonals; with speculative blocks on problems of more
 * than 256 x 128 pairs, 128 candidates, of which only the speculated steps'
 * columns are formed); steps whose pivot is a candidate then only
 * subtract the vectors made since.  0 disables it (each step streams all of L).
 * With speculative blocks on, it also caps their length (at most 48).
 * Default 48; valid range [0, 256]. */
int cds_set_cd_lookahead(cds_ctx *ctx, int32_t block_steps);
/* Speculative look-ahead blocks of the Cholesky decomposition: 1 (default)
 * = after each look-ahead pass, the next (up to 48) steps restricted to the
 * candidates are decomposed in one small kernel, one launch makes those vectors
 * for every row and checks that no other row would have been chosen, the steps
 * before the first failing one are committed, and the next look-ahead block
 * starts there (a per-step kernel only when nothing could be committed);
 * 0 = a look-ahead pass every block_steps steps and per-step kernels.  The
 * pivots are the same either way. */
int cds_set_cd_speculate(cds_ctx *ctx, int32_t on);
/* How the host follows speculative blocks: 1 (default) = each block's commit
 * writes a word (committed step count, stall flag, block count) to coherent
 * pinned host memory of the context; the host keeps two blocks queued beyond
 * the last commit it has seen and reads the device state only at a stall.
 * 0 = four blocks are queued per read of the device state.  Results are the
 * same either way; 1 falls back to 0 by itself where the word cannot be
 * allocated or does not follow the device state.  cds_stats.n_cd_state_read
 * counts the reads. */
int cds_set_cd_mailbox(cds_ctx *ctx, int32_t on);
/* Cholesky code path by problem size: 0 (default) = automatic; 1 = the path of
 * large pair counts at any size (pivot search through 64 super-tile maxima,
 * then tiles, then rows, instead of one sweep over all 64-row tile records; four
 * tiles per step block instead of one; the speculative block formed once and
 * then read by the row updates, instead of by every workgroup of 128 rows with
 * the rows one step behind it).  Automatic: the sweep up to 1024 tiles, one
 * tile per block up to 1280 tiles, the speculative block in every row
 * workgroup up to 256 of them.  Results are the same either way. */
int cds_set_cd_large_path(cds_ctx *ctx, int32_t on);
/* Working precision of cds_transform for FP32 and BF16X3 outputs: 0 (default)
 * runs its GEMMs in the output precision; 1 runs them in FP64 and rounds only
 * the output blocks (for ill-conditioned MO coefficients, where rounding inside
 * the transform is amplified by about 1 / lambda_min of the overlap matrix). */
int cds_set_transform_fp64(cds_ctx *ctx, int32_t on);
/* Targets per contraction launch in cds_sigma2, cds_qp_solve and
 * cds_qp_adjoint: 0 (default) = as many as the workspace limits allow (all of
 * them on the fused self-energy path); n >= 1 = at most n.  The results do
 * not depend on it (every target's sums are formed in the same order);
 * it exists to bound memory and to exercise the chunked loops.  Valid range
 * [0, 65535]. */
int cds_set_target_chunk(cds_ctx *ctx, int32_t n);
/* Library version string (static). */
const char *cds_version(void);

/*
 * ERI columns, Eq. (integral) of Sec. II.A, closed form for s-Gaussians:
 *   V_IJ = K_I K_J 2 pi^(5/2) / (p q sqrt(p+q)) F0(pq/(p+q) |P-Q|^2),
 *   F0(T) = 1/2 sqrt(pi/T) erf(sqrt T)  (series 1 - T/3 + T^2/10 for T < 1e-12).
 * centres: nbf x 3 (row mu = centre of chi_mu), alpha: nbf exponents.
 * cols: ncol pair indices (device int64).  out: ncol x npairs, column c of V
 * at out + c*npairs.  Errors: EINVAL for nbf < 1, ncol < 0, NULL pointers.
 */
int cds_eri_columns(cds_ctx *ctx, int32_t nbf, const double *centres, const double *alpha,
                    int64_t ncol, const int64_t *cols, double *out);

/*
 * Diagonal-pivoted incomplete Cholesky decomposition of the ERI supermatrix
 * to threshold delta (Sec. II.A: Eqs. (gs_coulomb), (CD), (stricterr)).
 * Columns are evaluated on demand from the basis (no npairs^2 storage).
 *
 * Each step picks the pivot p = the lowest pair index I (not yet a pivot)
 * with D_I >= D_max - min(tau, D_max / 100), where D is the residual diagonal
 * and D_max its largest non-pivot entry (a tie window: symmetry-equivalent
 * pairs have equal diagonals up to rounding); forms c = V[:,p] - L[:, :k] L[p, :k]^T;
 * L[:,k] = c / sqrt(D_p) with L[p,k] = sqrt(D_p) and exactly 0 on earlier
 * pivots; D -= L[:,k]^2; D_p = 0.  It stops when D_max <= delta, after
 * max_vec vectors, or when every pair is a pivot.
 *
 * L: vector-major, vector k at L + k*ldl, entries 0..npairs-1 (ldl >= npairs);
 *    the library may read (never write) entries npairs..ldl-1 of each vector.
 * piv: int64[max_vec] pivot pair of each vector.  D: double[npairs] residual
 *    diagonal, 0 on pivots.
 * tau < 0 selects the default 1e-10 * max_I V_II.  psd_tol < 0 selects
 *    1e3 * 2^-52 * max_I V_II; a non-pivot D_I < -psd_tol stops with ENOTPSD.
 * nvec_in: 0 starts afresh; > 0 resumes from vectors 0..nvec_in-1, their
 *    pivots and D exactly as an earlier call left them (to a smaller delta or
 *    larger max_vec).  Resumed and direct runs make the same pivots; with the
 *    look-ahead off (cds_set_cd_lookahead(ctx, 0)) they are bitwise identical,
 *    with it on the vectors agree to rounding (different summation grouping).
 *
 * The residual columns are formed with a look-ahead over candidate pivots
 * (see cds_set_cd_lookahead); the pivot rule and the results are those of the
 * plain one-vector-per-step algorithm above.
 * h_nvec: vectors made in total; h_dmax: final D_max; h_status: CDS_CD_*.
 * Returns CDS_OK (converged or full rank), CDS_ECAP, CDS_ENOTPSD, or an error.
 */
int cds_cholesky_sgauss(cds_ctx *ctx, int32_t nbf, const double *centres, const double *alpha,
                        double delta, double tau, double psd_tol, int64_t max_vec,
                        double *L, int64_t ldl, int64_t *piv, double *D, int64_t nvec_in,
                        int64_t *h_nvec, double *h_dmax, int32_t *h_status);

/* Same decomposition of a dense symmetric npairs x npairs matrix V (column I
 * at V + I*ldv).  Used to separate ERI rounding from decomposition rounding. */
int cds_cholesky_dense(cds_ctx *ctx, int64_t npairs, const double *V, int64_t ldv,
                       double delta, double tau, double psd_tol, int64_t max_vec,
                       double *L, int64_t ldl, int64_t *piv, double *D, int64_t nvec_in,
                       int64_t *h_nvec, double *h_dmax, int32_t *h_status);

/* Same decomposition with the pivots restricted to the pairs I with
 * allowed[I] != 0 (device uint8[npairs]); every other non-pivot row is still
 * updated.  The vectors then span the inner projection of Eq. (int_approx) onto
 * the allowed products: L L^T = V[:, A] V[A, A]^-1 V[A, :] once every allowed
 * product is a pivot (status FULLRANK) or the allowed residuals are <= delta.
 * This is the molecular step of the atomic CD (Sec. II.A), whose allowed set
 * holds the one-centre products chosen atom by atom.  D_max, the tie window
 * and the termination rules range over allowed non-pivots; the PSD check over
 * all non-pivots.  Other arguments, layouts and errors as cds_cholesky_sgauss. */
int cds_cholesky_sgauss_subset(cds_ctx *ctx, int32_t nbf, const double *centres,
                               const double *alpha, const uint8_t *allowed, double delta,
                               double tau, double psd_tol, int64_t max_vec, double *L,
                               int64_t ldl, int64_t *piv, double *D, int64_t nvec_in,
                               int64_t *h_nvec, double *h_dmax, int32_t *h_status);

/*
 * AO->MO transform of the Cholesky vectors, Eq. (transformation):
 *   B^K_pq = sum_{mu,nu} C_mu,p L^K_mu,nu C_nu,q   (all ordered AO pairs),
 * for the two blocks the self-energy reads (Eq. (SE) via Eq. (aomo)):
 *   Bsel[(s*nmo + r)*ldk + K] = B^K[h_sel[s], r]          s < nsel, r < nmo
 *   Bvo [(a*nocc + i)*ldk + K] = B^K[nocc + a, i]          a < nmo-nocc, i < nocc
 * Entries K in [nvec, ldk) are written as 0 (ldk >= nvec; ldk a multiple of 64
 * is fastest).  C: nbf x nmo row-major (C[mu*nmo + p]), columns are MOs.
 * prec: CDS_PREC_FP64 writes double; CDS_PREC_FP32 writes float;
 * CDS_PREC_BF16X3 writes each block as two bf16 planes, the hi plane (rows x
 * ldk) followed by the lo plane, with hi = x rounded to bf16 and lo = the FP32
 * remainder x - hi rounded to bf16.  The transform itself runs in FP64 for FP64
 * output and in the requested precision otherwise (see
 * cds_set_transform_fp64).  h_sel: host int32[nsel], each in [0, nmo).
 */
int cds_transform(cds_ctx *ctx, int32_t prec, int32_t nbf, int64_t nvec, const double *L,
                  int64_t ldl, const double *C, int32_t nmo, int32_t nocc, int32_t nsel,
                  const int32_t *h_sel, int64_t ldk, void *Bsel, void *Bvo);

/*
 * The decomposition of cds_cholesky_sgauss from a fresh start (nvec_in = 0)
 * and the transform of cds_transform of its vectors (Eq. (transformation)) in
 * one call, the transform overlapped with the decomposition: vectors become
 * final when the decomposition's host loop reads its device state or the word
 * a look-ahead block's commit writes to pinned host memory, and once 112 of
 * them wait (56 on the path with 128 candidates, whose blocks are longer and
 * fewer), the next block's pass is followed by their transform on a second
 * stream of the library (default priority), which fills the device while the
 * block's single-workgroup kernels run; the vectors not yet queued when the
 * decomposition ends are transformed on the caller's stream, beside the
 * batches the side stream has not finished (a second set of batch buffers).
 * The results are those of
 * cds_cholesky_sgauss(..., nvec_in = 0, ...) followed by cds_transform(...,
 * nvec = *h_nvec, ...) with the same arguments, bit for bit (each vector's
 * blocks do not depend on how the vectors are batched), over the entries K <
 * min(ldk, *h_nvec rounded up to 64).  ldk >= max_vec (the number of vectors
 * is known only at the end); entries K in [*h_nvec, min(ldk, *h_nvec rounded
 * up to 64)) are written as 0 and those beyond are left untouched: no
 * consumer of the blocks reads past that multiple of 64.  On CDS_ECAP and CDS_ENOTPSD the vectors
 * made are transformed as well.  Before returning, the call makes the caller's
 * stream wait for the side stream, so work queued there afterwards sees Bsel
 * and Bvo.  Arguments, layouts and other errors as the two calls.  The
 * statistics record the decomposition as cds_cholesky_sgauss does and, as the
 * transform time, only the part left after the decomposition ends.
 */
int cds_cholesky_transform_sgauss(cds_ctx *ctx, int32_t nbf, const double *centres,
                                  const double *alpha, double delta, double tau, double psd_tol,
                                  int64_t max_vec, double *L, int64_t ldl, int64_t *piv, double *D,
                                  int32_t prec, const double *C, int32_t nmo, int32_t nocc,
                                  int32_t nsel, const int32_t *h_sel, int64_t ldk, void *Bsel,
                                  void *Bvo, int64_t *h_nvec, double *h_dmax, int32_t *h_status);

/*
 * Layout of the blocks B^K of Eq. (transformation): rows of ldk entries become
 * rows of ldk_new entries in place, each row keeping its first ldk_new entries
 * (entries K < ldk_new; the buffer keeps its size and the rest of it is left
 * unspecified).  For the blocks cds_cholesky_transform_sgauss writes, whose
 * row stride has to be chosen before the number of vectors is known: the
 * contraction reads rows of nvec entries faster at a row stride near nvec.
 * rows: rows of the block (Bsel: nsel * nmo, Bvo: nvirt * nocc), in the
 * layout cds_transform writes for prec (for CDS_PREC_BF16X3 the hi plane and
 * the lo plane after it, both re-strided, the lo plane then starting at
 * rows * ldk_new).  Requires 1 <= ldk_new <= ldk / 2 (each launch then moves
 * rows whose new places lie below the old ones of the rows it moves, about
 * log(rows) / log(ldk / ldk_new) launches), rows of ldk and of ldk_new entries
 * multiples of 16 bytes and B 16-byte aligned (device memory of at least rows
 * * ldk entries, times two planes for CDS_PREC_BF16X3), else CDS_EINVAL with
 * nothing written.  Queued on the context's stream; the time counts as
 * transform time in the statistics.
 */
int cds_restride_blocks(cds_ctx *ctx, int32_t prec, int64_t rows, int64_t ldk, int64_t ldk_new,
                        void *B);

/*
 * Second-order self-energy, Eq. (SE), and its energy derivative at T trial
 * energies per target, with (qi|aj) and (qa|ib) formed from B by Eq. (aomo):
 *   h_sigma[s*T + t]  = Sigma_qq(h_omega[s*T + t]),   q = h_sel[s]
 *   h_dsigma[s*T + t] = dSigma_qq/domega at the same energy.
 * Bsel, Bvo as written by cds_transform with the same prec, nvec, ldk, nmo,
 * nocc, nsel (entries K in [nvec, min(ldk, nvec rounded up to 64)) must be 0;
 * entries past that are never read).  eps: device double[nmo] orbital energies (occupied first).
 * The contraction runs in `prec`; denominators and sums run in FP64.
 */
int cds_sigma2(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo, int32_t nocc,
               int32_t nsel, const int32_t *h_sel, const void *Bsel, const void *Bvo,
               const double *eps, int32_t T, const double *h_omega, double *h_sigma,
               double *h_dsigma);

/*
 * cds_sigma2 without any device allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, results and summation order as cds_sigma2 (bit for bit), but every device
 * buffer it needs lives in one array of CDS_NOALLOC_SCRATCH_BYTES per GPU, reserved when the
 * library is loaded and held until the process ends: no hipMalloc, no workspace growth, no
 * statistics.  Limits: the blocks must suit the fused contraction (16-byte aligned, ldk >=
 * nvec rounded up to 16 (FP64) or 32 (FP32, BF16X3), ldk times the element size a multiple of
 * 16); the scratch holds the per-task partial sums of the targets of one launch (targets per
 * launch x tasks per target x T x 16 bytes, tasks per target = nocc ceil(nvirt/128)
 * (ceil(nvirt/128)+1)/2 + nvirt ceil(nocc/128)(ceil(nocc/128)+1)/2) plus 24 nsel T + 4 nsel
 * bytes; a call that needs more returns CDS_EINVAL (fewer targets per launch with
 * cds_set_target_chunk, or fewer trial energies, make it fit).  All calls on one GPU share
 * the array: calls that overlap on one GPU (several contexts or threads) race.
 */
#define CDS_NOALLOC_SCRATCH_BYTES (32 << 20)
int cds_sigma2_noalloc(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo, int32_t nocc,
                       int32_t nsel, const int32_t *h_sel, const void *Bsel, const void *Bvo,
                       const double *eps, int32_t T, const double *h_omega, double *h_sigma,
                       double *h_dsigma);

/*
 * Quasi-particle equation w = e_q + Sigma_qq(w), Eq. (qpapp), solved per
 * target by Newton-Raphson, Eq. (iter), with pole strength Eq. (ps):
 *   P_n = 1/(1 - Sigma'(w_n)),  w_{n+1} = w_n + (e_q + Sigma(w_n) - w_n) P_n,
 * starting at w_0 = e_q (h_omega0 == NULL) or h_omega0[s], stopping when
 * |w_{n+1} - w_n| <= conv (Eq. (NR)).  Outputs per target: h_omega = w_{n+1},
 * h_pole = P_n, h_iters = n+1, h_status = CDS_QP_*.  IP = -w for an occupied
 * target, EA = -w for a virtual one.  mode: CDS_QP_RECOMPUTE or
 * CDS_QP_RESIDUES.  max_iter >= 1.
 */
int cds_qp_solve(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo,
                 int32_t nocc, int32_t nsel, const int32_t *h_sel, const void *Bsel,
                 const void *Bvo, const double *eps, const double *h_omega0, double conv,
                 int32_t max_iter, int32_t mode, double *h_omega, double *h_pole,
                 int32_t *h_iters, int32_t *h_status);

/*
 * Adjoint of the converged quasi-particle solve by implicit differentiation
 * of F(w, theta) = e_q + Sigma_qq(w; theta) - w = 0 (not in the paper):
 *   d(w*)/d(theta) = P dF/dtheta,  P = 1/(1 - Sigma'(w*)).
 * Given converged h_omega[s] and cotangents h_omega_bar[s], accumulates
 * (overwrites) Bsel_bar, Bvo_bar and eps_bar (device double[nmo]) with
 * sum_s omega_bar_s d(w*_s)/d(theta).  Bsel_bar and Bvo_bar have the row
 * layout of Bsel and Bvo (rows of ldk entries, K contiguous) in double for
 * CDS_PREC_FP64 and in float for CDS_PREC_FP32 and CDS_PREC_BF16X3 (one plane,
 * not the split pair); entries K in [nvec, ldk) are written as 0.  The
 * gradient w.r.t. B is taken with Bsel and Bvo as independent inputs.
 */
int cds_qp_adjoint(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo,
                   int32_t nocc, int32_t nsel, const int32_t *h_sel, const void *Bsel,
                   const void *Bvo, const double *eps, const double *h_omega,
                   const double *h_omega_bar, void *Bsel_bar, void *Bvo_bar, double *eps_bar);

/*
 * Adjoint of cds_transform with respect to C (FP64):
 *   C_bar = sum_K L^K C (Bbar^K + Bbar^K^T),
 * where Bbar^K (nmo x nmo) holds Bsel_bar[s, r, K] at row h_sel[s] and
 * Bvo_bar[a, i, K] at (nocc + a, i), zero elsewhere (accumulated where they
 * overlap).  Bsel_bar, Bvo_bar: rows of ldk entries as cds_qp_adjoint writes
 * them, double for prec = CDS_PREC_FP64 and float for CDS_PREC_FP32 or
 * CDS_PREC_BF16X3.  C_bar:
 * nbf x nmo row-major, overwritten.
 */
int cds_transform_adjoint(cds_ctx *ctx, int32_t prec, int32_t nbf, int64_t nvec,
                          const double *L, int64_t ldl, const double *C, int32_t nmo,
                          int32_t nocc, int32_t nsel, const int32_t *h_sel, int64_t ldk,
                          const void *Bsel_bar, const void *Bvo_bar, double *C_bar);

/*
 * MP2 correlation energy, Eq. (MP2) of Sec. II.A, from the transformed
 * Cholesky block Bvo (layout and precision `prec` of cds_transform; ldk a
 * multiple of 64) and the orbital energies eps (device double[nmo]):
 *   E = sum_{i,j occ; a,b virt} (2 (ai|bj) - (aj|bi)) (ai|bj) / (e_i + e_j - e_a - e_b),
 *   (ai|bj) = sum_K B^K_ai B^K_bj.
 * The integrals are formed by the MFMA contraction in `prec` (FP32 storage for
 * FP32 and BF16X3) in chunks of virtual orbitals; numerators, denominators and
 * all sums in FP64 with a fixed summation order (deterministic).  Writes E to
 * *h_energy (host) and synchronizes the stream.  1 <= nocc < nmo,
 * nocc <= 1024.  Errors: CDS_EINVAL (nothing written), CDS_ENOMEM, CDS_EDEVICE.
 */
int cds_mp2(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo, int32_t nocc,
            const void *Bvo, const double *eps, double *h_energy);

/*
 * Second-order self-energy as a matrix over the selected orbitals S = h_sel
 * (Sec. II.B; its diagonal is Eq. (SE)):
 *   Sigma_st(w) = sum_{a,i,j} (si|aj) (2(ti|aj) - (tj|ai)) / (w + e_a - e_i - e_j)
 *               + sum_{i,a,b} (sa|ib) (2(ta|ib) - (tb|ia)) / (w + e_i - e_a - e_b),
 * and dSigma_st/dw, at T trial energies h_omega[T] (host).  B blocks, eps and
 * precisions as cds_sigma2 (ldk a multiple of 64); 1 <= nsel <= 31 (symmetric
 * output: h_sigma, h_dsigma host double[T][nsel][nsel]).  The integrals of all
 * selected orbitals are formed at once (at most 16 GiB).  Synchronizes.
 */
int cds_sigma2_matrix(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo,
                      int32_t nocc, int32_t nsel, const int32_t *h_sel, const void *Bsel,
                      const void *Bvo, const double *eps, int32_t T, const double *h_omega,
                      double *h_sigma, double *h_dsigma);

/*
 * Poles of the Dyson equation restricted to the selected orbitals,
 * det(w - e_S - Sigma_SS(w)) = 0 (Eqs. (Dyson), (DysonSol2)), one root per
 * selected orbital q: start at w_0 = e_q, u_0 = unit vector q; at each step
 * diagonalise diag(e_S) + Sigma_SS(w_n), follow the eigenvector u of largest
 * overlap with the previous one (eigenvalue lambda) and set
 *   w_{n+1} = w_n + (lambda - w_n) P_n,   P_n = 1 / (1 - u^T Sigma'(w_n) u)
 * (Hellmann-Feynman slope; with nsel = 1 this is Eq. (iter)) until
 * |w_{n+1} - w_n| <= conv (Eq. (NR)).  Outputs (host, per root k): h_omega =
 * w_{n+1}, h_pole = P_n, h_vec[k][nsel] = u, h_iters, h_status (CDS_QP_*).
 * Other arguments as cds_sigma2_matrix.
 */
int cds_dyson_solve(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo,
                    int32_t nocc, int32_t nsel, const int32_t *h_sel, const void *Bsel,
                    const void *Bvo, const double *eps, double conv, int32_t max_iter,
                    double *h_omega, double *h_pole, double *h_vec, int32_t *h_iters,
                    int32_t *h_status);

/* Device workspace the context holds now (bytes, all slots); it grows on
 * demand and is released by cds_destroy. */
int cds_workspace_bytes(const cds_ctx *ctx, size_t *out);

#ifdef __cplusplus
}
#endif
#endif /* CDSIGMA_H */
