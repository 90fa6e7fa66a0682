// Internal declarations of the cdsigma HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "cdsigma.h"

// Workspace slots: each slot is an independent device buffer owned by the
// context and grown on demand.  Calls use fixed slots so that one call never
// clobbers memory another part of the same call still needs.
enum CdsSlot {
    WS_PAIRS = 0,   // pair table (SoA) of the basis
    WS_CD_PART,     // partial GEMV sums of the CD step
    WS_CD_TILE,     // per-tile max/min of the residual diagonal
    WS_CD_MASK,     // pivot mask
    WS_CD_STATE,    // device CD state
    WS_TR_UNPACK,   // unpacked L^K batch for the transform
    WS_TR_T,        // L^K C_X batch
    WS_TR_B,        // K-major B blocks before the transpose
    WS_TR_CX,       // gathered occupied + selected columns of C
    WS_SG_G,        // contraction output G (integrals)
    WS_SG_PART,     // per-block partial sums of the denominator reduction
    WS_SG_RES,      // pole residues (residue mode)
    WS_SG_OMEGA,    // trial energies on the device
    WS_SG_OUT,      // reduced sigma / dsigma on the device
    WS_AD_G,        // adjoint: dSigma/dG weights
    WS_AD_TMP,      // adjoint scratch
    WS_AD_TMP2,
    WS_MP_G,        // MP2: integral chunk
    WS_MP_S,        // MP2: per-(a, b) sums
    WS_DY_G,        // self-energy matrix: integrals of all selected orbitals
    WS_DY_PART,     // self-energy matrix: partial pair sums
    WS_AD_T1,       // adjoint: K-contiguous copies of transposed GEMM operands
    WS_AD_T2,
    WS_AD_T3,
    WS_SG_TSEL,     // target slots of the fused self-energy launches
    WS_TR_UNPACK2,  // second set of transform batch buffers (the overlapped call's last
    WS_TR_T2,       // vectors, on the caller's stream beside the side stream's batches)
    WS_TR_B2,
    WS_SLOTS
};

struct CdsTimer {
    hipEvent_t a = nullptr, b = nullptr;
    double *acc = nullptr;
};

struct cds_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    void *ws[WS_SLOTS] = {};
    size_t ws_bytes[WS_SLOTS] = {};
    void *pinned = nullptr;          // small pinned host buffer (state readback)
    size_t pinned_bytes = 0;
    cds_stats stats = {};
    std::vector<CdsTimer> pending;   // recorded event pairs not yet accumulated
    std::vector<hipEvent_t> free_events;
    bool broken = false;
    bool kernel_timing = false;      // time every CD step / pass launch with events
    int cd_lookahead = 48;           // Cholesky look-ahead block length (0: plain steps)
    int cd_large_path = 0;           // 1: Cholesky code path of large pair counts at any size
    int cd_speculate = 1;            // 1: speculative look-ahead blocks
    int transform_fp64 = 0;          // 1: transform GEMMs in FP64, output rounded to its precision
    int target_chunk = 0;            // >0: at most this many targets per contraction launch
    hipStream_t stream2 = nullptr;   // side stream (default priority) of the overlapped transform
    hipEvent_t join = nullptr;       // orders stream2 after / before the caller's stream
    hipEvent_t gate = nullptr;       // orders a stream2 batch after a point of the caller's stream
    hipEvent_t trset = nullptr;      // the overlapped transform's coefficient copies are made
    uint64_t *mail = nullptr;        // coherent pinned word the Cholesky commits write (host address)
    uint64_t *mail_dev = nullptr;    // the same word's device address
    bool mail_off = false;           // 1: the word did not follow the state (state read after every batch)
    int cd_mailbox = 1;              // 0: the caller turned the word off
    uint64_t mail_base = 0;          // block count the last Cholesky call started from
    void *scratch = nullptr;         // device address of the allocation-free path's array on this device
};

// device address of the allocation-free path's scratch array on the current device
int cds_noalloc_scratch_address(void **out);

// error helpers -------------------------------------------------------------
int cds_fail(cds_ctx *ctx, int code, const char *fmt, ...);

#define CDS_HIP(ctx, expr)                                                          \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return cds_fail((ctx), CDS_EDEVICE, "%s failed: %s (%s:%d)", #expr,      \
                            hipGetErrorString(e_), __FILE__, __LINE__);             \
    } while (0)

#define CDS_REQUIRE(ctx, cond, ...)                                                 \
    do {                                                                            \
        if (!(cond)) return cds_fail((ctx), CDS_EINVAL, __VA_ARGS__);               \
    } while (0)

#define CDS_CALL(expr)                                                              \
    do {                                                                            \
        int r_ = (expr);                                                            \
        if (r_ != CDS_OK) return r_;                                                \
    } while (0)

// launch check: reports launch-configuration errors immediately
#define CDS_LAUNCHED(ctx) CDS_HIP(ctx, hipGetLastError())

// device workspace of at least `bytes` in `slot` (contents not preserved on growth)
int cds_ws(cds_ctx *ctx, int slot, size_t bytes, void **out);
// pinned host scratch of at least `bytes`
int cds_pinned(cds_ctx *ctx, size_t bytes, void **out);
// begin context entry: checks ctx, sets device, clears the error text
int cds_enter(cds_ctx *ctx);

// event timing: start records an event now; stop records the closing event and
// queues the pair, whose elapsed time is added to *acc at the next flush.
int cds_timer_start(cds_ctx *ctx, CdsTimer *t);
int cds_timer_stop(cds_ctx *ctx, CdsTimer *t, double *acc);
int cds_timers_flush(cds_ctx *ctx);   // synchronizes the stream

static inline int64_t cds_npairs(int64_t nbf) { return nbf * (nbf + 1) / 2; }
__host__ __device__ static inline int64_t cds_ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline bool cds_aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ---- shared device helpers -------------------------------------------------
// pair I -> (mu, nu), mu <= nu, I = nu(nu+1)/2 + mu
__device__ __forceinline__ void cds_pair_decode(int64_t I, int64_t &mu, int64_t &nu)
{
    int64_t n = (int64_t)((sqrt(8.0 * (double)I + 1.0) - 1.0) * 0.5);
    if (n * (n + 1) / 2 > I) --n;
    if ((n + 1) * (n + 2) / 2 <= I) ++n;
    nu = n;
    mu = I - n * (n + 1) / 2;
}

// precision tags ---------------------------------------------------------------
static inline size_t cds_prec_bytes(int prec) { return prec == CDS_PREC_FP64 ? 8 : 4; }

// internal entry points shared between translation units ----------------------
// Progress of a decomposition: after each read of its device state, and of the mailbox word a
// speculative block's commit writes, the host loop calls committed(user, k) with the number
// of vectors that are final (no later kernel of the decomposition writes L[0..k) again, and
// the kernels that wrote them have completed).
// A non-zero return ends the decomposition with that status.
// block(user, wide) is called after each look-ahead block's pass has been queued on the
// caller's stream (may be NULL); wide is 1 on the path with the wider candidate set (longer
// blocks, fewer of them), else 0.
struct CdHook {
    int (*committed)(void *user, int64_t k);
    int (*block)(void *user, int wide);
    void *user;
};
// cds_cholesky_sgauss from a fresh start (nvec_in = 0) with a progress hook
int cds_cholesky_hooked(cds_ctx *ctx, int32_t nbf, const double *centres, const double *alpha, double delta,
                        double tau, double psd_tol, int64_t max_vec, double *L, int64_t ldl, int64_t *piv,
                        double *D, int64_t *h_nvec, double *h_dmax, int32_t *h_status, const CdHook *hook);

// One direct-to-LDS load of 16 bytes per lane (global_load_lds_dwordx4: lane t's bytes go to
// LDS address dst + 16 t, dst wave-uniform, passed in m0).  Written out in assembly so that the
// compiler does not track it: its tracking of such loads cannot tell a double-buffered kernel's
// two LDS stages apart and makes every LDS read wait for every load in flight, the next stage's
// prefetch included.  The caller therefore waits itself (s_waitcnt vmcnt, then a workgroup
// barrier) before the data is read, and before a buffer is refilled every wave must have read
// it.  The instruction writes no register.  No kernel of this library uses m0 otherwise.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
static __device__ __forceinline__ void cds_lds_dma16(const void *src, void *dst)
{
    const unsigned m = __builtin_amdgcn_readfirstlane(
        (unsigned)(uintptr_t)(__attribute__((address_space(3))) void *)dst);
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(m)
                 : "memory", "m0");
}
#pragma clang diagnostic pop

// GEMM engine (gemm.hip): C[b][m][n] = alpha * sum_k A(m,k) B(k,n) (+ beta C)
struct GemmDesc {
    int64_t M, N, K, batch;
    const void *A;
    int64_t sAm, sAk, sAb;   // element strides of A(m,k) and per batch
    const void *B;
    int64_t sBk, sBn, sBb;
    void *C;
    int64_t sCm, sCn, sCb;
    double alpha, beta;      // beta: 0 overwrite, 1 accumulate
    void *Clo;               // BF16X3 only, beta 0: C and Clo receive the hi and lo bf16 planes
                             // of the result (same element offsets) instead of floats
    int big;                 // BF16X3 only: 0 = 256 x 256 tiles when M and N are both >= 512,
                             // 1 = never, 2 = whenever the operands allow (a choice that must not
                             // depend on how a caller batches its rows)
};
// prec of A/B/C: FP64 -> double, FP32/BF16X3 -> float storage
int cds_gemm(cds_ctx *ctx, int prec, const GemmDesc &d);
// Alo/Blo: lo planes of BF16X3 operands (hi planes at d.A / d.B); NULL otherwise
int cds_gemm_ex(cds_ctx *ctx, int prec, const GemmDesc &d, const void *Alo, const void *Blo);
// out[c*ldo + r] = in[r*ldi + c] for r < rows, c < cols; elements of es bytes (4 or 8)
int cds_transpose(cds_ctx *ctx, int es, int64_t rows, int64_t cols, const void *in, int64_t ldi, void *out,
                  int64_t ldo);

// Fused self-energy contraction (sigma_fused.hip): the integrals of Eq. (SE) are formed by MFMA
// products and reduced over the energy denominators in one kernel, task by task (a task = one
// tile pair of the (qi|aj) matrix of a virtual a or the (qa|ib) matrix of an occupied i).
struct CdsFusedPlan {
    int64_t ns;              // K stages
    int nTA, nTB, nPA, nPB;  // 128-row tiles and tile pairs of parts A and B
    int64_t tpt;             // tasks per target
    int64_t sizeA, sizeB;    // residues per virtual a / per occupied i
    int64_t nres;            // residues per target
};
// false when the blocks do not suit the fused kernel (alignment, K padding); p filled otherwise
bool cds_fused_plan(int prec, int64_t nvec, int64_t ldk, int nmo, int nocc, const void *Bsel, const void *Bvo,
                    const void *Bsel_lo, const void *Bvo_lo, CdsFusedPlan *p);
// partial sums d_part[nsc][tpt][T][2] of Sigma and Sigma' for the targets d_tsel[0..nsc) at
// d_omega[nsc][T]
int cds_fused_sigma(cds_ctx *ctx, int prec, const CdsFusedPlan &p, int64_t ldk, int nmo, int nocc, int nsc,
                    const int *d_tsel, const void *Bsel, const void *Bvo, const void *Bsel_lo, const void *Bvo_lo,
                    const double *eps, const double *d_omega, int T, double *d_part);
// pole residues R[nsc][nres] (double for FP64, float otherwise) of the targets d_tsel[0..nsc); with
// d_part, also the sums at d_omega0[nsc] from the stored residues, d_part[nsc][tpt][2] (the
// layout of a sweep's partials)
int cds_fused_residues(cds_ctx *ctx, int prec, const CdsFusedPlan &p, int64_t ldk, int nmo, int nocc, int nsc,
                       const int *d_tsel, const void *Bsel, const void *Bvo, const void *Bsel_lo, const void *Bvo_lo,
                       const double *eps, void *R, const double *d_omega0 = nullptr, double *d_part = nullptr);
// one Newton sweep: d_part[nactive][tpt][2] for the targets d_active at d_omega[target]; with
// d_cnt, only the first d_cnt[0] <= nactive of them (read on the device)
int cds_fused_sweep(cds_ctx *ctx, int prec, const CdsFusedPlan &p, int nmo, int nocc, int nactive,
                    const int *d_active, const double *eps, const double *d_omega, const void *R, double *d_part,
                    const int *d_cnt = nullptr);
