// Diagonal-pivoted incomplete Cholesky decomposition of the ERI supermatrix
// (Sec. II.A of the paper: Eqs. (gs_coulomb), (CD), (stricterr)) with ERI
// columns of normalized s-Gaussians evaluated on demand (Eq. (integral),
// closed form through the Boys function F0).
//
// Each step k picks the pivot p (lowest index within the tie window of the largest residual
// diagonal), forms the residual column c = V[:,p] - sum_{j<k} L[j] L[j][p], sets
// L[k] = c / sqrt(D_p) and updates D.  Done literally, step k streams k*npairs*8
// bytes of L and needs a grid-wide argmax before the next step.  This implementation
// makes the same steps (same pivot rule, the vectors equal to rounding) in look-ahead
// blocks that start at step k0:
//     cd_cand    the pivot of step k0 plus the rows with the largest residual
//                diagonals (CD_NCAND candidates in all)
//     cd_candcol R[c][I] = V[I][cand_c]                               (ERI columns)
//     cd_gather  P[j][c] = L[j][cand_c]                               j < k0
//     cd_pass    R[c][I] -= sum_{j<k0} L[j][I] P[j][c]                (one read of L,
//                FP64 MFMA)
//   speculative block (default, one-sweep pivot search):
//     cd_spec    the next steps restricted to the candidates (one wave, their 64 x 64
//                residual block in LDS): pivots, sqrt(D_p), the pivots' rows
//     cd_rows    those vectors for every row, with a check per step that no row
//                outside the candidates would have changed the pivot choice
//     cd_commit  the steps before the first failing one become real (D, mask, tile
//                records, pivots); the next block starts there
//   large path (separate speculative and row kernels): only the speculated pivots' columns
//   are ever read, so the candidates' own 64 x 64 block comes first from the gathered rows
//   (cd_cc, the pass's operations entry for entry), cd_spec chooses the steps, and the pass
//   forms just those columns (cd_pass_cols, 16 per group): the same values, a fraction of
//   the work
//   per-step kernel (block_steps steps per block when speculation is off, or when
//   nothing could be committed): ONE launch per step (cd_step), each block of one
//   (or, for many tiles, four) 64-row tiles:
//     - picks the pivot itself from the previous step's tile records (largest and
//       smallest residual of each 64-row tile, and its lowest row within the tie window of its
//       largest): one sweep over all records, or for many tiles 64 super-tile maxima
//       kept with order-preserving integer atomics first; every block reaches the
//       same pivot;
//     - c_I = R[slot][I] - sum_{k0<=j<k} L[j][I] L[j][p] when p is candidate `slot`,
//       else V_Ip - sum_{j<k} L[j][I] L[j][p] (a miss);
//     - writes L[k], the next residual diagonal and pivot mask, tile statistics.
//   D, the mask and the tile records are double-buffered and the super-tile
//   keys triple-buffered by step parity, so no block reads what another
//   block of the same launch writes: no fences or grid barriers.
//
// Device layout (HBM): pair table SoA p, Px, Py, Pz, K (5 x npairs FP64); L vector-
// major (vector k at L + k*ldl); D FP64[2][npairs] (the first copy is the caller's);
// pivot mask u8[2][npairs]; candidate residual columns R[c][ldr]; candidate rows
// P[j][CD_NCAND].
#include "cds_internal.h"

#include <cfloat>
#include <chrono>
#include <climits>

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int CD_TILE = 64;             // rows per step/pass block (= pivot scan tile)
constexpr int CD_NT = 256;              // threads of the step kernel
constexpr int CD_PCHUNK = 1024;         // pivot-row entries staged in LDS per chunk
constexpr int CD_AUX_NT = 1024;         // threads of the one-block kernels
constexpr int CD_NSUP = 64;             // super-tiles of the hierarchical pivot search
constexpr int CD_NCAND = 64;            // candidate residual columns per look-ahead block
constexpr int CD_NCAND_L = 128;         // candidates per speculative block on the large path
constexpr int CD_CG = 8;                 // candidate columns per thread in the column kernels
constexpr int CD_NCG = CD_NCAND / CD_CG; // column groups (rows of the column grid)
constexpr int CD_PASS_D = 2;            // k-steps (4 vectors each) in flight per wave in the pass
constexpr int CD_PASS_ZROWS = 8;        // zero rows of P after row k0
constexpr int CD_TPT = 4;               // tile records per thread in the flat pivot search
constexpr int CD_ONE_TILE_MAX = 1280;   // tiles up to which a step block holds one tile
constexpr int CD_SPEC_MAX = 48;         // steps of one speculative look-ahead block (multiple of 8, <= 64)
constexpr int CD_SPEC_CHUNK = 8;        // steps between the rows kernel's looks at the published checks
constexpr int CD_SPEC_MARGIN = 8;       // speculated steps past the last one that is sure to stand
constexpr int CD_FUSE_MAXBLK = 256;     // row workgroups up to which every one forms the speculative block
constexpr int CD_CAND_MAXTILE = 8192;   // tiles the candidate selection handles (look-ahead
                                        // is off above 8192 * 64 pairs)

struct PairTable {
    double *p, *Px, *Py, *Pz, *K;
};

struct CdState {
    int64_t k;       // vectors made so far (block 0 of every step)
    double dmax;     // largest non-pivot residual diagonal seen by the last step
    int32_t done;    // 1 once a termination rule fired
    int32_t status;  // CDS_CD_* once done
    int32_t ncand;   // candidates of the current look-ahead block
    int32_t stall;   // 1: the last speculative block kept no step (the host runs one per-step launch)
    int64_t nmiss;   // steps whose pivot was not a candidate
    double bytes;    // bytes the step kernels must move (algorithmic, per the formula at the update)
    int64_t nspec;   // steps committed by speculative blocks
    int64_t kdone;   // step whose launch found a termination rule (INT64_MAX before): later
                     // launches return at once; blocks of that same launch all still see it
                     // as not earlier than their step, so no block splits on it
    int64_t npass;   // speculative blocks that ran a pass
    double sumk0;    // sum of their start steps (for the pass work counts)
    int32_t nmap;    // entries of the row -> candidate slot map that are set (cand[0 .. nmap))
    int32_t pad2;
    double dnc;      // bound on the residual diagonals of the eligible rows that are not candidates
    int64_t nblk;    // speculative blocks that reached their commit (kept steps or stalled)
    double sumk0s;   // sum over committed blocks of start step x steps kept (the pass's share of
                     // the plain algorithm's products: each kept step needs vectors 0 .. k0-1)
    double sumwin;   // sum over committed blocks of j for each kept step j (the block's own share)
    double sumk0c;   // large path: sum over passes of start step x columns formed (16 per group)
    int64_t ncols;   // large path: columns the passes formed
};

// Host mailbox word, written by each speculative block's commit: the committed step count,
// the stall flag and the block count (modulo 2^23), in one 64-bit store the host can read
// while later blocks run.
constexpr int MB_KBITS = 40;
constexpr uint64_t MB_KMASK = (1ull << MB_KBITS) - 1;
constexpr int MB_NSHIFT = MB_KBITS + 1;
constexpr uint64_t MB_NMASK = (1ull << (64 - MB_NSHIFT)) - 1;
__host__ __device__ inline uint64_t mb_word(int64_t nblk, int stall, int64_t k)
{
    return (((uint64_t)nblk & MB_NMASK) << MB_NSHIFT) | ((uint64_t)(stall != 0) << MB_KBITS) |
           ((uint64_t)k & MB_KMASK);
}

// Per 64-row tile, over its non-pivot rows: the largest and smallest residual diagonal,
// and the lowest row whose residual is within the tie window of the largest (with that
// residual).
struct TileStat {
    double mx, mn, dfirst;
    int64_t first;                      // -1: no non-pivot row
};

struct CdBufs {
    double *D[2];                       // residual diagonal, by parity
    unsigned char *mask[2];             // pivot mask, by parity
    TileStat *ts[2];                    // tile records, by parity
    unsigned long long *smax[3];        // super-tile max keys (atomicMax), triple-buffered
    unsigned long long *smin[3];        // super-tile min keys (atomicMin)
    int64_t ntile, tps;                 // tiles; tiles per super-tile
    int flat;                           // 1: pivot search over all tile records (no keys)
    signed char *slot;                  // row -> candidate slot of the current block, -1 otherwise
    double *rc;                         // rc[s][c] = R[s][cand_c], the candidates' own block
};

struct CdParams {
    int64_t npairs, max_vec;
    double delta, tau, psd_tol;
    int64_t nvec_in;   // vectors given on entry (buffer parities count steps from there)
    int32_t spec_len;  // longest speculative block
    int32_t pad;
};

// order-preserving map of doubles to unsigned keys; 0 means "no entry" (-inf),
// ~0 means "no entry" for minima (+inf)
__device__ __forceinline__ unsigned long long okey(double v)
{
    long long b = __double_as_longlong(v);
    return b < 0 ? ~(unsigned long long)b : ((unsigned long long)b | 0x8000000000000000ull);
}
__device__ __forceinline__ double okey_max(unsigned long long u)
{
    if (u == 0ull) return -INFINITY;
    return (u & 0x8000000000000000ull) ? __longlong_as_double((long long)(u & 0x7fffffffffffffffull))
                                       : __longlong_as_double((long long)~u);
}
__device__ __forceinline__ double okey_min(unsigned long long u)
{
    if (u == ~0ull) return INFINITY;
    return okey_max(u);
}

// F0(T) = (1/2) sqrt(pi / T) erf(sqrt T) = (sqrt(pi) / 2) erf(t) / t with t = sqrt T (one
// square root, one division); the series near T = 0
__device__ __forceinline__ double boys_f0(double T)
{
#pragma clang fp contract(off)
    if (T < 1e-12) return 1.0 - T / 3.0 + T * T / 10.0;
    const double t = sqrt(T);
    return 0.88622692545275801365 * erf(t) / t;           // sqrt(pi) / 2
}

// (rho_I | V | rho_J) for two s-Gaussian product densities.  No implicit contraction: the fused
// multiply-adds are written out, so every kernel that inlines it forms the same value (the
// speculative path relies on the candidates' block and the pass agreeing bit for bit).
__device__ __forceinline__ double eri_pp(double p, double Px, double Py, double Pz, double Kp,
                                         double q, double Qx, double Qy, double Qz, double Kq)
{
#pragma clang fp contract(off)
    const double two_pi_52 = 2.0 * 17.493418327624862;   // 2 pi^(5/2)
    const double dx = Px - Qx, dy = Py - Qy, dz = Pz - Qz;
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const double s = p + q, pq = p * q;
    const double e = 1.0 / (pq * s);                        // one division for both factors
    const double T = pq * pq * e * r2;                      // p q / (p + q) * r2
    return Kp * Kq * two_pi_52 * sqrt(s) * e * boys_f0(T);  // ... / (p q sqrt(p + q))
}

__global__ void pair_setup_kernel(int32_t nbf, const double *__restrict__ centres,
                                  const double *__restrict__ alpha, int64_t npairs, PairTable pt)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= npairs) return;
    int64_t mu, nu;
    cds_pair_decode(I, mu, nu);
    double a = alpha[mu], b = alpha[nu];
    double Ax = centres[3 * mu], Ay = centres[3 * mu + 1], Az = centres[3 * mu + 2];
    double Bx = centres[3 * nu], By = centres[3 * nu + 1], Bz = centres[3 * nu + 2];
    double p = a + b;
    double r2 = (Ax - Bx) * (Ax - Bx) + (Ay - By) * (Ay - By) + (Az - Bz) * (Az - Bz);
    double na = pow(2.0 * a / M_PI, 0.75), nb = pow(2.0 * b / M_PI, 0.75);
    pt.p[I] = p;
    pt.Px[I] = (a * Ax + b * Bx) / p;
    pt.Py[I] = (a * Ay + b * By) / p;
    pt.Pz[I] = (a * Az + b * Bz) / p;
    pt.K[I] = na * nb * exp(-a * b * r2 / p);
}

__global__ void eri_diag_kernel(int64_t npairs, PairTable pt, double *__restrict__ D)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= npairs) return;
    double p = pt.p[I], K = pt.K[I];
    D[I] = eri_pp(p, pt.Px[I], pt.Py[I], pt.Pz[I], K, p, pt.Px[I], pt.Py[I], pt.Pz[I], K);
}

__global__ void dense_diag_kernel(int64_t npairs, const double *__restrict__ V, int64_t ldv,
                                  double *__restrict__ D)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= npairs) return;
    D[I] = V[I * ldv + I];
}

__global__ void eri_columns_kernel(int64_t npairs, PairTable pt, int64_t ncol,
                                   const int64_t *__restrict__ cols, double *__restrict__ out)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t c = blockIdx.y;
    if (I >= npairs || c >= ncol) return;
    int64_t J = cols[c];
    out[c * npairs + I] = eri_pp(pt.p[I], pt.Px[I], pt.Py[I], pt.Pz[I], pt.K[I], pt.p[J], pt.Px[J],
                                 pt.Py[J], pt.Pz[J], pt.K[J]);
}

// ---- block reductions ---------------------------------------------------------
template <int NT>
__device__ __forceinline__ double block_max(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    v = (threadIdx.x < NT / 64) ? sh[threadIdx.x] : -INFINITY;
    if (w == 0)
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if (threadIdx.x == 0) sh[0] = v;
    __syncthreads();
    return sh[0];
}

template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int *sh, int *total)
{
    // inclusive scan within each wave, then over the wave totals (fixed order)
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (l >= o) x += y;
    }
    __syncthreads();
    if (l == 63) sh[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0;
        for (int i = 0; i < NT / 64; ++i) {
            int t = sh[i];
            sh[i] = a;
            a += t;
        }
        sh[NT / 64] = a;
    }
    __syncthreads();
    int r = sh[w] + x - v;
    *total = sh[NT / 64];
    __syncthreads();
    return r;
}

// ---- pivot choice (identical in every block that calls it) --------------------
enum { PICK_GO = -100 };

struct Pick {
    int status;      // PICK_GO or a CDS_CD_* termination
    int slot;        // the pivot's look-ahead candidate slot, -1 if none
    double mx;       // largest non-pivot residual diagonal
    int64_t p;       // pivot
    double dp;       // its residual diagonal
};

struct PickShared {
    double v[2 * 16];
    int64_t i[16];
    TileStat rec;
    Pick pk;
};

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
// Wave reductions through DPP row operations (quad swaps, half-row and row mirrors) and
// four lane reads, instead of six rounds of cross-lane permutes: result in every lane.
__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
// maximum over the wave (DPP row_shr 1, 2, 4, 8, then row_bcast 15, 31; lane 63 holds it)
__device__ __forceinline__ unsigned wave_max_u32_dpp(unsigned v)
{
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
// largest order-preserving key (okey) over the wave: high words, then the low words of the
// lanes that hold the largest high word
__device__ __forceinline__ unsigned long long wave_max_key(unsigned long long k)
{
    const unsigned hi = wave_max_u32_dpp((unsigned)(k >> 32));
    const unsigned lo = wave_max_u32_dpp((unsigned)(k >> 32) == hi ? (unsigned)k : 0u);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ int64_t i64_min(int64_t a, int64_t b) { return b < a ? b : a; }
template <int CTRL>
__device__ __forceinline__ int64_t dpp_i64(int64_t v)
{
    const int lo = __builtin_amdgcn_update_dpp((int)(v & 0xffffffff), (int)(v & 0xffffffff), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(v >> 32), (int)(v >> 32), CTRL, 0xF, 0xF, false);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int64_t readlane_i64(int64_t v, int lane)
{
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int64_t wave_min_i64_dpp(int64_t v)
{
    v = i64_min(v, dpp_i64<0xB1>(v));
    v = i64_min(v, dpp_i64<0x4E>(v));
    v = i64_min(v, dpp_i64<0x141>(v));
    v = i64_min(v, dpp_i64<0x140>(v));
    return i64_min(i64_min(readlane_i64(v, 0), readlane_i64(v, 16)), i64_min(readlane_i64(v, 32), readlane_i64(v, 48)));
}

__device__ __forceinline__ int64_t wave_min_i64(int64_t v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    return v;
}

// Tie window of the pivot rule: tau, but at most 1% of the largest residual, so that near
// the end of a decomposition to a threshold close to tau it still only separates ties.
__device__ __forceinline__ double tie_window(double mx, double tau) { return fmin(tau, 1e-2 * mx); }

__device__ __forceinline__ int pick_status(double mx, double mn, const CdParams &cp, int64_t k)
{
    if (mn < -cp.psd_tol) return CDS_CD_NOTPSD;
    if (mx == -INFINITY) return CDS_CD_FULLRANK;
    if (mx <= cp.delta) return CDS_CD_CONVERGED;
    if (k >= cp.max_vec) return CDS_CD_CAP;
    return PICK_GO;
}

// Within tile t (whose largest residual is >= thresh): the lowest non-pivot row with
// D >= thresh.  One wave.  The tile record names it directly when the tile holds the
// overall maximum (its own window is then the same); otherwise the tile's rows are read.
__device__ __forceinline__ void pick_in_tile(const CdBufs &b, int r, const CdParams &cp, int64_t t,
                                             const TileStat &rec, double mx, double thresh, Pick &pk)
{
    if (rec.mx == mx) {
        pk.p = rec.first;
        pk.dp = rec.dfirst;
        return;
    }
    const int l = threadIdx.x & 63;
    const int64_t I = t * CD_TILE + l;
    const double d = I < cp.npairs ? b.D[r][I] : -INFINITY;
    const bool ok = I < cp.npairs && !b.mask[r][I] && d >= thresh;
    const unsigned long long bp = __ballot(ok);
    if (!bp) {
        pk.status = CDS_CD_NOTPSD;                 // only with non-finite residuals
        return;
    }
    const int lp = __ffsll((long long)bp) - 1;
    pk.p = t * CD_TILE + lp;
    pk.dp = __shfl(d, lp, 64);
}

// Hierarchical search for large tile counts (one wave): 64 super-tile keys, then the first
// super-tile's tile records, then one tile.
__device__ Pick cd_pick_super(const CdBufs &b, int r, int sr, const CdParams &cp, int64_t k)
{
    const int l = threadIdx.x & 63;               // CD_NSUP == 64: one super-tile per lane
    const double v = okey_max(b.smax[sr][l]);
    const double mx = wave_max(v);
    const double mn = wave_min(okey_min(b.smin[sr][l]));
    Pick pk;
    pk.mx = mx;
    pk.p = -1;
    pk.dp = 0.0;
    pk.slot = -1;
    pk.status = pick_status(mx, mn, cp, k);
    if (pk.status != PICK_GO) return pk;
    const double thresh = mx - tie_window(mx, cp.tau);
    const unsigned long long bs = __ballot(v >= thresh);
    int64_t t = -1;
    if (bs) {
        const int64_t sidx = __ffsll((long long)bs) - 1;
        const int64_t t0 = sidx * b.tps, t1 = min(b.ntile, t0 + b.tps);
        for (int64_t u0 = t0; u0 < t1; u0 += 64) {
            const int64_t u = u0 + l;
            const unsigned long long bt = __ballot(u < t1 && b.ts[r][u].mx >= thresh);
            if (bt) {
                t = u0 + __ffsll((long long)bt) - 1;
                break;
            }
        }
    }
    if (t < 0) {
        pk.status = CDS_CD_NOTPSD;
        return pk;
    }
    const TileStat rec = b.ts[r][t];
    pick_in_tile(b, r, cp, t, rec, mx, thresh, pk);
    return pk;
}

// Pivot of step k from the tile records of parity r (every thread of the block calls it;
// the result is the same in every block).  Up to NT * CD_TPT tiles the records are read
// in one sweep by the whole block; beyond that the super-tile keys lead the way.
template <int NT>
__device__ Pick cd_pick(const CdBufs &b, int r, int sr, const CdParams &cp, int64_t k, PickShared &sh)
{
    constexpr int NW = NT / 64;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (!b.flat) {
        if (w == 0) {
            const Pick pk = cd_pick_super(b, r, sr, cp, k);
            if (l == 0) sh.pk = pk;
        }
        __syncthreads();
        return sh.pk;
    }
    TileStat rc[CD_TPT];
    double lmx = -INFINITY, lmn = INFINITY;
#pragma unroll
    for (int i = 0; i < CD_TPT; ++i) {
        const int64_t u = threadIdx.x + (int64_t)NT * i;
        if (u < b.ntile) {
            rc[i] = b.ts[r][u];
        } else {
            rc[i].mx = -INFINITY;
            rc[i].mn = INFINITY;
            rc[i].dfirst = 0.0;
            rc[i].first = -1;
        }
        lmx = fmax(lmx, rc[i].mx);
        lmn = fmin(lmn, rc[i].mn);
    }
    lmx = wave_max(lmx);
    lmn = wave_min(lmn);
    if (l == 0) {
        sh.v[w] = lmx;
        sh.v[NW + w] = lmn;
    }
    __syncthreads();
    double mx = -INFINITY, mn = INFINITY;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        mx = fmax(mx, sh.v[q]);
        mn = fmin(mn, sh.v[NW + q]);
    }
    Pick pk;
    pk.mx = mx;
    pk.p = -1;
    pk.dp = 0.0;
    pk.slot = -1;
    pk.status = pick_status(mx, mn, cp, k);
    if (pk.status != PICK_GO) return pk;          // uniform over the block
    const double thresh = mx - tie_window(mx, cp.tau);
    int64_t tf = INT64_MAX;
#pragma unroll
    for (int i = CD_TPT - 1; i >= 0; --i)
        if (rc[i].mx >= thresh) tf = threadIdx.x + (int64_t)NT * i;
    tf = wave_min_i64(tf);
    if (l == 0) sh.i[w] = tf;
    __syncthreads();
    int64_t t = INT64_MAX;
#pragma unroll
    for (int q = 0; q < NW; ++q) t = sh.i[q] < t ? sh.i[q] : t;
    if (t == INT64_MAX) {
        pk.status = CDS_CD_NOTPSD;                 // only with non-finite residuals
        return pk;
    }
    if (threadIdx.x == t % NT) {
#pragma unroll
        for (int i = 0; i < CD_TPT; ++i)
            if (t == threadIdx.x + (int64_t)NT * i) sh.rec = rc[i];
    }
    __syncthreads();
    const TileStat rec = sh.rec;
    if (rec.mx == mx) {                            // the usual case: no further read
        pk.p = rec.first;
        pk.dp = rec.dfirst;
        return pk;
    }
    if (w == 0) {
        pick_in_tile(b, r, cp, t, rec, mx, thresh, pk);
        if (l == 0) sh.pk = pk;
    }
    __syncthreads();
    return sh.pk;
}

// pivot mask of a restricted decomposition: 0 = may become a pivot, 2 = never (row updated)
// The decomposition's starting buffers in one launch: the pivot mask cleared (unless a kernel of
// its own set it), no row a candidate, the three super-tile buffers empty, the state, and on a
// fresh start the residual diagonal D = the ERI diagonal.
__global__ __launch_bounds__(256) void cd_setup_kernel(int64_t npairs, unsigned char *__restrict__ mask0,
                                                       int clear_mask, signed char *__restrict__ slot,
                                                       unsigned long long *__restrict__ smax,
                                                       unsigned long long *__restrict__ smin, double *__restrict__ D,
                                                       const double *__restrict__ diag, int copy_d, CdState st0,
                                                       CdState *__restrict__ st)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < npairs) {
        if (clear_mask) mask0[t] = 0;
        slot[t] = -1;
        if (copy_d) D[t] = diag[t];
    }
    if (t < 3 * CD_NSUP) {
        smax[t] = 0ull;
        smin[t] = ~0ull;
    }
    if (t == 0) *st = st0;
}

__global__ void init_mask_kernel(int64_t npairs, const unsigned char *__restrict__ allowed,
                                 unsigned char *__restrict__ mask)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I < npairs) mask[I] = allowed[I] ? 0 : 2;
}

__global__ void mark_pivots_kernel(int64_t n, const int64_t *__restrict__ piv, int64_t npairs,
                                   unsigned char *__restrict__ mask)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) {
        int64_t p = piv[j];
        if (p >= 0 && p < npairs) mask[p] = 1;
    }
}

// Record of one 64-row tile from its rows' new residuals (one wave; `active` = a row that
// may still become a pivot, `nonpiv` = any non-pivot row): largest residual and the lowest
// row within the tie window of it over the active rows, smallest over the non-pivot rows.
__device__ __forceinline__ void tile_record(const CdBufs &b, int w, int sw, const CdParams &cp, int64_t tile,
                                            bool active, bool nonpiv, double dn)
{
    const int l = threadIdx.x & 63;
    const double tmx = wave_max(active ? dn : -INFINITY);
    const double tmn = wave_min(nonpiv ? dn : INFINITY);
    const unsigned long long fb = __ballot(active && dn >= tmx - tie_window(tmx, cp.tau));
    const int fl = fb ? __ffsll((long long)fb) - 1 : 0;
    const double df = __shfl(dn, fl, 64);
    if (l == 0) {
        TileStat s;
        s.mx = tmx;
        s.mn = tmn;
        s.dfirst = fb ? df : 0.0;
        s.first = fb ? tile * CD_TILE + fl : -1;
        b.ts[w][tile] = s;
        if (!b.flat) {
            const int64_t sidx = tile / b.tps;
            if (tmx != -INFINITY) atomicMax(&b.smax[sw][sidx], okey(tmx));
            if (tmn != INFINITY) atomicMin(&b.smin[sw][sidx], okey(tmn));
        }
    }
}

// tile records (and super-tile keys) of D[0] / mask[0] (start or resume)
__global__ __launch_bounds__(CD_TILE) void tile_stats_kernel(CdBufs b, CdParams cp)
{
    const int64_t I = (int64_t)blockIdx.x * CD_TILE + threadIdx.x;
    const unsigned char m = I < cp.npairs ? b.mask[0][I] : 1;
    const double d = m != 1 ? b.D[0][I] : 0.0;
    tile_record(b, 0, 0, cp, blockIdx.x, m == 0, m != 1, d);
}

// One Cholesky step (one launch).  Block = TB tiles (64 TB rows); thread (jg, rl): rows
// I0..I0+VW-1, vectors j = jstart + jg, + JG, ...; partial sums combined in LDS in fixed
// order; wave w finalizes tile w of the block.  TB > 1 for large pair counts, so that the
// per-block pivot search runs once for several tiles and the grid fits the chip in one
// round.
// r/w: read/write parity of D, mask and tile records; sr/sw/sz: super-tile buffers read,
// written (atomics) and reset for the step after next.  Loads that do not depend on the
// pivot (the vectors made since the block start, D, mask, the candidate list) are issued
// before the pivot search.
struct SpecOut;
// the column of R that the large path's pass formed for candidate slot sl (its speculated step),
// or -1 (defined below)
__device__ int spec_column(const SpecOut *so, int sl);

template <int VW, int TB, bool DENSE>
__global__ __launch_bounds__(CD_NT) void cd_step_kernel(
    CdBufs b, CdParams cp, int r, int sr, int sw, int sz, int64_t k, int64_t k0, int bsteps,
    PairTable pt, const double *__restrict__ V, int64_t ldv, double *__restrict__ L, int64_t ldl,
    const double *__restrict__ R, int64_t ldr, const int64_t *__restrict__ cand, CdState *st,
    int64_t *__restrict__ piv, const SpecOut *__restrict__ sov)
{
    constexpr int NR = CD_TILE * TB;            // rows per block
    constexpr int RL = NR / VW;                 // row lanes
    constexpr int JG = CD_NT / RL;              // vector groups
    constexpr int NPF = JG >= 8 ? 2 : 16 / JG;  // prefetched vectors per thread (a 16-step block)
    static_assert(JG >= 1 && CD_NT % RL == 0 && TB * 64 <= CD_NT, "step kernel shape");
    __shared__ double sp[CD_PCHUNK];
    __shared__ double red[JG][NR];
    __shared__ PickShared psh;
    __shared__ int sslot;
    const int64_t kdone = st->kdone;
    const int rl = threadIdx.x % RL, jg = threadIdx.x / RL;
    const int64_t tile0 = (int64_t)blockIdx.x * NR;
    const int64_t I0 = tile0 + (int64_t)VW * rl;
    const bool rows_ok = I0 < cp.npairs;
    // prefetch (independent of the pivot)
    const int64_t nblk = bsteps > 0 ? k - k0 : 0;        // vectors since the block start
    double pf[NPF][VW];
#pragma unroll
    for (int m = 0; m < NPF; ++m) {
        const int64_t j = k0 + jg + (int64_t)m * JG;
#pragma unroll
        for (int v = 0; v < VW; ++v) pf[m][v] = 0.0;
        if (rows_ok && j < k0 + nblk) {
            if constexpr (VW == 2) {
                double2 x = *reinterpret_cast<const double2 *>(L + j * ldl + I0);
                pf[m][0] = x.x;
                pf[m][1] = x.y;
            } else {
                pf[m][0] = L[j * ldl + I0];
            }
        }
    }
    const int64_t If = tile0 + threadIdx.x;              // finalize row of threads < NR
    double d_old = 0.0;
    unsigned char m_old = 1;
    if (threadIdx.x < NR && If < cp.npairs) {
        d_old = b.D[r][If];
        m_old = b.mask[r][If];
    }
    // candidate list of the current look-ahead block (up to 128: two per lane of wave 0; the
    // list always has room for 128)
    int64_t cl = -1, cl2 = -1;
    int nc = 0;
    if (bsteps > 0 && threadIdx.x < 64) {
        nc = st->ncand;
        cl = cand[threadIdx.x];
        cl2 = cand[threadIdx.x + 64];
    }
    if (kdone < k) return;
    Pick pk = cd_pick<CD_NT>(b, r, sr, cp, k, psh);
    if (pk.status != PICK_GO) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->k = k;
            st->dmax = pk.mx;
            st->status = pk.status;
            st->kdone = k;
            st->done = 1;
        }
        return;
    }
    const int64_t p = pk.p;
    const double sq = sqrt(pk.dp);
    if (threadIdx.x < 64) {
        const unsigned long long hit = __ballot((int)threadIdx.x < nc && cl == p);
        const unsigned long long hit2 = __ballot((int)threadIdx.x + 64 < nc && cl2 == p);
        if (threadIdx.x == 0) {
            int sl = hit ? __ffsll((long long)hit) - 1 : (hit2 ? 64 + __ffsll((long long)hit2) - 1 : -1);
            // large path (sov set): R holds the speculated steps' columns only, by step
            if (sl >= 0 && sov) sl = spec_column(sov, sl);
            sslot = sl;
        }
    }
    __syncthreads();
    const int slot = sslot;                              // the pivot's column of R, or -1
    // this row's entry of the pivot column (residual from the look-ahead pass on a hit),
    // issued before the pivot-row gather so the two loads overlap
    double cfin = 0.0;
    if (threadIdx.x < NR && If < cp.npairs && m_old != 1 && If != p) {
        if (slot >= 0) {
            cfin = R[(int64_t)slot * ldr + If];
        } else if constexpr (DENSE) {
            cfin = V[p * ldv + If];
        } else {
            cfin = eri_pp(pt.p[If], pt.Px[If], pt.Py[If], pt.Pz[If], pt.K[If], pt.p[p], pt.Px[p], pt.Py[p],
                          pt.Pz[p], pt.K[p]);
        }
    }
    double acc[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[v] = 0.0;
    if (slot >= 0) {
        // hit: subtract the vectors made since the block start (prefetched first)
        for (int64_t c0 = k0; c0 < k; c0 += CD_PCHUNK) {
            const int nj = (int)min((int64_t)CD_PCHUNK, k - c0);
            __syncthreads();
            for (int t = threadIdx.x; t < nj; t += CD_NT) sp[t] = L[(c0 + t) * ldl + p];
            __syncthreads();
            if (rows_ok) {
                int j = jg;
                if (c0 == k0) {
#pragma unroll
                    for (int m = 0; m < NPF; ++m, j += JG)
                        if (j < nj)
#pragma unroll
                            for (int v = 0; v < VW; ++v) acc[v] = fma(pf[m][v], sp[j], acc[v]);
                }
                for (; j < nj; j += JG) {
                    const double *Lp = L + (c0 + j) * ldl + I0;
#pragma unroll
                    for (int v = 0; v < VW; ++v) acc[v] = fma(Lp[v], sp[j], acc[v]);
                }
            }
        }
    } else {
        // miss (or no look-ahead): subtract all earlier vectors
        for (int64_t c0 = 0; c0 < k; c0 += CD_PCHUNK) {
            const int nj = (int)min((int64_t)CD_PCHUNK, k - c0);
            __syncthreads();
            for (int t = threadIdx.x; t < nj; t += CD_NT) sp[t] = L[(c0 + t) * ldl + p];
            __syncthreads();
            if (rows_ok) {
                const double *Lp = L + c0 * ldl + I0;
                int j = jg;
                if constexpr (VW == 2) {
                    double b0 = 0.0, b1 = 0.0;
                    for (; j + 3 * JG < nj; j += 4 * JG) {
                        double2 v0 = *reinterpret_cast<const double2 *>(Lp + (int64_t)j * ldl);
                        double2 v1 = *reinterpret_cast<const double2 *>(Lp + (int64_t)(j + JG) * ldl);
                        double2 v2 = *reinterpret_cast<const double2 *>(Lp + (int64_t)(j + 2 * JG) * ldl);
                        double2 v3 = *reinterpret_cast<const double2 *>(Lp + (int64_t)(j + 3 * JG) * ldl);
                        acc[0] = fma(v0.x, sp[j], acc[0]);
                        acc[1] = fma(v0.y, sp[j], acc[1]);
                        b0 = fma(v1.x, sp[j + JG], b0);
                        b1 = fma(v1.y, sp[j + JG], b1);
                        acc[0] = fma(v2.x, sp[j + 2 * JG], acc[0]);
                        acc[1] = fma(v2.y, sp[j + 2 * JG], acc[1]);
                        b0 = fma(v3.x, sp[j + 3 * JG], b0);
                        b1 = fma(v3.y, sp[j + 3 * JG], b1);
                    }
                    for (; j < nj; j += JG) {
                        double2 v = *reinterpret_cast<const double2 *>(Lp + (int64_t)j * ldl);
                        acc[0] = fma(v.x, sp[j], acc[0]);
                        acc[1] = fma(v.y, sp[j], acc[1]);
                    }
                    acc[0] += b0;
                    acc[1] += b1;
                } else {
                    double b0 = 0.0;
                    for (; j + JG < nj; j += 2 * JG) {
                        acc[0] = fma(Lp[(int64_t)j * ldl], sp[j], acc[0]);
                        b0 = fma(Lp[(int64_t)(j + JG) * ldl], sp[j + JG], b0);
                    }
                    for (; j < nj; j += JG) acc[0] = fma(Lp[(int64_t)j * ldl], sp[j], acc[0]);
                    acc[0] += b0;
                }
            }
        }
    }
#pragma unroll
    for (int v = 0; v < VW; ++v) red[jg][VW * rl + v] = acc[v];
    __syncthreads();
    const int w = 1 - r;
    if (threadIdx.x < NR) {                              // wave t: tile t of the block
        const int64_t I = If;
        bool active = false, nonpiv = false;
        double dn = 0.0;
        if (I < cp.npairs) {
            double l;
            unsigned char m = m_old;
            if (m == 1) {
                l = 0.0;                          // earlier pivot: exactly zero
                dn = d_old;
            } else if (I == p) {
                l = sq;                           // the pivot's own entry
                dn = 0.0;
                m = 1;
            } else {
                double s = 0.0;
#pragma unroll
                for (int g = 0; g < JG; ++g) s += red[g][threadIdx.x];
                l = (cfin - s) / sq;
                dn = d_old - l * l;
                nonpiv = true;
                active = m == 0;                  // m == 2: updated, never a pivot
            }
            L[k * ldl + I] = l;
            b.D[w][I] = dn;
            b.mask[w][I] = m;
        }
        const int64_t tile = (int64_t)blockIdx.x * TB + (threadIdx.x >> 6);
        if (tile < b.ntile) tile_record(b, w, sw, cp, tile, active, nonpiv, dn);
    }
    if (blockIdx.x == 0) {
        if (!b.flat && threadIdx.x < CD_NSUP) {
            b.smax[sz][threadIdx.x] = 0ull;
            b.smin[sz][threadIdx.x] = ~0ull;
        }
        if (threadIdx.x == 0) {
            piv[k] = p;
            st->k = k + 1;
            st->dmax = pk.mx;
            if (bsteps > 0 && slot < 0) st->nmiss += 1;
            // per row: 8 B per vector subtracted; D, mask read and written and L_k written
            // (34 B); the column entry from R or V (8 B) or the pair table (40 B, on demand)
            const double col = (slot >= 0 || DENSE) ? 8.0 : 40.0;
            st->bytes += (double)cp.npairs * (8.0 * (double)(k - (slot >= 0 ? k0 : 0)) + 26.0 + col);
        }
    }
}

// ---- speculative look-ahead block ---------------------------------------------
// After a look-ahead pass the candidates' residual columns are known, so the next
// steps restricted to the candidates form a small pivoted Cholesky problem
// (cd_spec_kernel, one wave, one candidate per lane; its first pivot is the true one,
// since the candidates hold the largest residuals and the pivot of step k0).
// cd_rows_kernel then makes those vectors for every row in one launch and checks every
// step: step j stands if no
// eligible row has a residual above the candidates' maximum, nor a residual in its tie
// window at a lower index than the chosen pivot (candidate rows cannot, since both
// kernels evaluate them with the same operations), nor any non-pivot row a residual
// below -psd_tol.  cd_commit_kernel commits the steps before the first one that fails, and
// the next block starts there.
struct SpecOut {
    int32_t nspec;           // speculated steps
    int32_t pad;
    uint64_t viol;           // bit j: step j does not stand (atomicOr by cd_rows_kernel)
    int64_t p[CD_SPEC_MAX];  // pivots
    int32_t slot[CD_SPEC_MAX];
    double sq[CD_SPEC_MAX], cmax[CD_SPEC_MAX], thr[CD_SPEC_MAX];
    double lpiv[CD_SPEC_MAX][CD_SPEC_MAX];   // lpiv[i][j] = L[k0+i][p_j], i < j
    int64_t k0;              // start step of the block
};

// Speculative blocks are chained on the device: each kernel of a block takes the block's
// start step from the state (the candidate, gather, pass and speculative kernels from
// st->k, which only the commit changes; the rows and commit kernels from so->k0) and the
// buffer parities from the steps made since entry, so the host can queue several blocks
// without reading anything back.  A block that can keep no step raises st->stall; the
// kernels of later blocks then return at once until the host has run one per-step launch.
__device__ __forceinline__ bool spec_idle(const CdState *st) { return st->done || st->stall; }

__device__ int spec_column(const SpecOut *so, int sl)
{
    int col = -1;
    for (int j = 0; j < so->nspec; ++j)
        if (so->slot[j] == sl) col = j;
    return col;
}

// steps of the block that stand: those before the first failed check
__device__ __forceinline__ int spec_keep(const SpecOut *so)
{
    const uint64_t v = so->viol;
    const int first = v ? __ffsll((long long)v) - 1 : 64;
    return min(so->nspec, first);
}

// LDS of the speculative block: the candidates' residual block, their entries of the speculated
// vectors and the per-step records
struct SpecLds {
    double Rcc[CD_NCAND][CD_NCAND + 1];           // Rcc[s][c] = R[s][cand_c]
    __align__(16) double Lt[64][CD_SPEC_MAX + 2]; // Lt[c][i] = L[k0+i][cand_c]
    int64_t spj[CD_SPEC_MAX];
    int ssj[CD_SPEC_MAX];
    double ssq[CD_SPEC_MAX], scm[CD_SPEC_MAX], sth[CD_SPEC_MAX];
};

// orders one wave's LDS accesses across lanes without a workgroup barrier: the wave's LDS
// operations so far have completed (lgkmcnt(0)) and the compiler moves no access across
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The speculative block, run by one wave (threads 0..63 of the workgroup; no workgroup
// barrier inside): lane c = candidate c, its column of the speculated vectors in registers
// (lc), the pivot's entries through LDS.  init() loads the block; step(j) forms step j (a
// no-op once the block has ended), with j a compile-time constant (unrolled callers);
// finish() writes every field of `out` but viol.
struct SpecWave {
    int64_t k0, I;
    int nmax, nspec, stop_at;
    bool have, alive;
    double d, dnc;
    unsigned char m;
    double lc[CD_SPEC_MAX];

    __device__ __forceinline__ void init(const CdBufs &b, const CdParams &cp, const int64_t *__restrict__ cand,
                                         const CdState *st, SpecLds &sm)
    {
        k0 = st->k;
        const int r = (int)((k0 - cp.nvec_in) & 1);
        nmax = (int)min((int64_t)cp.spec_len, cp.max_vec - k0);
        const int l = threadIdx.x;
        const int nc = st->ncand;
        have = l < nc;
        I = have ? cand[l] : -1;
        d = have ? b.D[r][I] : 0.0;
        m = have ? b.mask[r][I] : 1;
        // the candidates' 64 x 64 residual block (compact, written by the pass or, on the large
        // path, by cd_cc_kernel), 32 loads in flight
        {
            double v[CD_NCAND];
#pragma unroll
            for (int u = 0; u < CD_NCAND; ++u) v[u] = b.rc[u * CD_NCAND + l];
#pragma unroll
            for (int u = 0; u < CD_NCAND; ++u) sm.Rcc[u][l] = (have && u < nc) ? v[u] : 0.0;
        }
        if (l < CD_SPEC_MAX) {
            sm.spj[l] = -1;
            sm.ssj[l] = 0;
            sm.ssq[l] = sm.scm[l] = sm.sth[l] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < CD_SPEC_MAX; ++j) lc[j] = 0.0;
        nspec = 0;
        alive = true;                                     // uniform over the wave
        // steps whose tie threshold stays above every non-candidate residual stand for sure
        // (those residuals only decrease); speculation goes CD_SPEC_MARGIN steps past them
        dnc = st->dnc;
        stop_at = nmax;
    }

    __device__ __forceinline__ void step(int j, const CdParams &cp, SpecLds &sm)
    {
        const int l = threadIdx.x;
        if (j >= nmax) alive = false;
        if (!alive) return;
        const bool elig = have && m == 0;
        const double sql = sqrt(d);                                 // off the serial path
        const double cmax = okey_max(wave_max_key(elig ? okey(d) : 0ull));   // as fmax, on integer keys
        if (cmax == -INFINITY || cmax <= cp.delta) alive = false;   // termination: per-step path
        if (!alive) return;
        const double thr = cmax - tie_window(cmax, cp.tau);
        if (!(thr > dnc) && j + CD_SPEC_MARGIN < stop_at) stop_at = j + CD_SPEC_MARGIN;
        if (j >= stop_at) alive = false;
        if (!alive) return;
        // pivot: the lowest row index within the tie window; usually one lane is in it
        const unsigned long long win = __ballot(elig && d >= thr);
        int64_t pm;
        if (__popcll(win) == 1) {
            const int wl = __ffsll((long long)win) - 1;
            pm = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(I >> 32), wl) << 32) |
                           (uint32_t)__builtin_amdgcn_readlane((int)(I & 0xffffffff), wl));
        } else {
            pm = wave_min_i64_dpp((elig && d >= thr) ? I : INT64_MAX);
        }
        if (win == 0 || pm == INT64_MAX) alive = false;             // non-finite residuals
        if (!alive) return;
        const unsigned long long bs = __ballot(have && I == pm);
        const int slot = __ffsll((long long)bs) - 1;
        const double sq = readlane_f64(sql, slot);
        double c = sm.Rcc[slot][l];
        const double *lp = &sm.Lt[slot][0];                                         // L[k0+i][p_j]
#pragma unroll
        for (int i = 0; i < j; ++i) c = fma(-lc[i], lp[i], c);
        double lj;
        if (m == 1) {
            lj = 0.0;
        } else if (l == slot) {
            lj = sq;
            d = 0.0;
            m = 1;
        } else {
            lj = c / sq;
            d = fma(-lj, lj, d);
        }
        lc[j] = lj;
        sm.Lt[l][j] = lj;
        wave_lds_sync();
        if (l == 0) {
            sm.ssj[j] = slot;
            sm.ssq[j] = sq;
            sm.scm[j] = cmax;
            sm.sth[j] = thr;
            sm.spj[j] = pm;                   // step j is formed
        }
        nspec = j + 1;
    }

    // the per-step records (for the commit)
    __device__ __forceinline__ void records(const SpecLds &sm, SpecOut &out) const
    {
        const int l = threadIdx.x;
        if (l < CD_SPEC_MAX) {
            out.p[l] = sm.spj[l];
            out.slot[l] = sm.ssj[l];
            out.sq[l] = sm.ssq[l];
            out.cmax[l] = sm.scm[l];
            out.thr[l] = sm.sth[l];
        }
        if (l == 0) {
            out.nspec = nspec;
            out.pad = 0;
            out.k0 = k0;
        }
    }

    // the records and lpiv[i][j] = L[k0+i][p_j] = Lt[slot of p_j][i] (for the row updates)
    __device__ __forceinline__ void finish(const SpecLds &sm, SpecOut &out) const
    {
        const int l = threadIdx.x;
        for (int q = l; q < CD_SPEC_MAX * CD_SPEC_MAX; q += 64) {
            const int i = q / CD_SPEC_MAX, j = q % CD_SPEC_MAX;
            out.lpiv[i][j] = (i < j && j < nspec) ? sm.Lt[sm.ssj[j]][i] : 0.0;
        }
        records(sm, out);
    }
};

// copy of the record without viol (which the rows update while the copy may still run)
__device__ __forceinline__ void spec_publish(const SpecOut &ss, SpecOut *so)
{
    constexpr int n = (int)(sizeof(SpecOut) / 8);
    constexpr int iv = (int)(offsetof(SpecOut, viol) / 8);
    for (int q = threadIdx.x; q < n; q += blockDim.x)
        if (q != iv) ((int64_t *)so)[q] = ((const int64_t *)&ss)[q];
}

// The large path's speculative block over CD_NCAND_L = 128 candidates (more candidates keep more
// steps sure to stand: a block ends 8 steps after its tie threshold meets the largest residual
// outside the candidates), one wave: lane l holds candidates l and l + 64 (halves h = 0, 1) and
// their columns of the speculated vectors in registers; the pivot's earlier entries come from
// its lane (readlane), so the 128 x 128 residual block fits in LDS.  Every candidate takes
// SpecWave's operations in SpecWave's order.
struct SpecLds2 {
    double Rcc[CD_NCAND_L][CD_NCAND_L + 1];   // Rcc[s][c] = R[s][cand_c]
    int64_t spj[CD_SPEC_MAX];
    int ssj[CD_SPEC_MAX];
    double ssq[CD_SPEC_MAX], scm[CD_SPEC_MAX], sth[CD_SPEC_MAX];
};

struct SpecWave2 {
    int64_t k0, I[2];
    int nmax, nspec, stop_at, pj[2];
    bool have[2], alive;
    double d[2], dnc;
    unsigned char m[2];
    double lc[2][CD_SPEC_MAX];

    __device__ __forceinline__ void init(const CdBufs &b, const CdParams &cp, const int64_t *__restrict__ cand,
                                         const CdState *st, SpecLds2 &sm)
    {
        k0 = st->k;
        const int r = (int)((k0 - cp.nvec_in) & 1);
        nmax = (int)min((int64_t)cp.spec_len, cp.max_vec - k0);
        const int l = threadIdx.x;
        const int nc = st->ncand;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = l + 64 * h;
            have[h] = c < nc;
            I[h] = have[h] ? cand[c] : -1;
            d[h] = have[h] ? b.D[r][I[h]] : 0.0;
            m[h] = have[h] ? b.mask[r][I[h]] : 1;
            pj[h] = -1;
        }
        // the candidates' 128 x 128 residual block (compact, from cd_cc_kernel), 64 loads in flight
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u0 = 0; u0 < CD_NCAND_L; u0 += 64) {
                double v[64];
#pragma unroll
                for (int u = 0; u < 64; ++u) v[u] = b.rc[(u0 + u) * CD_NCAND_L + l + 64 * h];
#pragma unroll
                for (int u = 0; u < 64; ++u) sm.Rcc[u0 + u][l + 64 * h] = (have[h] && u0 + u < nc) ? v[u] : 0.0;
            }
        if (l < CD_SPEC_MAX) {
            sm.spj[l] = -1;
            sm.ssj[l] = 0;
            sm.ssq[l] = sm.scm[l] = sm.sth[l] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < CD_SPEC_MAX; ++j) lc[0][j] = lc[1][j] = 0.0;
        nspec = 0;
        alive = true;                                     // uniform over the wave
        dnc = st->dnc;
        stop_at = nmax;
    }

    __device__ __forceinline__ void step(int j, const CdParams &cp, SpecLds2 &sm)
    {
        const int l = threadIdx.x;
        if (j >= nmax) alive = false;
        if (!alive) return;
        bool elig[2];
        double sql[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            elig[h] = have[h] && m[h] == 0;
            sql[h] = sqrt(d[h]);                                      // off the serial path
        }
        const unsigned long long key = max(elig[0] ? okey(d[0]) : 0ull, elig[1] ? okey(d[1]) : 0ull);
        const double cmax = okey_max(wave_max_key(key));             // as fmax, on integer keys
        if (cmax == -INFINITY || cmax <= cp.delta) alive = false;    // termination: per-step path
        if (!alive) return;
        const double thr = cmax - tie_window(cmax, cp.tau);
        if (!(thr > dnc) && j + CD_SPEC_MARGIN < stop_at) stop_at = j + CD_SPEC_MARGIN;
        if (j >= stop_at) alive = false;
        if (!alive) return;
        // pivot: the lowest row index within the tie window; usually one candidate is in it
        const bool in0 = elig[0] && d[0] >= thr, in1 = elig[1] && d[1] >= thr;
        const unsigned long long w0 = __ballot(in0), w1 = __ballot(in1);
        int64_t pm;
        if (__popcll(w0) + __popcll(w1) == 1) {
            const bool hi = w1 != 0;
            const int wl = __ffsll((long long)(hi ? w1 : w0)) - 1;
            pm = readlane_i64(hi ? I[1] : I[0], wl);
        } else {
            pm = wave_min_i64_dpp(min(in0 ? I[0] : INT64_MAX, in1 ? I[1] : INT64_MAX));
        }
        if ((w0 | w1) == 0 || pm == INT64_MAX) alive = false;       // non-finite residuals
        if (!alive) return;
        const unsigned long long b0 = __ballot(have[0] && I[0] == pm), b1 = __ballot(have[1] && I[1] == pm);
        const int slot = b0 ? __ffsll((long long)b0) - 1 : 64 + __ffsll((long long)b1) - 1;
        const bool shi = slot >= 64;
        const int sl = slot & 63;
        const double sq = readlane_f64(shi ? sql[1] : sql[0], sl);
        double c[2] = {sm.Rcc[slot][l], sm.Rcc[slot][l + 64]};
#pragma unroll
        for (int i = 0; i < j; ++i) {
            const double lp = readlane_f64(shi ? lc[1][i] : lc[0][i], sl);   // L[k0+i][p_j]
            c[0] = fma(-lc[0][i], lp, c[0]);
            c[1] = fma(-lc[1][i], lp, c[1]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            double lj;
            if (m[h] == 1) {
                lj = 0.0;
            } else if (l + 64 * h == slot) {
                lj = sq;
                d[h] = 0.0;
                m[h] = 1;
                pj[h] = j;
            } else {
                lj = c[h] / sq;
                d[h] = fma(-lj, lj, d[h]);
            }
            lc[h][j] = lj;
        }
        if (l == 0) {
            sm.ssj[j] = slot;
            sm.ssq[j] = sq;
            sm.scm[j] = cmax;
            sm.sth[j] = thr;
            sm.spj[j] = pm;                   // step j is formed
        }
        nspec = j + 1;
    }

    // the records and lpiv[i][j] = L[k0+i][p_j] (i < j < nspec; 0 elsewhere): the candidate that
    // became the pivot of step j writes column j from its registers
    __device__ __forceinline__ void finish(const SpecLds2 &sm, SpecOut &out) const
    {
        const int l = threadIdx.x;
        for (int q = l; q < CD_SPEC_MAX * CD_SPEC_MAX; q += 64) (&out.lpiv[0][0])[q] = 0.0;
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int jj = pj[h];
            if (jj >= 0) {
#pragma unroll
                for (int i = 0; i < CD_SPEC_MAX; ++i)
                    if (i < jj) out.lpiv[i][jj] = lc[h][i];
            }
        }
        if (l < CD_SPEC_MAX) {
            out.p[l] = sm.spj[l];
            out.slot[l] = sm.ssj[l];
            out.sq[l] = sm.ssq[l];
            out.cmax[l] = sm.scm[l];
            out.thr[l] = sm.sth[l];
        }
        if (l == 0) {
            out.nspec = nspec;
            out.pad = 0;
            out.k0 = k0;
        }
    }
};

// (the large path: before the pass, which then forms the ns speculated columns in groups of 16)
__global__ __launch_bounds__(64) void cd_spec_kernel(CdBufs b, CdParams cp, const int64_t *__restrict__ cand,
                                                     CdState *st, SpecOut *so)
{
    __shared__ SpecLds2 sm;
    __shared__ SpecOut ss;
    if (spec_idle(st)) return;
    {
        SpecWave2 sw;
        sw.init(b, cp, cand, st, sm);
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < CD_SPEC_MAX; ++j) sw.step(j, cp, sm);
        wave_lds_sync();
        sw.finish(sm, ss);
    }
    wave_lds_sync();
    spec_publish(ss, so);
    if (threadIdx.x == 0) {
        so->viol = 0ull;
        const int cols = 16 * ((ss.nspec + 15) / 16);
        st->sumk0c += (double)ss.k0 * (double)cols;
        st->ncols += cols;
    }
}

// every row of the workgroup: the speculated vectors L[k0+j] (same operations as
// SpecWave), the residual at the end of each chunk of CD_SPEC_CHUNK steps (Dbuf[j][I] = D after
// vector j, for j = CD_SPEC_CHUNK - 1, 2 CD_SPEC_CHUNK - 1, ...; the commit replays the steps
// after the last such checkpoint from L) and the step checks
__device__ __forceinline__ void rows_body(const CdBufs &b, const CdParams &cp, const double *__restrict__ R,
                                          int64_t ldr, double *__restrict__ L, int64_t ldl,
                                          double *__restrict__ Dbuf, SpecOut *so, const SpecOut &ss,
                                          const double *__restrict__ lpg)
{
    const int ns = ss.nspec;
    const int64_t k0 = ss.k0;
    const int r = (int)((k0 - cp.nvec_in) & 1);
    const int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool ok = I < cp.npairs;
    unsigned char m = ok ? b.mask[r][I] : 1;
    double d = ok ? b.D[r][I] : 0.0;
    // right-looking within the row: cv[j] holds R[I][p_j] minus the terms of the vectors made
    // so far; once L_j[I] is known every later cv[j'] takes its term at once.  Each cv[j]
    // still receives its terms in the order i = 0, 1, ..., j-1 (the speculative wave's order),
    // but only one fused multiply-add per step stays on the serial path.
    double cv[CD_SPEC_MAX];
#pragma unroll
    for (int j = 0; j < CD_SPEC_MAX; ++j) cv[j] = (ok && j < ns) ? R[(int64_t)j * ldr + I] : 0.0;
    // Steps in chunks of CD_SPEC_CHUNK.  After each chunk a wave publishes the checks it saw
    // fail, and it stops once any step before the next chunk has failed anywhere (that read
    // is issued at the chunk's start and may be late, which only delays the stop): the
    // commit keeps the steps before the first failure, all of which every row has made.
    unsigned long long viol = 0ull, pub = 0ull;
    bool live = ok;
#pragma clang loop unroll(full)
    for (int c = 0; c < CD_SPEC_MAX / CD_SPEC_CHUNK; ++c) {
        const unsigned long long seen =
            c > 0 ? __hip_atomic_load(&so->viol, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
#pragma clang loop unroll(full)
        for (int u = 0; u < CD_SPEC_CHUNK; ++u) {
            const int j = c * CD_SPEC_CHUNK + u;
            if (j >= ns || !live) continue;
            if (m == 0 && (d > ss.cmax[j] || (d >= ss.thr[j] && I < ss.p[j]))) viol |= 1ull << j;
            if (m != 1 && d < -cp.psd_tol) viol |= 1ull << j;     // NOT_PSD is the per-step path's call
            double lj;
            if (m == 1) {
                lj = 0.0;
            } else if (I == ss.p[j]) {
                lj = ss.sq[j];
                d = 0.0;
                m = 1;
            } else {
                lj = cv[j] / ss.sq[j];
                d = fma(-lj, lj, d);
            }
            L[(k0 + j) * ldl + I] = lj;
            if (u == CD_SPEC_CHUNK - 1) Dbuf[(int64_t)j * cp.npairs + I] = d;
            if (m != 1) {
                // a pivot row (also the one made now) takes no further values; lpiv[j][j'] =
                // L_j[p_j'], 0 for j' >= ns
#pragma clang loop unroll(full)
                for (int jj = j + 1; jj < CD_SPEC_MAX; ++jj) cv[jj] = fma(-lj, lpg[j * CD_SPEC_MAX + jj], cv[jj]);
            }
        }
        // wave OR of the failed checks; new ones are published at once
        unsigned long long w = viol;
        for (int o = 32; o > 0; o >>= 1) w |= (unsigned long long)__shfl_xor((long long)w, o, 64);
        if (w & ~pub) {
            if ((threadIdx.x & 63) == 0) atomicOr((unsigned long long *)&so->viol, w);
            pub |= w;
        }
        const int next = (c + 1) * CD_SPEC_CHUNK;
        if ((seen | w) & (next >= 64 ? ~0ull : ((1ull << next) - 1))) live = false;
    }
}

__global__ __launch_bounds__(256) void cd_rows_kernel(CdBufs b, CdParams cp, const CdState *st,
                                                      const double *__restrict__ R, int64_t ldr, double *__restrict__ L,
                                                      int64_t ldl, double *__restrict__ Dbuf, SpecOut *so,
                                                      const double *__restrict__ lpg)
{
    __shared__ SpecOut ss;
    if (spec_idle(st)) return;
    // the record up to the pivots' vector entries, and its start step, into LDS (those entries,
    // wave-uniform operands, come through the scalar cache from lpg)
    constexpr int NW = (int)(offsetof(SpecOut, lpiv) / 8), NQ = (NW + 255) / 256;
    constexpr int KW = (int)(offsetof(SpecOut, k0) / 8);
    static_assert(offsetof(SpecOut, lpiv) % 8 == 0 && offsetof(SpecOut, k0) % 8 == 0, "record words");
    int64_t v[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int q = (int)threadIdx.x + 256 * i;
        v[i] = q < NW ? ((const int64_t *)so)[q] : q == NW ? ((const int64_t *)so)[KW] : 0;
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int q = (int)threadIdx.x + 256 * i;
        if (q < NW) ((int64_t *)&ss)[q] = v[i];
        else if (q == NW) ((int64_t *)&ss)[KW] = v[i];
    }
    __syncthreads();
    rows_body(b, cp, R, ldr, L, ldl, Dbuf, so, ss, lpg);
}

// One row of the lockstep kernel, left-looking: step j forms L_j[I] = (R[I][p_j] - sum_{i<j}
// L_i[I] L_i[p_j]) / sqrt(D_j), the terms in the order i = 0, 1, ... with the same fused
// multiply-adds as SpecWave::step, so the candidates' rows agree with the speculative wave bit
// for bit; D_j[I] and the checks of step j as the right-looking row update.
struct RowWave {
    int64_t I;
    bool ok;
    unsigned char m;
    double d;
    unsigned long long viol;
    double lr[CD_SPEC_MAX];   // L_i[I], i < j

    __device__ __forceinline__ void step(int j, const CdParams &cp, const SpecLds &sm, double rpj, double *__restrict__ L,
                                         int64_t ldl, int64_t k0, double *__restrict__ Dbuf)
    {
        const int64_t pj = sm.spj[j];
        const int slot = sm.ssj[j];
        const double sq = sm.ssq[j];
        if (m == 0 && (d > sm.scm[j] || (d >= sm.sth[j] && I < pj))) viol |= 1ull << j;
        if (m != 1 && d < -cp.psd_tol) viol |= 1ull << j;         // NOT_PSD is the per-step path's call
        double lj;
        if (m == 1) {
            lj = 0.0;
        } else if (I == pj) {
            lj = sq;
            d = 0.0;
            m = 1;
        } else {
            double c = rpj;
            const double *lp = &sm.Lt[slot][0];
#pragma unroll
            for (int i = 0; i < j; ++i) c = fma(-lr[i], lp[i], c);
            lj = c / sq;
            d = fma(-lj, lj, d);
        }
        lr[j] = lj;
        if (ok) {
            L[(k0 + j) * ldl + I] = lj;
            if (j % CD_SPEC_CHUNK == CD_SPEC_CHUNK - 1) Dbuf[(int64_t)j * cp.npairs + I] = d;
        }
    }
};

// The speculative block and the row updates in lockstep (grids of at most CD_FUSE_MAXBLK
// workgroups of CD_LS_ROWS rows): wave 0 of every workgroup forms the speculative block (the
// same operations on the same data, so every workgroup holds the same record), and the other
// waves update the workgroup's rows one step behind it, left-looking, so their work runs while
// wave 0 forms the next step; a workgroup barrier per step hands each step over.  The rows'
// candidate columns are staged in LDS first (R[I][p_j] is known only when p_j is).  Workgroup 0
// publishes the records for the commit; the candidate kernel has cleared the failure mask.
constexpr int CD_LS_ROWS = 128;

struct LockLds {
    SpecLds sp;
    double Rs[CD_NCAND][CD_LS_ROWS];   // Rs[c][t] = R[c][row t of the workgroup]
};

__global__ __launch_bounds__(64 + CD_LS_ROWS, 1) void cd_lockstep_kernel(CdBufs b, CdParams cp,
                                                                       const int64_t *__restrict__ cand,
                                                                       const CdState *st, const double *__restrict__ R,
                                                                       int64_t ldr, double *__restrict__ L, int64_t ldl,
                                                                       double *__restrict__ Dbuf, SpecOut *so)
{
    __shared__ LockLds sh;
    if (spec_idle(st)) return;
    const bool spec = threadIdx.x < 64;
    const int t = (int)threadIdx.x - 64;                 // row of the workgroup (row waves)
    SpecWave sw;
    RowWave rw;
    int64_t k0 = 0;
    if (spec) {
        sw.init(b, cp, cand, st, sh.sp);
    } else {
        k0 = st->k;
        const int r = (int)((k0 - cp.nvec_in) & 1);
        const int nc = st->ncand;
        rw.I = (int64_t)blockIdx.x * CD_LS_ROWS + t;
        rw.ok = rw.I < cp.npairs;
        rw.m = rw.ok ? b.mask[r][rw.I] : 1;
        rw.d = rw.ok ? b.D[r][rw.I] : 0.0;
        rw.viol = 0ull;
#pragma unroll
        for (int j = 0; j < CD_SPEC_MAX; ++j) rw.lr[j] = 0.0;
        // all 64 loads in flight, then the LDS stores
        double v[CD_NCAND];
#pragma unroll
        for (int c = 0; c < CD_NCAND; ++c) v[c] = R[(int64_t)c * ldr + (rw.ok ? rw.I : 0)];
#pragma unroll
        for (int c = 0; c < CD_NCAND; ++c) sh.Rs[c][t] = (rw.ok && c < nc) ? v[c] : 0.0;
    }
    __syncthreads();
    // iteration j: wave 0 forms step j, the row waves make step j - 1; once a step is missing
    // (read after the barrier, so the same in every wave) the rest is skipped
    bool ended = false;
#pragma clang loop unroll(full)
    for (int j = 0; j <= CD_SPEC_MAX; ++j) {
        if (ended) continue;
        if (spec) {
            if (j < CD_SPEC_MAX) sw.step(j, cp, sh.sp);
        } else if (j > 0) {
            rw.step(j - 1, cp, sh.sp, sh.Rs[sh.sp.ssj[j - 1]][t], L, ldl, k0, Dbuf);
        }
        __syncthreads();
        ended = j == CD_SPEC_MAX || sh.sp.spj[j] < 0;
    }
    if (!spec) {
        unsigned long long w = rw.viol;
        for (int o = 32; o > 0; o >>= 1) w |= (unsigned long long)__shfl_xor((long long)w, o, 64);
        if (w && (threadIdx.x & 63) == 0) atomicOr((unsigned long long *)&so->viol, w);
    } else if (blockIdx.x == 0) {
        sw.records(sh.sp, *so);
    }
}

// empty the two super-tile key buffers that the commit and the step after it fill
// (hierarchical search path, before the commit)
__global__ void reset_super_kernel(CdBufs b, CdParams cp, const CdState *st, const SpecOut *so)
{
    if (spec_idle(st)) return;
    const int nc = spec_keep(so);
    if (nc == 0) return;
    const int64_t s = so->k0 + nc - cp.nvec_in;
    const int b1 = (int)(s % 3), b2 = (int)((s + 1) % 3);
    const int t = threadIdx.x;
    if (t < CD_NSUP) {
        b.smax[b1][t] = 0ull;
        b.smin[b1][t] = ~0ull;
        b.smax[b2][t] = 0ull;
        b.smin[b2][t] = ~0ull;
    }
}

// commit the first nc speculated steps: residuals, pivot marks and tile records into the
// buffers of parity w (the step k0 + nc reads them), pivots and the state
__global__ __launch_bounds__(256) void cd_commit_kernel(CdBufs b, CdParams cp, const double *__restrict__ Dbuf,
                                                        const double *__restrict__ L, int64_t ldl,
                                                        const SpecOut *so, CdState *st, int64_t *__restrict__ piv,
                                                        uint64_t *mail)
{
    if (spec_idle(st)) return;
    const int nc = spec_keep(so);
    if (nc == 0) {                               // nothing stands: one per-step launch next
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->stall = 1;
            const int64_t nb = st->nblk + 1;
            st->nblk = nb;
            if (mail) __hip_atomic_store(mail, mb_word(nb, 1, st->k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return;
    }
    __shared__ int64_t sp[CD_SPEC_MAX];
    const int64_t k0 = so->k0, s = k0 - cp.nvec_in;
    const int r = (int)(s & 1), w = (int)((s + nc) & 1), sw = (int)((s + nc) % 3);
    const int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool ok = I < cp.npairs;
    // D after the kept steps: the rows kernel's last checkpoint before step nc (or D at the block
    // start), then the steps after it replayed from L with the rows kernel's own operations
    const int jc = (nc / CD_SPEC_CHUNK) * CD_SPEC_CHUNK;     // steps covered by the checkpoint
    unsigned char m = ok ? b.mask[r][I] : 1;
    double d = 0.0, lv[CD_SPEC_CHUNK];
    if (ok) {
        d = jc > 0 ? Dbuf[(int64_t)(jc - 1) * cp.npairs + I] : b.D[r][I];
#pragma unroll
        for (int u = 0; u < CD_SPEC_CHUNK; ++u) lv[u] = jc + u < nc ? L[(k0 + jc + u) * ldl + I] : 0.0;
    }
    // the block's pivots, loaded once (a loop of loads would wait on each)
    if ((int)threadIdx.x < CD_SPEC_MAX) sp[threadIdx.x] = (int)threadIdx.x < nc ? so->p[threadIdx.x] : -1;
    __syncthreads();
    if (ok) {
        for (int j = 0; j < jc; ++j)
            if (I == sp[j]) m = 1;
#pragma unroll
        for (int u = 0; u < CD_SPEC_CHUNK; ++u) {
            const int j = jc + u;
            if (j >= nc || m == 1) continue;
            if (I == sp[j]) {
                d = 0.0;
                m = 1;
            } else {
                d = fma(-lv[u], lv[u], d);
            }
        }
        b.D[w][I] = d;
        b.mask[w][I] = m;
    }
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile < b.ntile) tile_record(b, w, sw, cp, tile, ok && m == 0, ok && m != 1, d);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int j = 0; j < nc; ++j) piv[k0 + j] = so->p[j];
        st->k = k0 + nc;
        st->dmax = so->cmax[nc - 1];
        st->nspec += nc;
        st->sumk0s += (double)k0 * (double)nc;
        st->sumwin += 0.5 * (double)nc * (double)(nc - 1);
        const int64_t nb = st->nblk + 1;
        st->nblk = nb;
        if (mail) __hip_atomic_store(mail, mb_word(nb, 0, k0 + nc), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Boundary of the top `want` nonzero keys held in registers (KPT per thread, 0 = no key):
// four 8-bit radix passes over the key bits; returns the top 32 bits of the boundary key.
// Every thread of the block calls it.
template <int NT, int KPT>
__device__ unsigned long long radix_boundary(const unsigned long long (&u)[KPT], int want, unsigned int *hist,
                                             unsigned long long *s_prefix, int *s_need)
{
    if (threadIdx.x == 0) {
        *s_prefix = 0ull;
        *s_need = want;
    }
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 56 - 8 * pass;
        for (int q = threadIdx.x; q < 256; q += NT) hist[q] = 0;
        __syncthreads();
        const unsigned long long prefix = *s_prefix;
#pragma unroll
        for (int e = 0; e < KPT; ++e) {
            if (u[e] == 0ull) continue;
            if (pass > 0 && (u[e] >> (shift + 8)) != prefix) continue;
            atomicAdd(&hist[(u[e] >> shift) & 0xFF], 1u);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            // digit q = the largest with (count of keys >= q) >= need; need -= count above q.
            // Lane l holds bins 4l..4l+3; suffix sums over lanes locate q's lane.
            const int l = threadIdx.x, need = *s_need;
            const int h0 = hist[4 * l], h1 = hist[4 * l + 1], h2 = hist[4 * l + 2], h3 = hist[4 * l + 3];
            const int own = h0 + h1 + h2 + h3;
            int S = own;                                   // sum over lanes >= l
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_down(S, o, 64);
                if (l + o < 64) S += v;
            }
            const unsigned long long ok = __ballot(S >= need);
            if (ok == 0ull) {
                if (l == 0) {                              // fewer keys than wanted: take all
                    *s_prefix = prefix << 8;
                    *s_need = need - (S - h0);
                }
            } else if (l == 63 - __clzll((long long)ok)) {
                int rem = need - (S - own);
                int q;
                if (h3 >= rem) q = 3;
                else if (h2 >= (rem -= h3)) q = 2;
                else if (h1 >= (rem -= h2)) q = 1;
                else { rem -= h1; q = 0; }
                *s_prefix = (prefix << 8) | (unsigned long long)(4 * l + q);
                *s_need = rem;
            }
        }
        __syncthreads();
    }
    return *s_prefix;
}

// Writes the ids of the top `want` keys to out[] in a deterministic order (keys above the
// boundary first, then boundary keys, each by id); ids are threadIdx.x * KPT + e.  Returns
// how many were written.
template <int NT, int KPT, typename F>
__device__ int select_top(const unsigned long long (&u)[KPT], int want, unsigned int *hist,
                          unsigned long long *s_prefix, int *s_need, int *shs, F &&emit,
                          unsigned long long *s_rest)
{
    const unsigned long long thr = radix_boundary<NT, KPT>(u, want, hist, s_prefix, s_need);
    int na = 0, nbd = 0;
#pragma unroll
    for (int e = 0; e < KPT; ++e) {
        if (u[e] == 0ull) continue;
        if ((u[e] >> 32) > thr) ++na;
        else if ((u[e] >> 32) == thr) ++nbd;
    }
    int tot_a, tot_b;
    int ia = block_excl_scan<NT>(na, shs, &tot_a);
    int ib = block_excl_scan<NT>(nbd, shs, &tot_b);
    const int nabove = min(tot_a, want);
    unsigned long long rest = 0ull;             // largest key not selected
#pragma unroll
    for (int e = 0; e < KPT; ++e) {
        if (u[e] == 0ull) continue;
        const int id = threadIdx.x * KPT + e;
        if ((u[e] >> 32) > thr) {
            if (ia < want) emit(ia, id);
            else rest = max(rest, u[e]);
            ++ia;
        } else if ((u[e] >> 32) == thr) {
            if (nabove + ib < want) emit(nabove + ib, id);
            else rest = max(rest, u[e]);
            ++ib;
        } else {
            rest = max(rest, u[e]);
        }
    }
    // block maximum of rest (wave, then the waves through LDS)
    for (int o = 32; o > 0; o >>= 1) rest = max(rest, (unsigned long long)__shfl_xor((long long)rest, o, 64));
    if (threadIdx.x == 0) *s_rest = 0ull;
    __syncthreads();
    if ((threadIdx.x & 63) == 0 && rest) atomicMax(s_rest, rest);
    __syncthreads();
    return min(nabove + tot_b, want);
}

// Look-ahead block start (one block): candidates = this step's pivot, then the rows with
// the largest residual diagonals (NC - 1 of them; NC = CD_NCAND, or CD_NCAND_L on the large
// path).  Those rows lie in the NC tiles with the largest tile maxima, so the tiles are selected first (keys from the tile
// records), then the rows of those tiles; both selections are exact top-k on the IEEE
// bits (ties at the boundary by lowest position), deterministic.
// (NT threads, CD_AUX_NT in use: 512 measured far worse for 128 candidates, its 16 tile and 16
// row keys per thread spilling)
template <int NC, int NT>
__global__ __launch_bounds__(NT) void cd_cand_kernel(CdBufs b, CdParams cp, int r, int sr, int64_t k,
                                                     CdState *st, int64_t *__restrict__ cand, SpecOut *so)
{
    constexpr int TK = CD_CAND_MAXTILE / NT;                  // tile keys per thread
    constexpr int RK = NC * CD_TILE / NT;                     // row keys per thread
    static_assert(RK * NT == NC * CD_TILE && TK * NT == CD_CAND_MAXTILE && NC <= 128 && NT <= 1024 && NT > NC,
                  "candidate selection shape");
    __shared__ PickShared psh;
    __shared__ unsigned int hist[256];
    __shared__ unsigned long long s_prefix;
    __shared__ int s_need;
    __shared__ int shs[NT / 64 + 1];
    __shared__ int64_t stile[NC];
    __shared__ unsigned long long s_rest;
    if (st->done) return;
    const bool chained = k < 0;                  // speculative block: position from the state
    if (chained) {
        if (st->stall) return;
        if (threadIdx.x == 0) so->viol = 0ull;   // no check of this block has failed yet
        k = st->k;
        const int64_t s = k - cp.nvec_in;
        r = (int)(s & 1);
        sr = (int)(s % 3);
    }
    // the previous block's rows leave the slot map
    const int nmap = st->nmap;
    if ((int)threadIdx.x < nmap) b.slot[cand[threadIdx.x]] = -1;
    __syncthreads();
    const Pick pk = cd_pick<NT>(b, r, sr, cp, k, psh);
    if (pk.status != PICK_GO) {                  // the step kernel records the termination
        if (threadIdx.x == 0) {
            st->ncand = 0;                       // gather and pass have nothing to do
            st->nmap = 0;
        }
        return;
    }
    const int64_t p = pk.p;
    const TileStat *ts = b.ts[r];
    unsigned long long u[TK];
#pragma unroll
    for (int e = 0; e < TK; ++e) {
        const int64_t t = (int64_t)threadIdx.x * TK + e;
        const double v = t < b.ntile ? ts[t].mx : 0.0;
        u[e] = v > 0.0 ? (unsigned long long)__double_as_longlong(v) : 0ull;
    }
    const int ntsel = select_top<NT, TK>(u, NC, hist, &s_prefix, &s_need, shs,
                                                 [&](int pos, int id) { stile[pos] = id; }, &s_rest);
    const unsigned long long rest_tile = s_rest;  // largest maximum of a tile not selected
    __syncthreads();
    unsigned long long v[RK];
#pragma unroll
    for (int e = 0; e < RK; ++e) {
        const int i = threadIdx.x * RK + e;
        const int slot = i / CD_TILE;
        v[e] = 0ull;
        if (slot < ntsel) {
            const int64_t I = stile[slot] * CD_TILE + i % CD_TILE;
            if (I < cp.npairs && I != p && !b.mask[r][I]) {
                const double d = b.D[r][I];
                if (d > 0.0) v[e] = (unsigned long long)__double_as_longlong(d);
            }
        }
    }
    const int nrow = select_top<NT, RK>(v, NC - 1, hist, &s_prefix, &s_need, shs, [&](int pos, int id) {
        cand[1 + pos] = stile[id / CD_TILE] * CD_TILE + id % CD_TILE;
    }, &s_rest);
    // every eligible row outside the candidates is at most the larger of the two rests (keys
    // are the bits of positive doubles; 0 = none)
    const unsigned long long rest = max(rest_tile, s_rest);
    if (threadIdx.x == 0) cand[0] = p;
    __syncthreads();
    if ((int)threadIdx.x < 1 + nrow) b.slot[cand[threadIdx.x]] = (signed char)threadIdx.x;
    if (threadIdx.x == 0) {
        st->ncand = 1 + nrow;
        st->nmap = 1 + nrow;
        st->dnc = rest ? __longlong_as_double((long long)rest) : 0.0;
        if (chained) {
            st->npass += 1;
            st->sumk0 += (double)k;
        }
    }
}

// Base of the candidate residual columns: R[c][I] = V[I][cand_c] for the candidates c of group
// grp (CD_CG columns), rows I of x-block bx; the pass then subtracts the projection on the
// earlier vectors.  Each thread loads its pair's data once and evaluates its row of the group's
// columns (the pair table is read once per group, not once per column).
template <bool DENSE>
__device__ __forceinline__ void candcol_body(const PairTable &pt, const double *__restrict__ V, int64_t ldv,
                                             int64_t npairs, const int64_t *__restrict__ cand, int nc, int grp,
                                             int64_t bx, double *__restrict__ R, int64_t ldr)
{
    const int64_t I = bx * blockDim.x + threadIdx.x;
    if (I >= npairs) return;
    const int c0 = grp * CD_CG, c1 = min(nc, c0 + CD_CG);
    if constexpr (DENSE) {
        for (int c = c0; c < c1; ++c) R[(int64_t)c * ldr + I] = V[cand[c] * ldv + I];
    } else {
        const double p = pt.p[I], Px = pt.Px[I], Py = pt.Py[I], Pz = pt.Pz[I], K = pt.K[I];
        for (int c = c0; c < c1; ++c) {
            const int64_t q = cand[c];
            R[(int64_t)c * ldr + I] = eri_pp(p, Px, Py, Pz, K, pt.p[q], pt.Px[q], pt.Py[q], pt.Pz[q], pt.K[q]);
        }
    }
}

// P[j][c] = L[j][cand_c], j < k0, c < nc (stride over the entries from block b of nb);
// rows k0 .. k0 + CD_PASS_ZROWS - 1 are zero (the pass reads them for vectors past k0)
template <int NC = CD_NCAND>
__device__ __forceinline__ void gather_body(const double *__restrict__ L, int64_t ldl, int64_t k0, int nc,
                                            const int64_t *__restrict__ cand, double *__restrict__ P, int64_t b,
                                            int64_t nb)
{
    const int64_t ne = (k0 + CD_PASS_ZROWS) * NC;
    for (int64_t e = b * blockDim.x + threadIdx.x; e < ne; e += nb * blockDim.x) {
        const int64_t j = e / NC;
        const int c = (int)(e % NC);
        P[e] = (j < k0 && c < nc) ? L[j * ldl + cand[c]] : 0.0;
    }
}

template <bool DENSE>
__global__ void cd_candcol_kernel(PairTable pt, const double *__restrict__ V, int64_t ldv, int64_t npairs,
                                  const CdState *__restrict__ st, const int64_t *__restrict__ cand,
                                  double *__restrict__ R, int64_t ldr)
{
    const int grp = blockIdx.y, nc = st->ncand;
    if (spec_idle(st) || grp * CD_CG >= nc) return;
    candcol_body<DENSE>(pt, V, ldv, npairs, cand, nc, grp, blockIdx.x, R, ldr);
}

// the gather alone; k0 < 0: the start of the current speculative block
template <int NC>
__global__ void cd_gather_kernel(const double *__restrict__ L, int64_t ldl, int64_t k0, const CdState *__restrict__ st,
                                 const int64_t *__restrict__ cand, double *__restrict__ P)
{
    if (spec_idle(st) || st->ncand == 0) return;
    gather_body<NC>(L, ldl, k0 < 0 ? st->k : k0, st->ncand, cand, P, blockIdx.x, gridDim.x);
}

// one launch for both, at the start of the current speculative block (they need only the
// candidate list): block rows y < CD_NCG evaluate the columns of candidate group y, the rows after
// them gather (enough of them that each thread gathers at most one entry: a strided loop waits on
// each of its loads)
template <bool DENSE>
__global__ void cd_candcol_gather_kernel(PairTable pt, const double *__restrict__ V, int64_t ldv, int64_t npairs,
                                         const CdState *__restrict__ st, const int64_t *__restrict__ cand,
                                         double *__restrict__ R, int64_t ldr, const double *__restrict__ L,
                                         int64_t ldl, double *__restrict__ P)
{
    if (spec_idle(st)) return;
    const int nc = st->ncand;
    if ((int)blockIdx.y >= CD_NCG) {            // gather: rows CD_NCG.. of the grid, one entry per thread
        const int64_t gb = (int64_t)(blockIdx.y - CD_NCG) * gridDim.x + blockIdx.x;
        const int64_t nb = (int64_t)(gridDim.y - CD_NCG) * gridDim.x;
        if (nc > 0) gather_body(L, ldl, st->k, nc, cand, P, gb, nb);
        return;
    }
    if ((int)blockIdx.y * CD_CG >= nc) return;
    candcol_body<DENSE>(pt, V, ldv, npairs, cand, nc, blockIdx.y, blockIdx.x, R, ldr);
}

// R[c][I] -= sum_{j<k0} L[j][I] P[j][c] for all candidates (R holds V[I][cand_c]), one
// read of L.
// Block = 64 rows; its 4 waves split the vectors (k-steps of 4) into four contiguous
// ranges and each forms the whole 64 x 64 block over its range with 16 f64 MFMA tiles
// (v_mfma_f64_16x16x4f64: A = L, lane l: row l%16 of a 16-row group, vector l/16;
// B = P, lane l: candidate l%16 of a 16-candidate group, vector l/16).  Both operands go
// straight from memory to registers (P is small and stays in L2) through a ring of
// CD_PASS_D k-steps, so the main loop has no LDS traffic and no barrier.  The four
// partial blocks are then summed through LDS in a fixed order, (w0 + w2) + (w1 + w3).
// Every load is issued from a clamped in-range address; vectors past a wave's range read a
// zero row of P and add exactly 0.  L and P are deliberately not __restrict__: the
// compiler may then not move their loads across the compiler barrier that keeps the ring
// ahead of the MFMAs.
// W16 (even ldl, 16-byte aligned L): every lane loads two adjacent rows of L and two adjacent
// candidates of P at once (16 bytes), half the load instructions of one row each; the MFMA
// row (column) r16 of block 2u + h is then tile row (candidate) 32u + 2 r16 + h.  Each output
// takes the same products in the same order either way.
// ERI: R holds nothing yet; the epilogue evaluates the candidate columns' integrals V[I][cand_c]
// itself (the values the column kernel would have stored, bit for bit), which saves writing R and
// reading it back (2 x 8 x npairs x 64 bytes per block).
template <bool W16, bool ERI>
__global__ __launch_bounds__(256, 2) void cd_pass_kernel(const double *L, int64_t ldl, int64_t npairs,
                                                         int64_t k0, const CdState *__restrict__ st,
                                                         const double *P, double *__restrict__ R,
                                                         int64_t ldr, const signed char *__restrict__ slotmap,
                                                         double *__restrict__ rc, PairTable pt,
                                                         const int64_t *__restrict__ cand)
{
    constexpr int D = CD_PASS_D;
    __shared__ double red[2][CD_NCAND][CD_TILE];           // red[slot][cand][row ^ cand]
    if (spec_idle(st) || st->ncand == 0) return;
    if (k0 < 0) k0 = st->k;                                // speculative block: from the state
    const int nc = st->ncand;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
    const int64_t tile0 = (int64_t)blockIdx.x * CD_TILE;
    int64_t rowL[4];
    if constexpr (W16) {
        // pair starts are even and at most ldl - 2 (ldl even): a start past npairs - 1 only
        // feeds rows that are never written
#pragma unroll
        for (int u = 0; u < 2; ++u) rowL[u] = min(tile0 + 32 * u + 2 * r16, ldl - 2);
    } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) rowL[m] = min(tile0 + 16 * m + r16, npairs - 1);
    }
    const int64_t ks = (k0 + 3) / 4;                       // k-steps
    const int64_t s0 = ks * w / 4, s1 = ks * (w + 1) / 4;
    const int64_t jz = 4 * ks;                             // a zero row of P (k0 <= jz < k0 + 4)
    const int64_t jl_max = k0 > 0 ? k0 - 1 : 0;
    doublex4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = doublex4{0.0, 0.0, 0.0, 0.0};
    double a[D][4], b[D][4];
    auto load = [&](int64_t s, double *as, double *bs) {
        const int64_t j = 4 * s + g;
        const int64_t jl = min(j, jl_max);                 // L row: finite
        const int64_t jp = s < s1 ? j : jz;                // P row: zero past the range
        if constexpr (W16) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double2 x = *reinterpret_cast<const double2 *>(L + jl * ldl + rowL[u]);
                as[2 * u] = x.x;
                as[2 * u + 1] = x.y;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double2 y = *reinterpret_cast<const double2 *>(P + jp * CD_NCAND + 32 * u + 2 * r16);
                bs[2 * u] = y.x;
                bs[2 * u + 1] = y.y;
            }
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) as[m] = L[jl * ldl + rowL[m]];
#pragma unroll
            for (int n = 0; n < 4; ++n) bs[n] = P[jp * CD_NCAND + 16 * n + r16];
        }
    };
    // tile row of MFMA block m, lane row q (0..15), and candidate of block n, lane column r
    auto trow = [&](int m, int q) { return W16 ? 32 * (m >> 1) + 2 * q + (m & 1) : 16 * m + q; };
    auto tcol = [&](int n, int r) { return W16 ? 32 * (n >> 1) + 2 * r + (n & 1) : 16 * n + r; };
    if (k0 > 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            load(s0 + i, a[i], b[i]);                // slot order, as in the loop
            __builtin_amdgcn_sched_barrier(0);
        }
        for (int64_t s = s0; s < s1; s += D) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < 4; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][m], b[i][n], acc[m][n], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                asm volatile("" ::: "memory");       // the refill stays behind the MFMAs of its slot
                load(s + i + D, a[i], b[i]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // fixed-order sum of the four partial blocks, (w0 + w2) + (w1 + w3); the lane holds tile
    // rows trow(m, g + 4e) of candidate tcol(n, r16); LDS entry (c, row) sits at c * 64 + (row ^ c)
    auto put = [&](int slot) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = tcol(n, r16), row = trow(m, g + 4 * e);
                    red[slot][c][row ^ c] = acc[m][n][e];
                }
    };
    auto add = [&](int slot) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = tcol(n, r16), row = trow(m, g + 4 * e);
                    acc[m][n][e] += red[slot][c][row ^ c];
                }
    };
    // R[c][I] -= block[I][c], all 256 threads, consecutive threads on consecutive rows (each
    // thread keeps one row); a candidate row also goes to the compact block rc.  The row's data
    // is loaded under the reduction.
    const int row = threadIdx.x % CD_TILE;
    const int64_t I = tile0 + row;
    const int sl = I < npairs ? slotmap[I] : -1;
    double ip = 0.0, ipx = 0.0, ipy = 0.0, ipz = 0.0, ik = 0.0;
    if (ERI && I < npairs) {
        ip = pt.p[I];
        ipx = pt.Px[I];
        ipy = pt.Py[I];
        ipz = pt.Pz[I];
        ik = pt.K[I];
    }
    if (w >= 2) put(w - 2);
    __syncthreads();
    if (w < 2) add(w);
    __syncthreads();
    if (w < 2) put(w);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CD_TILE * CD_NCAND / 256; ++q) {
        const int c = (threadIdx.x + 256 * q) / CD_TILE;
        if (c < nc && I < npairs) {
            double base;                                           // V[I][cand_c]
            if constexpr (ERI) {
                const int64_t qc = cand[c];
                base = eri_pp(ip, ipx, ipy, ipz, ik, pt.p[qc], pt.Px[qc], pt.Py[qc], pt.Pz[qc], pt.K[qc]);
            } else {
                base = R[(int64_t)c * ldr + I];
            }
            const double v = base - (red[0][c][row ^ c] + red[1][c][row ^ c]);
            R[(int64_t)c * ldr + I] = v;
            if (sl >= 0) rc[c * CD_NCAND + sl] = v;
        }
    }
}

// Large path, step 1 of a speculative block: the candidates' own residual block before any
// full-length column exists, rc[c][s] = V[cand_s][cand_c] - sum_{j<k0} P[j][s] P[j][c] (s, c < nc;
// P[j][s] = L[j][cand_s] from the gather).  Each entry takes exactly the operations the pass
// applies to row cand_s, column c: the same f64 MFMA over k-steps of 4 vectors (lane g supplies
// vector 4s + g), the same four vector ranges accumulated in order, summed (w0 + w2) + (w1 + w3),
// subtracted from the same integral.  Steps past a range add products with a zero row of P,
// which change nothing, so the ring depth may differ from the pass's.  (NC / 16)^2 workgroups, one
// 16 x 16 block each; the speculative block then runs on rc exactly as when the pass wrote it.
template <bool DENSE, int NC>
__global__ __launch_bounds__(256) void cd_cc_kernel(const CdState *__restrict__ st, const double *P,
                                                    const int64_t *__restrict__ cand, int64_t npairs, PairTable pt,
                                                    const double *__restrict__ V, int64_t ldv,
                                                    double *__restrict__ rc)
{
    constexpr int D = 8;                                   // k-steps in flight per wave
    __shared__ double red[2][16][16];
    const int rg = (int)blockIdx.x / (NC / 16), cgp = (int)blockIdx.x % (NC / 16);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
    // the epilogue's integrals (wave 0: rows 16 rg + g + 4e, column 16 cgp + r16), their inputs
    // loaded with the state so that they land under the products; entries past the candidates
    // (and any index out of range) read pair 0 and are not used
    double base[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t ci = 0, ri[4] = {0, 0, 0, 0};
    if (w == 0) {
        ci = cand[16 * cgp + r16];
        ci = ci >= 0 && ci < npairs ? ci : 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            ri[e] = cand[16 * rg + g + 4 * e];
            ri[e] = ri[e] >= 0 && ri[e] < npairs ? ri[e] : 0;
        }
    }
    if (spec_idle(st) || st->ncand == 0) return;
    const int64_t k0 = st->k;
    const int nc = st->ncand;
    if (16 * rg >= nc || 16 * cgp >= nc) return;           // uniform over the workgroup
    // the integrals' inputs, issued before the ring (they land with its first loads); the
    // integrals themselves are formed after the products
    double rp[4][5], cp5[5];
    if (w == 0) {
        if constexpr (DENSE) {
#pragma unroll
            for (int e = 0; e < 4; ++e) base[e] = V[ci * ldv + ri[e]];   // V[cand_s][cand_c]
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                rp[e][0] = pt.p[ri[e]];
                rp[e][1] = pt.Px[ri[e]];
                rp[e][2] = pt.Py[ri[e]];
                rp[e][3] = pt.Pz[ri[e]];
                rp[e][4] = pt.K[ri[e]];
            }
            cp5[0] = pt.p[ci];
            cp5[1] = pt.Px[ci];
            cp5[2] = pt.Py[ci];
            cp5[3] = pt.Pz[ci];
            cp5[4] = pt.K[ci];
        }
    }
    const int64_t ks = (k0 + 3) / 4;
    const int64_t s0 = ks * w / 4, s1 = ks * (w + 1) / 4;
    const int64_t jz = 4 * ks;                             // a zero row of P
    doublex4 acc = doublex4{0.0, 0.0, 0.0, 0.0};
    double a[D], b[D];
    auto load = [&](int64_t s, double &as, double &bs) {
        const int64_t j = s < s1 ? 4 * s + g : jz;
        as = P[j * NC + 16 * rg + r16];
        bs = P[j * NC + 16 * cgp + r16];
    };
    if (s1 > s0) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            load(s0 + i, a[i], b[i]);
            __builtin_amdgcn_sched_barrier(0);
        }
        for (int64_t s = s0; s < s1; s += D) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[i], acc, 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                asm volatile("" ::: "memory");
                load(s + i + D, a[i], b[i]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // acc[e]: row g + 4e, column r16 of the block, over this wave's range
    if (w >= 2)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[w - 2][g + 4 * e][r16] = acc[e];
    __syncthreads();
    if (w < 2)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] += red[w][g + 4 * e][r16];
    __syncthreads();
    if (w < 2)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[w][g + 4 * e][r16] = acc[e];
    __syncthreads();
    if (w == 0) {
        const int c = 16 * cgp + r16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int s = 16 * rg + g + 4 * e;
            if (s < nc && c < nc) {
                if constexpr (!DENSE)                  // V[cand_s][cand_c], as the pass forms it
                    base[e] = eri_pp(rp[e][0], rp[e][1], rp[e][2], rp[e][3], rp[e][4], cp5[0], cp5[1], cp5[2],
                                     cp5[3], cp5[4]);
                rc[c * NC + s] = base[e] - (red[0][g + 4 * e][r16] + red[1][g + 4 * e][r16]);
            }
        }
    }
}

// Large path, step 3 of a speculative block (after the speculative wave has chosen its ns steps
// from rc): the pass for the speculated columns only.  Column j < ns is candidate slot_j:
// R[j][I] = V[I][cand_slot_j] - sum_{j'<k0} L[j'][I] P[j'][slot_j], every entry with the
// operations of cd_pass_kernel (same A operand and ring, same vector ranges, same reduction),
// so the values equal those of the full pass; the rows kernel reads exactly these columns.
// NG = ceil(ns / 16) column groups of 16; columns past ns read a zero row of P and are not
// written.  Work and R traffic scale with ns instead of all 64 candidates.
template <bool W16, bool DENSE, int NG>
__device__ __forceinline__ void pass_cols_body(const double *L, int64_t ldl, int64_t npairs, int64_t k0,
                                               const double *P, double *__restrict__ R, int64_t ldr,
                                               const PairTable &pt, const double *__restrict__ V, int64_t ldv,
                                               const int64_t *__restrict__ cand, int ns, const int (&sl3)[3],
                                               double (*cdat)[CD_SPEC_MAX], int64_t *ccol,
                                               double (*red)[CD_SPEC_MAX][CD_TILE])
{
    constexpr int D = CD_PASS_D;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
    const int64_t tile0 = (int64_t)blockIdx.x * CD_TILE;
    int64_t rowL[4];
    if constexpr (W16) {
#pragma unroll
        for (int u = 0; u < 2; ++u) rowL[u] = min(tile0 + 32 * u + 2 * r16, ldl - 2);
    } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) rowL[m] = min(tile0 + 16 * m + r16, npairs - 1);
    }
    // this lane's B columns: slot of column 16 n + r16, or a zero row of P past ns
    int bcol[NG];
    bool bon[NG];
#pragma unroll
    for (int n = 0; n < NG; ++n) {
        bon[n] = 16 * n + r16 < ns;
        bcol[n] = bon[n] ? sl3[n] : 0;
    }
    // lane l < 48 of wave 0 owns column l (its slot is sl3[l / 16]): later the column's
    // candidate data for the epilogue
    const bool own = threadIdx.x < CD_SPEC_MAX;
    const int osl = threadIdx.x < ns ? (g == 0 ? sl3[0] : g == 1 ? sl3[1] : sl3[2]) : 0;
    const int64_t ks = (k0 + 3) / 4;
    const int64_t s0 = ks * w / 4, s1 = ks * (w + 1) / 4;
    const int64_t jz = 4 * ks;
    const int64_t jl_max = k0 > 0 ? k0 - 1 : 0;
    doublex4 acc[4][NG];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NG; ++n) acc[m][n] = doublex4{0.0, 0.0, 0.0, 0.0};
    double a[D][4], b[D][NG];
    auto load = [&](int64_t s, double *as, double *bs) {
        const int64_t j = 4 * s + g;
        const int64_t jl = min(j, jl_max);
        const int64_t jp = s < s1 ? j : jz;
        if constexpr (W16) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double2 x = *reinterpret_cast<const double2 *>(L + jl * ldl + rowL[u]);
                as[2 * u] = x.x;
                as[2 * u + 1] = x.y;
            }
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) as[m] = L[jl * ldl + rowL[m]];
        }
#pragma unroll
        for (int n = 0; n < NG; ++n) bs[n] = P[(bon[n] ? jp : jz) * CD_NCAND_L + bcol[n]];
    };
    auto trow = [&](int m, int q) { return W16 ? 32 * (m >> 1) + 2 * q + (m & 1) : 16 * m + q; };
    if (k0 > 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            load(s0 + i, a[i], b[i]);
            __builtin_amdgcn_sched_barrier(0);
        }
        for (int64_t s = s0; s < s1; s += D) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < NG; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][m], b[i][n], acc[m][n], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                asm volatile("" ::: "memory");
                load(s + i + D, a[i], b[i]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // the epilogue's data, loaded under the reduction: the column's candidate (owners), then the
    // row's pair data
    const int row = threadIdx.x % CD_TILE;
    const int64_t I = tile0 + row;
    const int64_t Ir = min(I, npairs - 1);
    const int64_t q = own ? cand[osl] : 0;
    double ip = 0.0, ipx = 0.0, ipy = 0.0, ipz = 0.0, ik = 0.0;
    if constexpr (!DENSE) {
        ip = pt.p[Ir];
        ipx = pt.Px[Ir];
        ipy = pt.Py[Ir];
        ipz = pt.Pz[Ir];
        ik = pt.K[Ir];
    }
    // (w0 + w2) + (w1 + w3) as in cd_pass_kernel; entry (column c, row) at red[.][c][row ^ c]
    auto put = [&](int slot) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < NG; ++n)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = 16 * n + r16, rw = trow(m, g + 4 * e);
                    red[slot][c][rw ^ c] = acc[m][n][e];
                }
    };
    auto add = [&](int slot) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < NG; ++n)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = 16 * n + r16, rw = trow(m, g + 4 * e);
                    acc[m][n][e] += red[slot][c][rw ^ c];
                }
    };
    if (w >= 2) put(w - 2);
    __syncthreads();
    if (w < 2) add(w);
    __syncthreads();
    if (w < 2) put(w);
    if (own) {
        ccol[threadIdx.x] = q;
        if constexpr (!DENSE) {
            cdat[0][threadIdx.x] = pt.p[q];
            cdat[1][threadIdx.x] = pt.Px[q];
            cdat[2][threadIdx.x] = pt.Py[q];
            cdat[3][threadIdx.x] = pt.Pz[q];
            cdat[4][threadIdx.x] = pt.K[q];
        }
    }
    __syncthreads();
    if (I >= npairs) return;
#pragma unroll
    for (int qq = 0; qq < 16 * NG * CD_TILE / 256; ++qq) {
        const int c = (threadIdx.x + 256 * qq) / CD_TILE;        // uniform over the wave
        if (c < ns) {
            double base;
            if constexpr (DENSE)
                base = V[ccol[c] * ldv + I];
            else
                base = eri_pp(ip, ipx, ipy, ipz, ik, cdat[0][c], cdat[1][c], cdat[2][c], cdat[3][c], cdat[4][c]);
            R[(int64_t)c * ldr + I] = base - (red[0][c][row ^ c] + red[1][c][row ^ c]);
        }
    }
}

template <bool W16, bool DENSE>
__global__ __launch_bounds__(256, 3) void cd_pass_cols_kernel(const double *L, int64_t ldl, int64_t npairs,
                                                              const CdState *__restrict__ st, const SpecOut *so,
                                                              const double *P, double *__restrict__ R, int64_t ldr,
                                                              PairTable pt, const double *__restrict__ V, int64_t ldv,
                                                              const int64_t *__restrict__ cand)
{
    __shared__ double red[2][CD_SPEC_MAX][CD_TILE];   // 48 KB: three workgroups per CU
    __shared__ double cdat[5][CD_SPEC_MAX];           // column j's pair data (integrals)
    __shared__ int64_t ccol[CD_SPEC_MAX];             // column j's pair index
    // the state, the record and this lane's three column slots in one round of loads (the
    // record's slot list has CD_SPEC_MAX entries, those past nspec finite and unused)
    const int r16 = threadIdx.x & 15;
    int sl3[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) sl3[n] = so->slot[16 * n + r16];
    const int ns = so->nspec;
    const int64_t k0 = so->k0;
    if (spec_idle(st) || ns <= 0) return;
    if (ns <= 16)
        pass_cols_body<W16, DENSE, 1>(L, ldl, npairs, k0, P, R, ldr, pt, V, ldv, cand, ns, sl3, cdat, ccol, red);
    else if (ns <= 32)
        pass_cols_body<W16, DENSE, 2>(L, ldl, npairs, k0, P, R, ldr, pt, V, ldv, cand, ns, sl3, cdat, ccol, red);
    else
        pass_cols_body<W16, DENSE, 3>(L, ldl, npairs, k0, P, R, ldr, pt, V, ldv, cand, ns, sl3, cdat, ccol, red);
}

// block maxima of x over a grid-stride range (the first pass of the largest ERI diagonal)
constexpr int CD_MAXPART = 512;          // blocks of the first pass
__global__ __launch_bounds__(256) void max_part_kernel(int64_t n, const double *__restrict__ x,
                                                       double *__restrict__ part)
{
    __shared__ double sh[256 / 64];
    double m = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) m = fmax(m, x[i]);
    m = block_max<256>(m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ void max_reduce_kernel(int64_t n, const double *__restrict__ x, double *__restrict__ out)
{
    __shared__ double sh[CD_AUX_NT / 64];
    double m = -INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += CD_AUX_NT) m = fmax(m, x[i]);
    m = block_max<CD_AUX_NT>(m, sh);
    if (threadIdx.x == 0) *out = m;
}

int setup_pairs(cds_ctx *ctx, int32_t nbf, const double *centres, const double *alpha,
                PairTable *pt)
{
    int64_t np = cds_npairs(nbf);
    void *w;
    CDS_CALL(cds_ws(ctx, WS_PAIRS, (size_t)5 * np * sizeof(double), &w));
    double *b = (double *)w;
    pt->p = b;
    pt->Px = b + np;
    pt->Py = b + 2 * np;
    pt->Pz = b + 3 * np;
    pt->K = b + 4 * np;
    hipLaunchKernelGGL(pair_setup_kernel, dim3((unsigned)cds_ceil_div(np, 256)), dim3(256), 0,
                       ctx->stream, nbf, centres, alpha, np, *pt);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}

template <int VW, int TB, bool DENSE>
void launch_step(cds_ctx *ctx, const CdBufs &b, const CdParams &cp, int r, int sr, int sw, int sz,
                 int64_t k, int64_t k0, int bsteps, const PairTable &pt, const double *V, int64_t ldv, double *L,
                 int64_t ldl, const double *R, int64_t ldr, const int64_t *cand, CdState *st, int64_t *piv,
                 const SpecOut *sov)
{
    const dim3 grid((unsigned)cds_ceil_div(b.ntile, TB));
    hipLaunchKernelGGL((cd_step_kernel<VW, TB, DENSE>), grid, dim3(CD_NT), 0, ctx->stream, b, cp, r, sr, sw, sz,
                       k, k0, bsteps, pt, V, ldv, L, ldl, R, ldr, cand, st, piv, sov);
}

// step-kernel shape: rows per thread (16-byte loads when the layout allows) and tiles per
// block (4 once one tile per block would need more than one round of blocks on the chip)
template <bool DENSE>
void launch_step_any(cds_ctx *ctx, int vw, int tb, const CdBufs &b, const CdParams &cp, int r, int sr, int sw,
                     int sz, int64_t k, int64_t k0, int bsteps, const PairTable &pt, const double *V, int64_t ldv,
                     double *L, int64_t ldl, const double *R, int64_t ldr, const int64_t *cand, CdState *st,
                     int64_t *piv, const SpecOut *sov)
{
    if (vw == 2 && tb == 4)
        launch_step<2, 4, DENSE>(ctx, b, cp, r, sr, sw, sz, k, k0, bsteps, pt, V, ldv, L, ldl, R, ldr, cand, st, piv, sov);
    else if (vw == 2)
        launch_step<2, 1, DENSE>(ctx, b, cp, r, sr, sw, sz, k, k0, bsteps, pt, V, ldv, L, ldl, R, ldr, cand, st, piv, sov);
    else if (tb == 4)
        launch_step<1, 4, DENSE>(ctx, b, cp, r, sr, sw, sz, k, k0, bsteps, pt, V, ldv, L, ldl, R, ldr, cand, st, piv, sov);
    else
        launch_step<1, 1, DENSE>(ctx, b, cp, r, sr, sw, sz, k, k0, bsteps, pt, V, ldv, L, ldl, R, ldr, cand, st, piv, sov);
}

// The mailbox word (coherent pinned host memory, written by the device over the bus), made
// once per context; false where it cannot be had or was seen not to follow the state.
bool mail_ready(cds_ctx *ctx)
{
    if (ctx->mail_off || !ctx->cd_mailbox) return false;
    if (!ctx->mail) {
        void *h = nullptr, *d = nullptr;
        if (hipHostMalloc(&h, 64, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
            ctx->mail_off = true;
            return false;
        }
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
            (void)hipHostFree(h);
            ctx->mail_off = true;
            return false;
        }
        ctx->mail = (uint64_t *)h;
        ctx->mail_dev = (uint64_t *)d;
    }
    return true;
}

// Spin until the word shows a block count in (seen, upto] (modulo its field); false once
// limit_ms passed without one.
bool mail_wait(const uint64_t *mail, int64_t seen, int64_t upto, double limit_ms, uint64_t *w)
{
    const uint64_t span = (uint64_t)(upto - seen);
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t it = 1;; ++it) {
        const uint64_t v = __atomic_load_n(mail, __ATOMIC_ACQUIRE);
        const uint64_t d = ((v >> MB_NSHIFT) - (uint64_t)seen) & MB_NMASK;
        if (d != 0 && d <= span) {
            *w = v;
            return true;
        }
        if ((it & 255) == 0 &&
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() > limit_ms)
            return false;
    }
}

int cholesky_impl(cds_ctx *ctx, bool dense, int32_t nbf, const double *centres,
                  const double *alpha, int64_t npairs, const double *V, int64_t ldv, double delta,
                  double tau, double psd_tol, int64_t max_vec, double *L, int64_t ldl,
                  int64_t *piv, double *D, int64_t nvec_in, int64_t *h_nvec, double *h_dmax,
                  int32_t *h_status, const unsigned char *allowed = nullptr, const CdHook *hook = nullptr)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, npairs >= 1, "npairs must be >= 1");
    CDS_REQUIRE(ctx, L && piv && D && h_nvec && h_dmax && h_status, "NULL output pointer");
    CDS_REQUIRE(ctx, ldl >= npairs, "ldl (%lld) < npairs (%lld)", (long long)ldl, (long long)npairs);
    CDS_REQUIRE(ctx, max_vec >= 1 && max_vec <= npairs, "max_vec must be in [1, npairs]");
    CDS_REQUIRE(ctx, nvec_in >= 0 && nvec_in <= max_vec, "nvec_in must be in [0, max_vec]");
    CDS_REQUIRE(ctx, delta > 0.0 && std::isfinite(delta), "delta must be positive and finite");
    CDS_REQUIRE(ctx, std::isfinite(tau) && std::isfinite(psd_tol), "tau/psd_tol must be finite");
    if (dense) CDS_REQUIRE(ctx, V && ldv >= npairs, "dense V NULL or ldv < npairs");

    PairTable pt = {};
    const unsigned nb = (unsigned)cds_ceil_div(npairs, 256);
    if (!dense) CDS_CALL(setup_pairs(ctx, nbf, centres, alpha, &pt));

    const int vw = (ldl % 2 == 0 && cds_aligned(L, 16)) ? 2 : 1;
    const int tb = (cds_ceil_div(npairs, CD_TILE) > CD_ONE_TILE_MAX || ctx->cd_large_path) ? 4 : 1;
    const int64_t ntile = cds_ceil_div(npairs, CD_TILE);
    const int bsteps = ntile <= CD_CAND_MAXTILE ? ctx->cd_lookahead : 0;
    const int64_t tps = cds_ceil_div(ntile, CD_NSUP);
    const int64_t ldr = cds_ceil_div(npairs, 64) * 64;

    // workspace: D copy, ERI diagonal, candidate rows P (max_vec x NCAND), residual columns R
    void *w_part, *w_tile, *w_mask, *w_state;
    // (P and the candidates' block have room for the large path's CD_NCAND_L candidates; R for
    // CD_NCAND columns: by candidate slot on the small path, by speculated step on the large one)
    const size_t nP = (size_t)(max_vec + CD_PASS_ZROWS) * CD_NCAND_L, nR = bsteps > 0 ? (size_t)CD_NCAND * ldr : 0;
    const bool spec_on = bsteps > 0 && ctx->cd_speculate;
    const size_t nDb = spec_on ? (size_t)CD_SPEC_MAX * npairs : 0;
    CDS_CALL(cds_ws(ctx, WS_CD_PART, ((size_t)2 * npairs + (bsteps > 0 ? nP : 0) + nR + nDb) * 8 + 256, &w_part));
    CDS_CALL(cds_ws(ctx, WS_CD_TILE, (size_t)2 * ntile * sizeof(TileStat) + (size_t)6 * CD_NSUP * 8 + 64 +
                                     (size_t)CD_MAXPART * 8, &w_tile));
    CDS_CALL(cds_ws(ctx, WS_CD_MASK, (size_t)3 * npairs, &w_mask));
    CDS_CALL(cds_ws(ctx, WS_CD_STATE, sizeof(CdState) + CD_NCAND_L * 8 + sizeof(SpecOut) + 64 +
                                      (size_t)CD_NCAND_L * CD_NCAND_L * 8 + 256, &w_state));
    double *D1 = (double *)w_part;
    double *diag = D1 + npairs;
    double *Pc = diag + npairs;
    double *Rc = Pc + (bsteps > 0 ? nP : 0);
    CdBufs bf;
    bf.D[0] = D;
    bf.D[1] = D1;
    bf.mask[0] = (unsigned char *)w_mask;
    bf.mask[1] = bf.mask[0] + npairs;
    bf.ts[0] = (TileStat *)w_tile;
    bf.ts[1] = bf.ts[0] + ntile;
    unsigned long long *sb = (unsigned long long *)(bf.ts[1] + ntile);
    for (int i = 0; i < 3; ++i) {
        bf.smax[i] = sb + i * CD_NSUP;
        bf.smin[i] = sb + (3 + i) * CD_NSUP;
    }
    bf.ntile = ntile;
    bf.tps = tps;
    bf.flat = (ntile <= (int64_t)CD_NT * CD_TPT && !ctx->cd_large_path) ? 1 : 0;
    double *dscratch = (double *)(sb + 6 * CD_NSUP);
    CdState *st = (CdState *)w_state;
    int64_t *cand = (int64_t *)(st + 1);
    SpecOut *so = (SpecOut *)(cand + CD_NCAND_L);
    bf.slot = (signed char *)(bf.mask[1] + npairs);
    bf.rc = (double *)(((uintptr_t)(so + 1) + 255) & ~(uintptr_t)255);
    double *Dbuf = Rc + nR;

    // largest ERI diagonal (for the default tie window / PSD tolerance)
    if (dense)
        hipLaunchKernelGGL(dense_diag_kernel, dim3(nb), dim3(256), 0, ctx->stream, npairs, V, ldv, diag);
    else
        hipLaunchKernelGGL(eri_diag_kernel, dim3(nb), dim3(256), 0, ctx->stream, npairs, pt, diag);
    CDS_LAUNCHED(ctx);
    {
        // two passes: block maxima over the whole chip, then one block over those
        double *dpart = dscratch + 8;
        const int64_t nbm = std::min<int64_t>(CD_MAXPART, cds_ceil_div(npairs, 256));
        hipLaunchKernelGGL(max_part_kernel, dim3((unsigned)nbm), dim3(256), 0, ctx->stream, npairs, diag, dpart);
        hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(CD_AUX_NT), 0, ctx->stream, nbm, (const double *)dpart,
                           dscratch);
        CDS_LAUNCHED(ctx);
    }
    void *hp;
    CDS_CALL(cds_pinned(ctx, 256, &hp));
    CDS_HIP(ctx, hipMemcpyAsync(hp, dscratch, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const double vmax = *(double *)hp;
    CdParams cp;
    cp.npairs = npairs;
    cp.max_vec = max_vec;
    cp.delta = delta;
    cp.tau = tau < 0 ? 1e-10 * vmax : tau;
    cp.psd_tol = psd_tol < 0 ? 1e3 * DBL_EPSILON * vmax : psd_tol;
    cp.nvec_in = nvec_in;
    cp.spec_len = std::min(bsteps, CD_SPEC_MAX);
    cp.pad = 0;

    CdsTimer tall;
    CDS_CALL(cds_timer_start(ctx, &tall));
    if (allowed) {
        hipLaunchKernelGGL(init_mask_kernel, dim3(nb), dim3(256), 0, ctx->stream, npairs, allowed, bf.mask[0]);
        CDS_LAUNCHED(ctx);
    }
    CdState st0 = {};
    st0.k = nvec_in;
    st0.kdone = INT64_MAX;
    // block counts of successive calls start 2^16 apart, so no word a call left can be taken
    // for one of the next call's commits
    st0.nblk = (int64_t)(ctx->mail_base += (1 << 16));
    // the mask (unless set above), no row a candidate, the super-tile buffers empty (0 and 1 are
    // read first; 2 is reset by the first step anyway), the state, D on a fresh start
    static_assert(sizeof(CdState) <= 2048, "the state goes as a kernel argument");
    {
        const int64_t nsb = std::max<int64_t>(nb, cds_ceil_div(3 * CD_NSUP, 256));
        hipLaunchKernelGGL(cd_setup_kernel, dim3((unsigned)nsb), dim3(256), 0, ctx->stream, npairs, bf.mask[0],
                           allowed ? 0 : 1, (signed char *)bf.slot, bf.smax[0], bf.smin[0], D, (const double *)diag,
                           nvec_in == 0 ? 1 : 0, st0, st);
        CDS_LAUNCHED(ctx);
    }
    if (nvec_in != 0) {
        hipLaunchKernelGGL(mark_pivots_kernel, dim3((unsigned)cds_ceil_div(nvec_in, 256)), dim3(256),
                           0, ctx->stream, nvec_in, piv, npairs, bf.mask[0]);
        CDS_LAUNCHED(ctx);
    }
    hipLaunchKernelGGL(tile_stats_kernel, dim3((unsigned)ntile), dim3(CD_TILE), 0, ctx->stream, bf, cp);
    CDS_LAUNCHED(ctx);

    int64_t k = nvec_in, k0 = nvec_in, next_start = nvec_in;
    int batch = 16;                     // batch ends fall on look-ahead block starts (16, 32, 64)
    CdState hs = {};
    const dim3 grid((unsigned)ntile);
    // 16-byte loads of L in the pass need an even row stride and an aligned base
    const bool pass16 = ldl % 2 == 0 && cds_aligned(L, 16);
    CdsTimer tk;
    bool run_timed = false;
    // speculative blocks, chained on the device.  With the mailbox, two blocks stay queued:
    // each commit's word tells the host to queue one more, and the stream is drained only at a
    // stall.  Without it, NB blocks are queued per read of the state.  A stall (a block that
    // kept no step: a termination or a failed first check) gets one per-step launch at the same
    // start, whose candidates and residual columns still hold.
    constexpr int NB = 4;
    constexpr int MB_AHEAD = 2;            // blocks queued beyond the last commit seen
    constexpr double MB_WAIT_MS = 1000.0;  // then the state is read after a drain instead
    const bool mb = spec_on && mail_ready(ctx);
    if (mb) __atomic_store_n(ctx->mail, mb_word(st0.nblk, 0, 0), __ATOMIC_RELEASE);
    bool blocks_ran = false;               // speculative blocks since the last read of the state
    // the large path (separate speculative and row kernels) forms the candidates' own block
    // first, lets the speculative wave choose its steps, and then passes over the speculated
    // columns only; the small path runs the full pass and the lockstep kernel
    const unsigned nrb = (unsigned)cds_ceil_div(npairs, 256);
    const unsigned nlb = (unsigned)cds_ceil_div(npairs, CD_LS_ROWS);
    const bool lockstep = nlb <= (unsigned)CD_FUSE_MAXBLK && !ctx->cd_large_path;
    const bool early = spec_on && !lockstep;
    auto queue_block = [&]() -> int {
        if (early)
            hipLaunchKernelGGL((cd_cand_kernel<CD_NCAND_L, CD_AUX_NT>), dim3(1), dim3(CD_AUX_NT), 0, ctx->stream, bf,
                               cp, 0, 0, (int64_t)-1, st, cand, so);
        else
            hipLaunchKernelGGL((cd_cand_kernel<CD_NCAND, CD_AUX_NT>), dim3(1), dim3(CD_AUX_NT), 0, ctx->stream, bf,
                               cp, 0, 0, (int64_t)-1, st, cand, so);
        CDS_LAUNCHED(ctx);
        const dim3 ggrid((unsigned)cds_ceil_div((max_vec + CD_PASS_ZROWS) * CD_NCAND, 256));
        if (early) {
            const dim3 ggl((unsigned)cds_ceil_div((max_vec + CD_PASS_ZROWS) * CD_NCAND_L, 256));
            hipLaunchKernelGGL(cd_gather_kernel<CD_NCAND_L>, ggl, dim3(256), 0, ctx->stream, (const double *)L, ldl,
                               (int64_t)-1, (const CdState *)st, (const int64_t *)cand, Pc);
            CDS_LAUNCHED(ctx);
            CdsTimer tcc;
            if (ctx->kernel_timing) CDS_CALL(cds_timer_start(ctx, &tcc));
            constexpr unsigned ncc = (CD_NCAND_L / 16) * (CD_NCAND_L / 16);
            if (dense)
                hipLaunchKernelGGL((cd_cc_kernel<true, CD_NCAND_L>), dim3(ncc), dim3(256), 0, ctx->stream,
                                   (const CdState *)st, (const double *)Pc, (const int64_t *)cand, npairs, pt, V, ldv,
                                   bf.rc);
            else
                hipLaunchKernelGGL((cd_cc_kernel<false, CD_NCAND_L>), dim3(ncc), dim3(256), 0, ctx->stream,
                                   (const CdState *)st, (const double *)Pc, (const int64_t *)cand, npairs, pt, V, ldv,
                                   bf.rc);
            CDS_LAUNCHED(ctx);
            hipLaunchKernelGGL(cd_spec_kernel, dim3(1), dim3(64), 0, ctx->stream, bf, cp, (const int64_t *)cand,
                               st, so);
            CDS_LAUNCHED(ctx);
            if (ctx->kernel_timing) CDS_CALL(cds_timer_stop(ctx, &tcc, &ctx->stats.t_cd_spec_ms));
            CdsTimer tp;
            if (ctx->kernel_timing) CDS_CALL(cds_timer_start(ctx, &tp));
            if (pass16 && !dense)
                hipLaunchKernelGGL((cd_pass_cols_kernel<true, false>), grid, dim3(256), 0, ctx->stream,
                                   (const double *)L, ldl, npairs, (const CdState *)st, (const SpecOut *)so,
                                   (const double *)Pc, Rc, ldr, pt, V, ldv, (const int64_t *)cand);
            else if (pass16)
                hipLaunchKernelGGL((cd_pass_cols_kernel<true, true>), grid, dim3(256), 0, ctx->stream,
                                   (const double *)L, ldl, npairs, (const CdState *)st, (const SpecOut *)so,
                                   (const double *)Pc, Rc, ldr, pt, V, ldv, (const int64_t *)cand);
            else if (!dense)
                hipLaunchKernelGGL((cd_pass_cols_kernel<false, false>), grid, dim3(256), 0, ctx->stream,
                                   (const double *)L, ldl, npairs, (const CdState *)st, (const SpecOut *)so,
                                   (const double *)Pc, Rc, ldr, pt, V, ldv, (const int64_t *)cand);
            else
                hipLaunchKernelGGL((cd_pass_cols_kernel<false, true>), grid, dim3(256), 0, ctx->stream,
                                   (const double *)L, ldl, npairs, (const CdState *)st, (const SpecOut *)so,
                                   (const double *)Pc, Rc, ldr, pt, V, ldv, (const int64_t *)cand);
            CDS_LAUNCHED(ctx);
            if (ctx->kernel_timing) CDS_CALL(cds_timer_stop(ctx, &tp, &ctx->stats.t_cd_pass_ms));
            if (hook && hook->block) CDS_CALL(hook->block(hook->user, early ? 1 : 0));
        }
        CdsTimer tsp;
        if (ctx->kernel_timing) CDS_CALL(cds_timer_start(ctx, &tsp));
        if (early) {
            hipLaunchKernelGGL(cd_rows_kernel, dim3(nrb), dim3(256), 0, ctx->stream, bf, cp, (const CdState *)st,
                               (const double *)Rc, ldr, L, ldl, Dbuf, so,
                               (const double *)((const char *)so + offsetof(SpecOut, lpiv)));
            CDS_LAUNCHED(ctx);
        } else {
            const int64_t cgx = cds_ceil_div(npairs, 256);
            const int64_t gy = cds_ceil_div(cds_ceil_div((max_vec + CD_PASS_ZROWS) * CD_NCAND, 256), cgx);
            const dim3 cgrid((unsigned)cgx, (unsigned)(CD_NCG + gy));
            // on demand, the pass evaluates the candidate columns' integrals in its epilogue and
            // only the gather runs before it
            if (dense)
                hipLaunchKernelGGL(cd_candcol_gather_kernel<true>, cgrid, dim3(256), 0, ctx->stream, pt, V, ldv,
                                   npairs, (const CdState *)st, (const int64_t *)cand, Rc, ldr, (const double *)L,
                                   ldl, Pc);
            else
                hipLaunchKernelGGL(cd_gather_kernel<CD_NCAND>, ggrid, dim3(256), 0, ctx->stream, (const double *)L,
                                   ldl, (int64_t)-1, (const CdState *)st, (const int64_t *)cand, Pc);
            CDS_LAUNCHED(ctx);
            if (ctx->kernel_timing) CDS_CALL(cds_timer_stop(ctx, &tsp, &ctx->stats.t_cd_spec_ms));
            CdsTimer tp;
            if (ctx->kernel_timing) CDS_CALL(cds_timer_start(ctx, &tp));
            if (pass16 && !dense)
                hipLaunchKernelGGL((cd_pass_kernel<true, true>), grid, dim3(256), 0, ctx->stream, (const double *)L,
                                   ldl, npairs, (int64_t)-1, (const CdState *)st, (const double *)Pc, Rc, ldr,
                                   (const signed char *)bf.slot, bf.rc, pt, (const int64_t *)cand);
            else if (pass16)
                hipLaunchKernelGGL((cd_pass_kernel<true, false>), grid, dim3(256), 0, ctx->stream, (const double *)L,
                                   ldl, npairs, (int64_t)-1, (const CdState *)st, (const double *)Pc, Rc, ldr,
                                   (const signed char *)bf.slot, bf.rc, pt, (const int64_t *)cand);
            else if (!dense)
                hipLaunchKernelGGL((cd_pass_kernel<false, true>), grid, dim3(256), 0, ctx->stream, (const double *)L,
                                   ldl, npairs, (int64_t)-1, (const CdState *)st, (const double *)Pc, Rc, ldr,
                                   (const signed char *)bf.slot, bf.rc, pt, (const int64_t *)cand);
            else
                hipLaunchKernelGGL((cd_pass_kernel<false, false>), grid, dim3(256), 0, ctx->stream, (const double *)L,
                                   ldl, npairs, (int64_t)-1, (const CdState *)st, (const double *)Pc, Rc, ldr,
                                   (const signed char *)bf.slot, bf.rc, pt, (const int64_t *)cand);
            CDS_LAUNCHED(ctx);
            if (ctx->kernel_timing) CDS_CALL(cds_timer_stop(ctx, &tp, &ctx->stats.t_cd_pass_ms));
            if (hook && hook->block) CDS_CALL(hook->block(hook->user, early ? 1 : 0));
            if (ctx->kernel_timing) CDS_CALL(cds_timer_start(ctx, &tsp));
            hipLaunchKernelGGL(cd_lockstep_kernel, dim3(nlb), dim3(64 + CD_LS_ROWS), 0, ctx->stream, bf, cp,
                               (const int64_t *)cand, (const CdState *)st, (const double *)Rc, ldr, L, ldl, Dbuf,
                               so);
            CDS_LAUNCHED(ctx);
        }
        if (!bf.flat) {
            hipLaunchKernelGGL(reset_super_kernel, dim3(1), dim3(64), 0, ctx->stream, bf, cp, (const CdState *)st,
                               (const SpecOut *)so);
            CDS_LAUNCHED(ctx);
        }
        hipLaunchKernelGGL(cd_commit_kernel, dim3((unsigned)cds_ceil_div(npairs, 256)), dim3(256), 0,
                           ctx->stream, bf, cp, (const double *)Dbuf, (const double *)L, ldl, (const SpecOut *)so,
                           st, piv,
                           mb && !ctx->mail_off ? ctx->mail_dev : nullptr);
        CDS_LAUNCHED(ctx);
        if (ctx->kernel_timing) CDS_CALL(cds_timer_stop(ctx, &tsp, &ctx->stats.t_cd_spec_ms));
        return CDS_OK;
    };
    while (spec_on) {
        CDS_HIP(ctx, hipMemcpyAsync(hp, st, sizeof(CdState), hipMemcpyDeviceToHost, ctx->stream));
        CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
        hs = *(CdState *)hp;
        ctx->stats.n_cd_state_read += 1;
        // every commit has landed: the word must show the last one (else it is not used again)
        if (mb && blocks_ran && hs.nblk != st0.nblk &&
            __atomic_load_n(ctx->mail, __ATOMIC_ACQUIRE) != mb_word(hs.nblk, hs.stall, hs.k))
            ctx->mail_off = true;
        blocks_ran = false;
        if (hs.done) break;
        k = hs.k;
        if (k > max_vec)
            return cds_fail(ctx, CDS_EDEVICE, "CD did not terminate at max_vec=%lld", (long long)max_vec);
        if (hook) CDS_CALL(hook->committed(hook->user, k));
        if (hs.stall) {
            CDS_HIP(ctx, hipMemsetAsync(&st->stall, 0, sizeof(int32_t), ctx->stream));
            const int64_t s = k - nvec_in;
            const int r2 = (int)(s & 1), sr2 = (int)(s % 3), sw2 = (int)((s + 1) % 3), sz2 = (int)((s + 2) % 3);
            if (ctx->kernel_timing) CDS_CALL(cds_timer_start(ctx, &tk));
            if (dense)
                launch_step_any<true>(ctx, vw, tb, bf, cp, r2, sr2, sw2, sz2, k, k, bsteps, pt, V, ldv, L, ldl, Rc,
                                      ldr, cand, st, piv, early ? (const SpecOut *)so : nullptr);
            else
                launch_step_any<false>(ctx, vw, tb, bf, cp, r2, sr2, sw2, sz2, k, k, bsteps, pt, V, ldv, L, ldl, Rc,
                                       ldr, cand, st, piv, early ? (const SpecOut *)so : nullptr);
            CDS_LAUNCHED(ctx);
            if (ctx->kernel_timing) CDS_CALL(cds_timer_stop(ctx, &tk, &ctx->stats.t_cd_kernel_ms));
            ctx->stats.n_cd_step_launch += 1;
            continue;
        }
        blocks_ran = true;
        if (!mb || ctx->mail_off) {
            for (int bi = 0; bi < NB; ++bi) CDS_CALL(queue_block());
            continue;
        }
        int64_t seen = hs.nblk, queued = hs.nblk;
        for (;;) {
            for (; queued < seen + MB_AHEAD; ++queued) CDS_CALL(queue_block());
            uint64_t w;
            if (!mail_wait(ctx->mail, seen, queued, MB_WAIT_MS, &w)) break;
            seen += (int64_t)(((w >> MB_NSHIFT) - (uint64_t)seen) & MB_NMASK);
            if ((w >> MB_KBITS) & 1) break;            // stalled: the blocks after it do nothing
            if (hook) CDS_CALL(hook->committed(hook->user, (int64_t)(w & MB_KMASK)));
        }
    }
    for (; !spec_on;) {
        CDS_HIP(ctx, hipMemcpyAsync(hp, st, sizeof(CdState), hipMemcpyDeviceToHost, ctx->stream));
        CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
        hs = *(CdState *)hp;
        if (hs.done) break;
        if (hs.k != k)
            return cds_fail(ctx, CDS_EDEVICE, "CD state out of step (device k=%lld host k=%lld)",
                            (long long)hs.k, (long long)k);
        if (k > max_vec)
            return cds_fail(ctx, CDS_EDEVICE, "CD did not terminate at max_vec=%lld", (long long)max_vec);
        if (hook) CDS_CALL(hook->committed(hook->user, k));
        // steps k <= max_vec: the step at k == max_vec only records the termination (CAP or
        // convergence) and writes no vector
        for (int bi = 0; bi < batch && k <= max_vec; ++bi, ++k) {
            int64_t s = k - nvec_in;
            const int r = (int)(s & 1), sr = (int)(s % 3);
            const bool block_start = bsteps > 0 && k == next_start;
            if (block_start && k < max_vec) {
                // look-ahead block start: candidates, their rows, one pass over L
                if (run_timed) {
                    CDS_CALL(cds_timer_stop(ctx, &tk, &ctx->stats.t_cd_kernel_ms));
                    run_timed = false;
                }
                k0 = k;
                next_start = k + bsteps;
                hipLaunchKernelGGL((cd_cand_kernel<CD_NCAND, CD_AUX_NT>), dim3(1), dim3(CD_AUX_NT), 0, ctx->stream, bf, cp, r, sr, k,
                                   st, cand, so);
                CDS_LAUNCHED(ctx);
                if (k > 0) {
                    hipLaunchKernelGGL(cd_gather_kernel<CD_NCAND>, dim3((unsigned)cds_ceil_div((k + CD_PASS_ZROWS) * CD_NCAND, 256)), dim3(256),
                                       0, ctx->stream, (const double *)L, ldl, k, (const CdState *)st,
                                       (const int64_t *)cand, Pc);
                    CDS_LAUNCHED(ctx);
                }
                const dim3 cgrid((unsigned)cds_ceil_div(npairs, 256), CD_NCG);
                if (dense)
                    hipLaunchKernelGGL(cd_candcol_kernel<true>, cgrid, dim3(256), 0, ctx->stream, pt, V, ldv, npairs,
                                       (const CdState *)st, (const int64_t *)cand, Rc, ldr);
                else
                    hipLaunchKernelGGL(cd_candcol_kernel<false>, cgrid, dim3(256), 0, ctx->stream, pt, V, ldv, npairs,
                                       (const CdState *)st, (const int64_t *)cand, Rc, ldr);
                CDS_LAUNCHED(ctx);
                CdsTimer tp;
                if (ctx->kernel_timing) CDS_CALL(cds_timer_start(ctx, &tp));
                if (pass16)
                    hipLaunchKernelGGL((cd_pass_kernel<true, false>), grid, dim3(256), 0, ctx->stream,
                                       (const double *)L, ldl, npairs, k, (const CdState *)st, (const double *)Pc, Rc,
                                       ldr, (const signed char *)bf.slot, bf.rc, pt, (const int64_t *)cand);
                else
                    hipLaunchKernelGGL((cd_pass_kernel<false, false>), grid, dim3(256), 0, ctx->stream,
                                       (const double *)L, ldl, npairs, k, (const CdState *)st, (const double *)Pc, Rc,
                                       ldr, (const signed char *)bf.slot, bf.rc, pt, (const int64_t *)cand);
                CDS_LAUNCHED(ctx);
                if (ctx->kernel_timing) CDS_CALL(cds_timer_stop(ctx, &tp, &ctx->stats.t_cd_pass_ms));
                ctx->stats.n_cd_pass_launch += 1;
            }
            const int r2 = (int)(s & 1), sr2 = (int)(s % 3), sw2 = (int)((s + 1) % 3), sz2 = (int)((s + 2) % 3);
            // one event pair around each run of consecutive step launches (a pair around
            // every launch would add its own overhead to each)
            if (ctx->kernel_timing && !run_timed) {
                CDS_CALL(cds_timer_start(ctx, &tk));
                run_timed = true;
            }
            if (dense)
                launch_step_any<true>(ctx, vw, tb, bf, cp, r2, sr2, sw2, sz2, k, k0, bsteps, pt, V, ldv, L, ldl, Rc,
                                      ldr, cand, st, piv, nullptr);
            else
                launch_step_any<false>(ctx, vw, tb, bf, cp, r2, sr2, sw2, sz2, k, k0, bsteps, pt, V, ldv, L, ldl, Rc,
                                       ldr, cand, st, piv, nullptr);
            CDS_LAUNCHED(ctx);
            ctx->stats.n_cd_step_launch += 1;
        }
        if (run_timed) {
            CDS_CALL(cds_timer_stop(ctx, &tk, &ctx->stats.t_cd_kernel_ms));
            run_timed = false;
        }
        if (batch < 64) batch *= 2;
    }
    // the residual diagonal of the final state lives in the buffer of parity (k - nvec_in)
    if ((hs.k - nvec_in) & 1)
        CDS_HIP(ctx, hipMemcpyAsync(D, D1, (size_t)npairs * 8, hipMemcpyDeviceToDevice, ctx->stream));
    CDS_CALL(cds_timer_stop(ctx, &tall, &ctx->stats.t_cd_ms));
    // algorithmic bytes of the steps made (plain left-looking count): 8 npairs k + 64 npairs
    for (int64_t j = nvec_in; j < hs.k; ++j)
        ctx->stats.bytes_cd += 8.0 * (double)npairs * (double)j + 64.0 * (double)npairs;
    ctx->stats.n_cd_steps += hs.k - nvec_in;
    // passes that did work: block starts before the final k (8 npairs B per vector read, one
    // row of R written per candidate; 2 flops per vector, pair and candidate slot)
    if (spec_on) {
        ctx->stats.n_cd_pass_launch += hs.npass;
        ctx->stats.n_cd_pass += hs.npass;
        ctx->stats.n_cd_spec_block += hs.npass;
        ctx->stats.n_cd_spec += hs.nspec;
        if (early) {
            // the columns formed (16 per group of speculated steps)
            ctx->stats.bytes_cd_pass += 8.0 * (double)npairs * hs.sumk0 + 8.0 * (double)npairs * (double)hs.ncols;
            ctx->stats.flops_cd_pass += 2.0 * (double)npairs * hs.sumk0c;
        } else {
            ctx->stats.bytes_cd_pass += 8.0 * (double)npairs * hs.sumk0 + 8.0 * CD_NCAND * (double)npairs * (double)hs.npass;
            ctx->stats.flops_cd_pass += 2.0 * (double)npairs * hs.sumk0 * CD_NCAND;
        }
        ctx->stats.flops_cd_pass_method += 2.0 * (double)npairs * hs.sumk0s;
        ctx->stats.flops_cd_block_method += 2.0 * (double)npairs * hs.sumwin;
    }
    if (bsteps > 0 && !spec_on)
        for (int64_t j = nvec_in; j < hs.k; j += bsteps) {
            ctx->stats.bytes_cd_pass += 8.0 * (double)npairs * (double)j + 8.0 * CD_NCAND * (double)npairs;
            ctx->stats.flops_cd_pass += 2.0 * (double)npairs * (double)j * CD_NCAND;
            ctx->stats.n_cd_pass += 1;
        }
    ctx->stats.n_cd_miss += hs.nmiss;
    ctx->stats.bytes_cd_step += hs.bytes;
    CDS_CALL(cds_timers_flush(ctx));
    *h_nvec = hs.k;
    *h_dmax = hs.dmax;
    *h_status = hs.status;
    if (hs.status == CDS_CD_CAP)
        return cds_fail(ctx, CDS_ECAP, "max_vec=%lld reached with D_max=%g > delta=%g",
                        (long long)max_vec, hs.dmax, delta);
    if (hs.status == CDS_CD_NOTPSD)
        return cds_fail(ctx, CDS_ENOTPSD, "residual diagonal below -%g", cp.psd_tol);
    return CDS_OK;
}

}  // namespace

int cds_cholesky_hooked(cds_ctx *ctx, int32_t nbf, const double *centres, const double *alpha, double delta,
                        double tau, double psd_tol, int64_t max_vec, double *L, int64_t ldl, int64_t *piv,
                        double *D, int64_t *h_nvec, double *h_dmax, int32_t *h_status, const CdHook *hook)
{
    if (!ctx) return CDS_EINVAL;
    if (nbf < 1 || !centres || !alpha) return cds_fail(ctx, CDS_EINVAL, "nbf < 1 or NULL basis");
    return cholesky_impl(ctx, false, nbf, centres, alpha, cds_npairs(nbf), nullptr, 0, delta, tau, psd_tol,
                         max_vec, L, ldl, piv, D, 0, h_nvec, h_dmax, h_status, nullptr, hook);
}

extern "C" {

int cds_eri_columns(cds_ctx *ctx, int32_t nbf, const double *centres, const double *alpha,
                    int64_t ncol, const int64_t *cols, double *out)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, nbf >= 1 && ncol >= 0, "nbf must be >= 1 and ncol >= 0");
    CDS_REQUIRE(ctx, ncol <= 65535, "ncol must be <= 65535 per call");
    CDS_REQUIRE(ctx, centres && alpha && (ncol == 0 || (cols && out)), "NULL pointer");
    if (ncol == 0) return CDS_OK;
    PairTable pt;
    CDS_CALL(setup_pairs(ctx, nbf, centres, alpha, &pt));
    int64_t np = cds_npairs(nbf);
    hipLaunchKernelGGL(eri_columns_kernel, dim3((unsigned)cds_ceil_div(np, 256), (unsigned)ncol),
                       dim3(256), 0, ctx->stream, np, pt, ncol, cols, out);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}

int cds_cholesky_sgauss(cds_ctx *ctx, int32_t nbf, const double *centres, const double *alpha,
                        double delta, double tau, double psd_tol, int64_t max_vec, double *L,
                        int64_t ldl, int64_t *piv, double *D, int64_t nvec_in, int64_t *h_nvec,
                        double *h_dmax, int32_t *h_status)
{
    if (!ctx) return CDS_EINVAL;
    if (nbf < 1 || !centres || !alpha) return cds_fail(ctx, CDS_EINVAL, "nbf < 1 or NULL basis");
    return cholesky_impl(ctx, false, nbf, centres, alpha, cds_npairs(nbf), nullptr, 0, delta, tau,
                         psd_tol, max_vec, L, ldl, piv, D, nvec_in, h_nvec, h_dmax, h_status);
}

int cds_cholesky_dense(cds_ctx *ctx, int64_t npairs, const double *V, int64_t ldv, double delta,
                       double tau, double psd_tol, int64_t max_vec, double *L, int64_t ldl,
                       int64_t *piv, double *D, int64_t nvec_in, int64_t *h_nvec, double *h_dmax,
                       int32_t *h_status)
{
    return cholesky_impl(ctx, true, 0, nullptr, nullptr, npairs, V, ldv, delta, tau, psd_tol,
                         max_vec, L, ldl, piv, D, nvec_in, h_nvec, h_dmax, h_status);
}

int cds_cholesky_sgauss_subset(cds_ctx *ctx, int32_t nbf, const double *centres, const double *alpha,
                               const uint8_t *allowed, double delta, double tau, double psd_tol,
                               int64_t max_vec, double *L, int64_t ldl, int64_t *piv, double *D,
                               int64_t nvec_in, int64_t *h_nvec, double *h_dmax, int32_t *h_status)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, nbf >= 1 && centres && alpha, "need nbf >= 1, centres and alpha");
    CDS_REQUIRE(ctx, allowed, "allowed is NULL");
    return cholesky_impl(ctx, false, nbf, centres, alpha, cds_npairs(nbf), nullptr, 0, delta, tau,
                         psd_tol, max_vec, L, ldl, piv, D, nvec_in, h_nvec, h_dmax, h_status,
                         (const unsigned char *)allowed);
}

int cds_set_cd_lookahead(cds_ctx *ctx, int32_t block_steps)
{
    if (!ctx) return CDS_EINVAL;
    if (block_steps < 0 || block_steps > 256)
        return cds_fail(ctx, CDS_EINVAL, "block_steps must be in [0, 256]");
    ctx->cd_lookahead = block_steps;
    return CDS_OK;
}

int cds_set_cd_speculate(cds_ctx *ctx, int32_t on)
{
    if (!ctx) return CDS_EINVAL;
    if (on != 0 && on != 1) return cds_fail(ctx, CDS_EINVAL, "on must be 0 or 1");
    ctx->cd_speculate = on;
    return CDS_OK;
}

int cds_set_cd_mailbox(cds_ctx *ctx, int32_t on)
{
    if (!ctx) return CDS_EINVAL;
    if (on != 0 && on != 1) return cds_fail(ctx, CDS_EINVAL, "on must be 0 or 1");
    ctx->cd_mailbox = on;
    return CDS_OK;
}

int cds_set_cd_large_path(cds_ctx *ctx, int32_t on)
{
    if (!ctx) return CDS_EINVAL;
    if (on != 0 && on != 1) return cds_fail(ctx, CDS_EINVAL, "on must be 0 or 1");
    ctx->cd_large_path = on;
    return CDS_OK;
}

int cds_set_kernel_timing(cds_ctx *ctx, int32_t on)
{
    if (!ctx) return CDS_EINVAL;
    ctx->kernel_timing = on != 0;
    return CDS_OK;
}

}  // extern "C"
