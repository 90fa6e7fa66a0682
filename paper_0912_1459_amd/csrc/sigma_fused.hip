// Fused second-order self-energy contraction for gfx950 (Sec. II.B of the paper):
//   Eq. (SE)   Sigma_qq(w) = sum_{a,i,j} (2(qi|aj) - (qj|ai)) (qi|aj) / (w + e_a - e_i - e_j)
//                          + sum_{i,a,b} (2(qa|ib) - (qb|ia)) (qa|ib) / (w + e_i - e_a - e_b)
//   Eq. (aomo) (pq|rs) = sum_K B^K_pq B^K_rs
// The MO integrals are formed by FP64 / FP32 / split-bf16 MFMA products and reduced over the
// energy denominators in the same kernel: they never reach HBM.
//
// Both families are matrices Y[r][c] = sum_K P_r^K Q_c^K over one fixed index:
//   part A (2h1p), fixed virtual a:  Y[i][j] = (qi|aj),  P_r = Bsel[q][r],        Q_c = Bvo[a][c]
//   part B (2p1h), fixed occupied i: Y[a][b] = (qa|ib),  P_r = Bsel[q][nocc + r], Q_c = Bvo[c][i]
// with the denominator w + e0 - e_r - e_c (e0 = e_a, resp. e_i).  The exchange partner of
// Y[r][c] is Y[c][r] and both share the denominator, so every unordered pair {r, c}
// contributes R / d once, R = 2 (Y_rc^2 + Y_cr^2 - Y_rc Y_cr) (r != c) or Y_rr^2.
// A workgroup owns one pair of 128-row tiles (TR <= TC) of one matrix: off the diagonal it
// forms Y[TR][TC] and, in the same registers' layout, Y[TC][TR]^T as Q[TR] P[TC]^T (both
// partners of an element sit in one lane); on the diagonal it forms Y[TR][TR] and reads each
// partner through an LDS transpose.  Operand slices (128 rows x 64 bytes per stage and plane) go
// straight from global memory into a ring of LDS stages (global_load_lds_dwordx4; four stages of
// 32 KB in FP64 and FP32, two of 64 KB in split bf16), one barrier per stage, the 16-byte chunks
// of a row XOR-swizzled so the fragment reads of consecutive rows hit distinct banks; 16 x 16
// MFMA blocks entirely past the matrix edge are skipped.  Tasks are ordered so that those sharing their P
// operand slices run at the same time on one XCD.
//
// SIGMA mode: each workgroup sums R / d and -R / d^2 over its elements at T trial energies in
// FP64 (fixed order) and writes one partial per trial energy; a second kernel adds the partials
// of a target in task order.  RESIDUE mode: each workgroup stores R once per element (the pole
// residues), for the Newton sweeps, in a task-major layout: a diagonal task its upper triangle
// packed by rows (8256 entries), an off-diagonal task its 128 x 128 tile by rows.
#include "cds_internal.h"

#include <type_traits>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int FT = 128;                         // tile edge
constexpr int FNT = 512;                        // threads per workgroup: 8 waves, 2 (rows) x 4 (cols)
constexpr int TPITCH = FT + 1;                  // transpose buffer pitch (elements)
constexpr int DIAG_SLOTS = FT * (FT + 1) / 2;   // residues of a diagonal task
constexpr int OFF_SLOTS = FT * FT;              // residues of an off-diagonal task
constexpr int FTT = 8;                          // trial energies per epilogue pass (at most)
// a diagonal task's transposition buffer (after the main loop, over the stage buffers): rows
// 0..63 at byte 0, rows 64..127 at TR_HALF
constexpr int TR_HALF = (FT / 2) * TPITCH * 8;

template <int PREC> struct FTr;
// k per stage, planes, row bytes per plane and stages in the ring: a stage holds four operand
// slices of 128 rows x RB x PL bytes (P[TR], Q[TC], Q[TR], P[TC]); NB stages of 32 KB (FP64,
// FP32) keep three stages in flight under the products of the fourth, in the same 128 KB as
// two stages of 64 KB (split bf16, whose MFMA takes 32 k at once)
template <> struct FTr<CDS_PREC_FP64> {
    typedef double E;
    typedef double A1;
    typedef doublex4 Acc;
    static constexpr int KS = 8, PL = 1, RB = 64, NB = 4;
};
template <> struct FTr<CDS_PREC_FP32> {
    typedef float E;
    typedef float A1;
    typedef floatx4 Acc;
    static constexpr int KS = 16, PL = 1, RB = 64, NB = 4;
};
template <> struct FTr<CDS_PREC_BF16X3> {
    typedef __bf16 E;
    typedef float A1;
    typedef floatx4 Acc;
    static constexpr int KS = 32, PL = 2, RB = 64, NB = 2;
};

struct FArgs {
    const unsigned char *Bsel, *Bvo;            // first (hi) planes
    const unsigned char *Bsel_lo, *Bvo_lo;      // split-bf16 lo planes (else unused)
    int64_t ldk;                                // elements per block row
    int64_t ns;                                 // K stages (the sum runs over ns * KS entries)
    int nmo, nocc, nvirt;
    int nsc;                                    // targets of this launch
    const int *tsel;                            // [nsc] target slot (row block of Bsel)
    int nTA, nTB, nPA, nPB;                     // tiles and tile pairs of parts A and B
    int64_t tpt;                                // tasks per target
    int64_t sizeA, sizeB;                       // residue entries per virtual a / occupied i
    int64_t nres;                               // residue entries per target
    const double *eps;
    const double *omega;                        // [nsc][T] trial energies (SIGMA)
    int T;
    double *part;                               // [nsc][tpt][T][2] partial sums (SIGMA)
    void *R;                                    // [nsc][nres] residues (RESIDUE)
};

struct Task {
    int fam;        // 0: part A (fixed virtual), 1: part B (fixed occupied)
    int idx;        // the fixed index
    int sl;         // target of the launch
    int TR, TC;     // tile pair, TR <= TC
    int pair;
    int64_t tin;    // task index within its target (partials, residue region)
};

// pair p of n tiles in row-major upper-triangle order -> (TR, TC)
__device__ __forceinline__ void pair_tiles(int p, int n, int &TR, int &TC)
{
    int r = 0;
    while (p >= n - r) {
        p -= n - r;
        ++r;
    }
    TR = r;
    TC = r + p;
}

// launch order: part B tasks by (target, pair, i), then part A tasks by (target, pair, a): runs of
// tasks that share the P operand slices (rows of Bsel for one target) and differ only in the Q rows
__device__ __forceinline__ Task task_of_launch(const FArgs &a, int64_t t)
{
    Task k;
    const int64_t nB = (int64_t)a.nocc * a.nsc * a.nPB;
    if (t < nB) {
        k.fam = 1;
        k.idx = (int)(t % a.nocc);
        const int64_t rem = t / a.nocc;
        k.pair = (int)(rem % a.nPB);
        k.sl = (int)(rem / a.nPB);
        pair_tiles(k.pair, a.nTB, k.TR, k.TC);
        k.tin = (int64_t)k.idx * a.nPB + k.pair;
    } else {
        t -= nB;
        k.fam = 0;
        k.idx = (int)(t % a.nvirt);
        const int64_t rem = t / a.nvirt;
        k.pair = (int)(rem % a.nPA);
        k.sl = (int)(rem / a.nPA);
        pair_tiles(k.pair, a.nTA, k.TR, k.TC);
        k.tin = (int64_t)a.nocc * a.nPB + (int64_t)k.idx * a.nPA + k.pair;
    }
    return k;
}

// task within a target (the partial and residue order) -> family, index, tiles
__device__ __forceinline__ Task task_in_target(const FArgs &a, int64_t tin)
{
    Task k;
    k.sl = 0;
    k.tin = tin;
    const int64_t nB = (int64_t)a.nocc * a.nPB;
    if (tin < nB) {
        k.fam = 1;
        k.idx = (int)(tin / a.nPB);
        k.pair = (int)(tin - (int64_t)k.idx * a.nPB);
        pair_tiles(k.pair, a.nTB, k.TR, k.TC);
    } else {
        const int64_t t = tin - nB;
        k.fam = 0;
        k.idx = (int)(t / a.nPA);
        k.pair = (int)(t - (int64_t)k.idx * a.nPA);
        pair_tiles(k.pair, a.nTA, k.TR, k.TC);
    }
    return k;
}

// start of a task's residues within its target's region
__device__ __forceinline__ int64_t residue_offset(const FArgs &a, const Task &k)
{
    const int ndiag = k.TR + (k.TC > k.TR ? 1 : 0);          // diagonal pairs before this one
    const int64_t off = (int64_t)ndiag * DIAG_SLOTS + (int64_t)(k.pair - ndiag) * OFF_SLOTS;
    return k.fam ? (int64_t)k.idx * a.sizeB + off : (int64_t)a.nocc * a.sizeB + (int64_t)k.idx * a.sizeA + off;
}

__device__ __forceinline__ int diag_slot(int r, int c) { return FT * r - r * (r - 1) / 2 + (c - r); }

// chunk position of logical 16-byte chunk lc of slice row rr: 128-byte rows (8 chunks) are
// permuted by rr & 7, 64-byte rows (4 chunks) by (rr >> 1) & 3, so that the 16-byte fragment
// reads of 8 consecutive rows (one LDS cycle) hit 8 different bank groups (measured: 1 % bank
// conflict cycles, against 48 % for a permutation by (rr & 7) ^ ((rr >> 3) & 1))
template <int RB>
__device__ __forceinline__ int chunk_pos(int lc, int rr)
{
    if constexpr (RB == 128) return lc ^ (rr & 7);
    else return lc ^ ((rr >> 1) & 3);
}

// s_waitcnt vmcnt(N) (other counters untouched)
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int PREC, int MODE, int TT>
__global__ __launch_bounds__(FNT, 1) void sigma_fused_kernel(FArgs a)
{
    typedef FTr<PREC> Tr;
    typedef typename Tr::E E;
    typedef typename Tr::A1 A1;
    typedef typename Tr::Acc Acc;
    constexpr int KS = Tr::KS, RB = Tr::RB, PL = Tr::PL, NB = Tr::NB;
    constexpr int ES = (int)sizeof(E);
    constexpr int RPW = 1024 / RB;              // slice rows per wave load (per plane)
    constexpr int LPR = RB / 16;                // lanes per slice row
    constexpr int SL = FT * RB * PL;            // one operand slice
    constexpr int STG = 4 * SL;                 // one stage
    constexpr int PPS = SL / 1024;              // wave loads per slice
    constexpr int LDS_ALL = NB * STG > 2 * TR_HALF ? NB * STG : 2 * TR_HALF;
    static_assert(NB >= 2 && NB <= 4 && PPS * 4 <= 64, "stage ring shape");

    // the stage ring (after the main loop: a diagonal task's transposition buffer)
    __shared__ __align__(16) unsigned char lds[LDS_ALL];
    __shared__ double red[FNT / 64][2 * FTT];
    __shared__ double seps[2][FT];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, r16 = lane & 15;
    const int wr = wave >> 2, wc = wave & 3;
    // workgroups are dealt to the 8 XCDs in turn; each group of 256 consecutive workgroups takes
    // 256 consecutive tasks, 32 per XCD, so the 32 tasks one XCD runs at a time read the same P
    // slices (one target, one tile pair) from its L2 and differ only in their Q rows.  Large
    // workload, FP64 residues: 57.0 ms in the order (index, target, pair) dealt round robin, 53.9
    // ms in the order (target, pair, index) dealt round robin, 53.3 ms with 32 per XCD (64 per
    // XCD: 53.3 ms; order (target, index, pair): 54.7 ms; one contiguous range per XCD: 59.8 ms)
    int64_t tid = blockIdx.x;
    {
        const int64_t full = ((int64_t)gridDim.x / 256) * 256;
        if (tid < full) tid = (tid / 256) * 256 + (tid % 8) * 32 + (tid / 8) % 32;
    }
    const Task k = task_of_launch(a, tid);
    const bool diag = k.TR == k.TC;
    const int n = k.fam ? a.nvirt : a.nocc;
    const int s = a.tsel[k.sl];
    const int64_t pb = (int64_t)s * a.nmo + (k.fam ? a.nocc : 0);     // P row r: Bsel row pb + r
    const int64_t qb = k.fam ? (int64_t)k.idx : (int64_t)k.idx * a.nocc;
    const int64_t qs = k.fam ? a.nocc : 1;                            // Q row c: Bvo row qb + c qs
    const int ebase = k.fam ? a.nocc : 0;
    const double e0 = a.eps[k.fam ? k.idx : a.nocc + k.idx];
    if (threadIdx.x < 2 * FT) {
        const int side = threadIdx.x / FT, rr = threadIdx.x % FT;
        const int gr = min((side ? k.TC : k.TR) * FT + rr, n - 1);
        seps[side][rr] = a.eps[ebase + gr];
    }

    // per-lane source of each wave load of a stage (the stage offset is added per stage):
    // wave load id = wave * nload + i covers slice id / PPS (0 P[TR], 1 Q[TC], 2 Q[TR], 3 P[TC]),
    // part id % PPS (plane part / 8 for split bf16)
    const int nload = diag ? PPS / 4 : PPS / 2; // wave loads per wave and stage
    const unsigned char *src[8];
    unsigned ldst[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int id = wave * nload + i;
        const int sl = id / PPS, part = id % PPS;
        const int plane = PL == 2 ? part >> 3 : 0;
        const int rr = (PL == 2 ? (part & 7) : part) * RPW + lane / LPR;
        const int pc = lane % LPR;
        const int lc = chunk_pos<RB>(pc, rr);
        const bool isP = sl == 0 || sl == 3;
        const int tile = (sl == 0 || sl == 2) ? k.TR : k.TC;
        const int64_t x = min(tile * FT + rr, n - 1);
        const int64_t row = isP ? pb + x : qb + x * qs;
        const unsigned char *base = isP ? (plane ? a.Bsel_lo : a.Bsel) : (plane ? a.Bvo_lo : a.Bvo);
        src[i] = base + (row * a.ldk) * ES + lc * 16;
        ldst[i] = (unsigned)(sl * SL + part * 1024);
    }
    auto stage_load = [&](unsigned char *buf, int64_t st) {
        const int64_t koff = st * KS * ES;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (i < nload)
                cds_lds_dma16(src[i] + koff, buf + ldst[i]);
    };

    // MFMA blocks of this wave inside the matrix (whole 16 x 16 blocks past its edge are skipped)
    const int r0 = k.TR * FT + wr * 64, c0 = k.TC * FT + wc * 32;
    const int nbr = __builtin_amdgcn_readfirstlane(max(0, min(4, (n - r0 + 15) / 16)));
    const int nbc = __builtin_amdgcn_readfirstlane(max(0, min(2, (n - c0 + 15) / 16)));

    Acc acc1[4][2], acc2[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc1[i][j][e] = acc2[i][j][e] = 0;

    // fragment address of slice sl, slice row rr, logical chunk lc (plane pl)
    auto frag = [&](const unsigned char *buf, int sl, int pl, int rr, int lc) {
        return buf + sl * SL + pl * 8192 + rr * RB + chunk_pos<RB>(lc, rr) * 16;
    };
    // one stage of products: acc1 += P[TR] Q[TC]^T, and off the diagonal acc2 += Q[TR] P[TC]^T.
    // Consecutive MFMAs go to different accumulators (each k slot over all blocks in turn).
    auto compute = [&](const unsigned char *buf, auto OFFc, auto FULLc) {
        constexpr bool off = decltype(OFFc)::value;
        constexpr bool full = decltype(FULLc)::value;
        auto on = [&](int i, int j) { return full || (i < nbr && j < nbc); };
        if constexpr (PREC == CDS_PREC_FP64) {
#pragma unroll
            for (int h = 0; h < RB / 64; ++h) {
                const int lc = g + 4 * h;
                double2 fa[4], fb[2], ga[4], gb[2];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    fa[i] = *reinterpret_cast<const double2 *>(frag(buf, 0, 0, wr * 64 + 16 * i + r16, lc));
                    if (off) ga[i] = *reinterpret_cast<const double2 *>(frag(buf, 2, 0, wr * 64 + 16 * i + r16, lc));
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    fb[j] = *reinterpret_cast<const double2 *>(frag(buf, 1, 0, wc * 32 + 16 * j + r16, lc));
                    if (off) gb[j] = *reinterpret_cast<const double2 *>(frag(buf, 3, 0, wc * 32 + 16 * j + r16, lc));
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        if (on(i, j)) {
                            acc1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].x, fb[j].x, acc1[i][j], 0, 0, 0);
                            if (off) acc2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[i].x, gb[j].x, acc2[i][j], 0, 0, 0);
                        }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        if (on(i, j)) {
                            acc1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].y, fb[j].y, acc1[i][j], 0, 0, 0);
                            if (off) acc2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[i].y, gb[j].y, acc2[i][j], 0, 0, 0);
                        }
            }
        } else if constexpr (PREC == CDS_PREC_FP32) {
#pragma unroll
            for (int h = 0; h < RB / 64; ++h) {
                const int lc = g + 4 * h;
                float4 fa[4], fb[2], ga[4], gb[2];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    fa[i] = *reinterpret_cast<const float4 *>(frag(buf, 0, 0, wr * 64 + 16 * i + r16, lc));
                    if (off) ga[i] = *reinterpret_cast<const float4 *>(frag(buf, 2, 0, wr * 64 + 16 * i + r16, lc));
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    fb[j] = *reinterpret_cast<const float4 *>(frag(buf, 1, 0, wc * 32 + 16 * j + r16, lc));
                    if (off) gb[j] = *reinterpret_cast<const float4 *>(frag(buf, 3, 0, wc * 32 + 16 * j + r16, lc));
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            if (on(i, j)) {
                                acc1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i][q], fb[j][q], acc1[i][j], 0, 0, 0);
                                if (off) acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[i][q], gb[j][q], acc2[i][j], 0, 0, 0);
                            }
            }
        } else {
            bf16x8 ah[4], al[4], bh[2], bl[2], gh[4], gl[4], hh[2], hl[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rr = wr * 64 + 16 * i + r16;
                ah[i] = *reinterpret_cast<const bf16x8 *>(frag(buf, 0, 0, rr, g));
                al[i] = *reinterpret_cast<const bf16x8 *>(frag(buf, 0, 1, rr, g));
                if (off) {
                    gh[i] = *reinterpret_cast<const bf16x8 *>(frag(buf, 2, 0, rr, g));
                    gl[i] = *reinterpret_cast<const bf16x8 *>(frag(buf, 2, 1, rr, g));
                }
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int rr = wc * 32 + 16 * j + r16;
                bh[j] = *reinterpret_cast<const bf16x8 *>(frag(buf, 1, 0, rr, g));
                bl[j] = *reinterpret_cast<const bf16x8 *>(frag(buf, 1, 1, rr, g));
                if (off) {
                    hh[j] = *reinterpret_cast<const bf16x8 *>(frag(buf, 3, 0, rr, g));
                    hl[j] = *reinterpret_cast<const bf16x8 *>(frag(buf, 3, 1, rr, g));
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        if (on(i, j)) {
                            // lo*hi, hi*lo, then hi*hi (smallest terms first)
                            acc1[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(q == 0 ? al[i] : ah[i], q == 1 ? bl[j] : bh[j],
                                                                                 acc1[i][j], 0, 0, 0);
                            if (off)
                                acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(q == 0 ? gl[i] : gh[i], q == 1 ? hl[j] : hh[j],
                                                                                     acc2[i][j], 0, 0, 0);
                        }
        }
    };

    // main loop: a ring of NB LDS stages, one barrier per stage.  At stage st the loads of
    // stages st+1 .. st+NB-2 may still run; after the barrier (every wave's loads of stage st
    // have landed and every wave is done with stage st-1) the freed buffer takes stage st+NB-1.
    // With two stages (split bf16) the next stage's loads are issued before the barrier instead,
    // and a second barrier frees the buffer read (measured faster there).
    auto main_loop = [&](auto OFFc, auto FULLc) {
        constexpr bool off = decltype(OFFc)::value;
        constexpr int NL = off ? PPS / 2 : PPS / 4;   // wave loads per wave and stage
        const int64_t ns = a.ns;
        if constexpr (NB == 2) {
            auto step = [&](unsigned char *cur, unsigned char *nxt, int64_t st) {
                if (st + 1 < ns) {
                    stage_load(nxt, st + 1);          // nxt was freed by the last barrier
                    wait_vm<NL>();                    // this wave's loads of stage st have landed
                } else {
                    wait_vm<0>();
                }
                __builtin_amdgcn_s_barrier();         // ... and every wave's
                compute(cur, OFFc, FULLc);
                __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's LDS reads are done
                __builtin_amdgcn_s_barrier();         // cur may be refilled
            };
            stage_load(lds, 0);
            step(lds, lds + STG, 0);
            for (int64_t st = 1; st < ns; st += 2) {
                step(lds + STG, lds, st);
                if (st + 1 < ns) step(lds, lds + STG, st + 1);
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < NB - 1; ++i)
            if (i < ns) stage_load(lds + i * STG, i);
        for (int64_t st = 0; st < ns; ++st) {
            const int64_t later = min((int64_t)NB - 2, ns - 1 - st);
            if (later >= 2) wait_vm<2 * NL>();
            else if (later == 1) wait_vm<NL>();
            else wait_vm<0>();
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");            // no LDS read moves above the barrier
            if (st + NB - 1 < ns) stage_load(lds + ((st + NB - 1) % NB) * STG, st + NB - 1);
            compute(lds + (st % NB) * STG, OFFc, FULLc);
        }
        __builtin_amdgcn_s_waitcnt(0xC07F);           // lgkmcnt(0): this wave's LDS reads are done
        __builtin_amdgcn_s_barrier();                 // ... and every wave's: the ring is free
        asm volatile("" ::: "memory");
    };
    typedef std::integral_constant<bool, true> T_;
    typedef std::integral_constant<bool, false> F_;
    const bool full = nbr == 4 && nbc == 2;
    if (diag) {
        if (full) main_loop(F_(), T_());
        else main_loop(F_(), F_());
    } else {
        if (full) main_loop(T_(), T_());
        else main_loop(T_(), F_());
    }

    // epilogue.  Lane element (i, j, e): tile row rl = wr*64 + 16 i + rowmap(g, e), tile column
    // cl = wc*32 + 16 j + r16 (FP64 MFMA rows g + 4e, FP32-accumulating rows 4g + e)
    // transposition buffer: tile row r at trow(r) (rows 0..63 from byte 0, 64..127 from TR_HALF)
    auto trow = [&](int r) {
        return reinterpret_cast<A1 *>(lds + (r < FT / 2 ? 0 : TR_HALF)) + (r & (FT / 2 - 1)) * TPITCH;
    };
    if (diag) {
        // partners through LDS: tm[rl][cl] = Y[rl][cl]; the stage buffers are free (last barrier)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int rl = wr * 64 + 16 * i + (PREC == CDS_PREC_FP64 ? g + 4 * e : 4 * g + e);
                    const int cl = wc * 32 + 16 * j + r16;
                    trow(rl)[cl] = acc1[i][j][e];
                }
    }
    __syncthreads();
    const int64_t gR0 = (int64_t)k.TR * FT, gC0 = (int64_t)k.TC * FT;
    // element value, its partner and whether it counts
    auto elem = [&](int i, int j, int e, int &rl, int &cl, double &x, double &xt) {
        rl = wr * 64 + 16 * i + (PREC == CDS_PREC_FP64 ? g + 4 * e : 4 * g + e);
        cl = wc * 32 + 16 * j + r16;
        x = (double)acc1[i][j][e];
        xt = diag ? (double)trow(cl)[rl] : (double)acc2[i][j][e];
        return gR0 + rl < n && gC0 + cl < n && (!diag || rl <= cl);
    };
    if constexpr (MODE == 0 || MODE == 2) {
        // MODE 2: the residues as in MODE 1 and, from the stored values, the sums at the one trial
        // energy (the Newton solve's first evaluation, without a sweep over the residues)
        typedef typename std::conditional<PREC == CDS_PREC_FP64, double, float>::type RT;
        RT *Rt = reinterpret_cast<RT *>(a.R) + (MODE == 2 ? (int64_t)k.sl * a.nres + residue_offset(a, k) : 0);
        for (int t0 = 0; t0 < a.T; t0 += TT) {
            double w[TT], s0[TT], s1[TT];
#pragma unroll
            for (int t = 0; t < TT; ++t) {
                w[t] = a.omega[(int64_t)k.sl * a.T + min(t0 + t, a.T - 1)] + e0;
                s0[t] = s1[t] = 0.0;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        int rl, cl;
                        double x, xt;
                        if (!elem(i, j, e, rl, cl, x, xt)) continue;
                        double R = (diag && rl == cl) ? x * x : 2.0 * (x * x + xt * xt - x * xt);
                        if constexpr (MODE == 2) {
                            const RT Rs = (RT)R;
                            Rt[diag ? diag_slot(rl, cl) : rl * FT + cl] = Rs;
                            R = (double)Rs;
                        }
                        const double dd = -seps[0][rl] - seps[1][cl];
#pragma unroll
                        for (int t = 0; t < TT; ++t) {
                            const double id = 1.0 / (w[t] + dd);
                            const double ri = R * id;
                            s0[t] += ri;
                            s1[t] -= ri * id;
                        }
                    }
            // fixed-order reduction: lanes by butterfly, then waves in order
#pragma unroll
            for (int t = 0; t < TT; ++t) {
                const double v0 = wave_sum(s0[t]), v1 = wave_sum(s1[t]);
                if (lane == 0) {
                    red[wave][2 * t] = v0;
                    red[wave][2 * t + 1] = v1;
                }
            }
            __syncthreads();
            if (threadIdx.x < 2 * TT && t0 + (int)threadIdx.x / 2 < a.T) {
                double v = 0.0;
#pragma unroll
                for (int w8 = 0; w8 < FNT / 64; ++w8) v += red[w8][threadIdx.x];
                a.part[(((int64_t)k.sl * a.tpt + k.tin) * a.T + t0) * 2 + threadIdx.x] = v;
            }
            __syncthreads();
        }
    } else {
        typedef typename std::conditional<PREC == CDS_PREC_FP64, double, float>::type RT;
        RT *Rt = reinterpret_cast<RT *>(a.R) + (int64_t)k.sl * a.nres + residue_offset(a, k);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    int rl, cl;
                    double x, xt;
                    if (!elem(i, j, e, rl, cl, x, xt)) continue;
                    const double R = (diag && rl == cl) ? x * x : 2.0 * (x * x + xt * xt - x * xt);
                    Rt[diag ? diag_slot(rl, cl) : rl * FT + cl] = (RT)R;
                }
    }
}

// Newton sweep over the stored residues of one task and one active target at its current
// energy: Sigma = sum R / d, Sigma' = -sum R / d^2 over the task's elements (fixed order).
template <typename RT>
__global__ __launch_bounds__(256) void fused_sweep_kernel(FArgs a, const int *__restrict__ active,
                                                          const int *__restrict__ cnt)
{
    __shared__ double sh[2][4];
    __shared__ double seps[2][FT];
    if (cnt && (int)blockIdx.y >= cnt[0]) return;       // past the targets still iterating
    const int s = active[blockIdx.y];
    const Task k = task_in_target(a, blockIdx.x);
    const bool diag = k.TR == k.TC;
    const int n = k.fam ? a.nvirt : a.nocc;
    const int ebase = k.fam ? a.nocc : 0;
    const double w = a.omega[s] + a.eps[k.fam ? k.idx : a.nocc + k.idx];
    if (threadIdx.x < 2 * FT) {
        // 256 threads: one entry each
        const int side = threadIdx.x / FT, rr = threadIdx.x % FT;
        seps[side][rr] = a.eps[ebase + min((side ? k.TC : k.TR) * FT + rr, n - 1)];
    }
    __syncthreads();
    const RT *Rt = reinterpret_cast<const RT *>(a.R) + (int64_t)s * a.nres + residue_offset(a, k);
    const int nslot = diag ? DIAG_SLOTS : OFF_SLOTS;
    const int gR0 = k.TR * FT, gC0 = k.TC * FT;
    constexpr int SU = 4;
    double s0 = 0.0, s1 = 0.0;
    for (int q0 = threadIdx.x; q0 < nslot; q0 += SU * 256) {
        double rv[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int q = q0 + u * 256;
            rv[u] = (double)Rt[q < nslot ? q : nslot - 1];
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int q = q0 + u * 256;
            if (q >= nslot) break;
            int rl, cl;
            if (diag) {
                // q = rowstart(r) + (c - r), rowstart(r) = r (257 - r) / 2: float root, then an
                // exact integer correction
                rl = (int)((257.0f - sqrtf(66049.0f - 8.0f * (float)q)) * 0.5f);
                if (rl > 0 && rl * (257 - rl) / 2 > q) --rl;
                if ((rl + 1) * (256 - rl) / 2 <= q) ++rl;
                cl = rl + (q - rl * (257 - rl) / 2);
            } else {
                rl = q >> 7;
                cl = q & (FT - 1);
            }
            if (gR0 + rl >= n || gC0 + cl >= n) continue;
            const double id = 1.0 / (w - seps[0][rl] - seps[1][cl]);
            const double ri = rv[u] * id;
            s0 += ri;
            s1 -= ri * id;
        }
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = s0;
        sh[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const double v = ((sh[threadIdx.x][0] + sh[threadIdx.x][1]) + sh[threadIdx.x][2]) + sh[threadIdx.x][3];
        a.part[((int64_t)blockIdx.y * a.tpt + blockIdx.x) * 2 + threadIdx.x] = v;
    }
}

}  // namespace

// ---- host side ---------------------------------------------------------------------------

static int fused_ks(int prec) { return prec == CDS_PREC_FP64 ? 8 : (prec == CDS_PREC_FP32 ? 16 : 32); }

bool cds_fused_plan(int prec, int64_t nvec, int64_t ldk, int nmo, int nocc, const void *Bsel, const void *Bvo,
                    const void *Bsel_lo, const void *Bvo_lo, CdsFusedPlan *p)
{
    const int ks = fused_ks(prec);
    const size_t es = prec == CDS_PREC_FP64 ? 8 : (prec == CDS_PREC_FP32 ? 4 : 2);
    const int64_t kp = cds_ceil_div(nvec, ks) * ks;
    if (kp > ldk || (ldk * (int64_t)es) % 16 != 0) return false;
    if (!cds_aligned(Bsel, 16) || !cds_aligned(Bvo, 16)) return false;
    if (prec == CDS_PREC_BF16X3 && (!cds_aligned(Bsel_lo, 16) || !cds_aligned(Bvo_lo, 16))) return false;
    const int nvirt = nmo - nocc;
    p->ns = kp / ks;
    p->nTA = (int)cds_ceil_div(nocc, FT);
    p->nTB = (int)cds_ceil_div(nvirt, FT);
    p->nPA = p->nTA * (p->nTA + 1) / 2;
    p->nPB = p->nTB * (p->nTB + 1) / 2;
    p->tpt = (int64_t)nocc * p->nPB + (int64_t)nvirt * p->nPA;
    p->sizeA = (int64_t)p->nTA * DIAG_SLOTS + (int64_t)(p->nPA - p->nTA) * OFF_SLOTS;
    p->sizeB = (int64_t)p->nTB * DIAG_SLOTS + (int64_t)(p->nPB - p->nTB) * OFF_SLOTS;
    p->nres = (int64_t)nvirt * p->sizeA + (int64_t)nocc * p->sizeB;
    return true;
}

static FArgs fused_args(int prec, const CdsFusedPlan &p, int64_t ldk, int nmo, int nocc, int nsc, const int *tsel,
                        const void *Bsel, const void *Bvo, const void *Bsel_lo, const void *Bvo_lo,
                        const double *eps)
{
    FArgs a = {};
    a.Bsel = (const unsigned char *)Bsel;
    a.Bvo = (const unsigned char *)Bvo;
    a.Bsel_lo = (const unsigned char *)(prec == CDS_PREC_BF16X3 ? Bsel_lo : Bsel);
    a.Bvo_lo = (const unsigned char *)(prec == CDS_PREC_BF16X3 ? Bvo_lo : Bvo);
    a.ldk = ldk;
    a.ns = p.ns;
    a.nmo = nmo;
    a.nocc = nocc;
    a.nvirt = nmo - nocc;
    a.nsc = nsc;
    a.tsel = tsel;
    a.nTA = p.nTA;
    a.nTB = p.nTB;
    a.nPA = p.nPA;
    a.nPB = p.nPB;
    a.tpt = p.tpt;
    a.sizeA = p.sizeA;
    a.sizeB = p.sizeB;
    a.nres = p.nres;
    a.eps = eps;
    return a;
}

template <int PREC, int MODE>
static void launch_fused_t(cds_ctx *ctx, const FArgs &a, unsigned nblk, int T)
{
    if (MODE == 1) hipLaunchKernelGGL((sigma_fused_kernel<PREC, 1, 1>), dim3(nblk), dim3(FNT), 0, ctx->stream, a);
    else if (MODE == 2) hipLaunchKernelGGL((sigma_fused_kernel<PREC, 2, 1>), dim3(nblk), dim3(FNT), 0, ctx->stream, a);
    else if (T <= 1) hipLaunchKernelGGL((sigma_fused_kernel<PREC, 0, 1>), dim3(nblk), dim3(FNT), 0, ctx->stream, a);
    else if (T <= 2) hipLaunchKernelGGL((sigma_fused_kernel<PREC, 0, 2>), dim3(nblk), dim3(FNT), 0, ctx->stream, a);
    else if (T <= 4) hipLaunchKernelGGL((sigma_fused_kernel<PREC, 0, 4>), dim3(nblk), dim3(FNT), 0, ctx->stream, a);
    else hipLaunchKernelGGL((sigma_fused_kernel<PREC, 0, 8>), dim3(nblk), dim3(FNT), 0, ctx->stream, a);
}

template <int MODE>
static int launch_fused(cds_ctx *ctx, int prec, const FArgs &a, int T)
{
    const int64_t nblk = (int64_t)a.nsc * a.tpt;
    if (nblk > 0x7fffffffLL) return cds_fail(ctx, CDS_EINVAL, "fused contraction: %lld tasks", (long long)nblk);
    if (prec == CDS_PREC_FP64) launch_fused_t<CDS_PREC_FP64, MODE>(ctx, a, (unsigned)nblk, T);
    else if (prec == CDS_PREC_FP32) launch_fused_t<CDS_PREC_FP32, MODE>(ctx, a, (unsigned)nblk, T);
    else launch_fused_t<CDS_PREC_BF16X3, MODE>(ctx, a, (unsigned)nblk, T);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}

int cds_fused_sigma(cds_ctx *ctx, int prec, const CdsFusedPlan &p, int64_t ldk, int nmo, int nocc, int nsc,
                    const int *d_tsel, const void *Bsel, const void *Bvo, const void *Bsel_lo, const void *Bvo_lo,
                    const double *eps, const double *d_omega, int T, double *d_part)
{
    FArgs a = fused_args(prec, p, ldk, nmo, nocc, nsc, d_tsel, Bsel, Bvo, Bsel_lo, Bvo_lo, eps);
    a.omega = d_omega;
    a.T = T;
    a.part = d_part;
    return launch_fused<0>(ctx, prec, a, T);
}

int cds_fused_residues(cds_ctx *ctx, int prec, const CdsFusedPlan &p, int64_t ldk, int nmo, int nocc, int nsc,
                       const int *d_tsel, const void *Bsel, const void *Bvo, const void *Bsel_lo, const void *Bvo_lo,
                       const double *eps, void *R, const double *d_omega0, double *d_part)
{
    FArgs a = fused_args(prec, p, ldk, nmo, nocc, nsc, d_tsel, Bsel, Bvo, Bsel_lo, Bvo_lo, eps);
    a.R = R;
    if (!d_part) return launch_fused<1>(ctx, prec, a, 1);
    a.omega = d_omega0;
    a.T = 1;
    a.part = d_part;
    return launch_fused<2>(ctx, prec, a, 1);
}

int cds_fused_sweep(cds_ctx *ctx, int prec, const CdsFusedPlan &p, int nmo, int nocc, int nactive,
                    const int *d_active, const double *eps, const double *d_omega, const void *R, double *d_part,
                    const int *d_cnt)
{
    FArgs a = fused_args(prec, p, 0, nmo, nocc, 1, nullptr, nullptr, nullptr, nullptr, nullptr, eps);
    a.omega = d_omega;
    a.R = const_cast<void *>(R);
    a.part = d_part;
    if (p.tpt > 0x7fffffffLL || nactive > 65535)
        return cds_fail(ctx, CDS_EINVAL, "fused sweep grid %lld x %d", (long long)p.tpt, nactive);
    const dim3 grid((unsigned)p.tpt, (unsigned)nactive);
    if (prec == CDS_PREC_FP64)
        hipLaunchKernelGGL(fused_sweep_kernel<double>, grid, dim3(256), 0, ctx->stream, a, d_active, d_cnt);
    else
        hipLaunchKernelGGL(fused_sweep_kernel<float>, grid, dim3(256), 0, ctx->stream, a, d_active, d_cnt);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}
