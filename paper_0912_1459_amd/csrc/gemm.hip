// MFMA GEMM engine for gfx950 used by the transform, the contraction and the
// adjoint:  C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n), batched.
//
// Tile 128 x 128 per workgroup of 256 threads (4 waves in 2 x 2, 64 x 64 per
// wave = 4 x 4 blocks of 16 x 16 MFMA outputs).  Both operands are staged in
// LDS as [row][k] with k contiguous (row = m for A, n for B), 128 bytes of k
// per stage and a 144-byte row pitch, so that the per-lane 16-byte fragment
// reads (ds_read_b128) of eight consecutive rows fall into distinct banks.
//
// Precisions
//   FP64   : v_mfma_f64_16x16x4_f64, 16 k per stage
//   FP32   : v_mfma_f32_16x16x4_f32, 32 k per stage
//   BF16X3 : operands stored as two bf16 planes (hi, lo) with x ~ hi + lo;
//            a*b ~ hi*hi + hi*lo + lo*hi, three v_mfma_f32_16x16x32_bf16 per
//            block and 32-k slice, FP32 accumulation; 64 k per stage
//
// MFMA lane layout (16 x 16 output, measured on gfx950): lane l holds column
// l%16; for the f32-accumulating MFMAs its four values are rows 4*(l/16)+e,
// for v_mfma_f64_16x16x4f64 rows (l/16)+4*e, e = 0..3.  Operand A supplies
// row l%16, operand B column l%16.  The k index carried by a lane is permuted consistently for A and B
// (lane group g = l/16 reads 16-byte chunks g and g+4 of the 128-byte k
// slice), which leaves the k-sum unchanged.
#include "cds_internal.h"

#include <type_traits>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, NT = 256;
constexpr int PITCH = 144;      // LDS row pitch in bytes

struct Args {
    int64_t M, N, K, batch;
    const unsigned char *A, *Alo;  // Alo: lo plane (BF16X3 only)
    int64_t sAm, sAk, sAb;
    const unsigned char *B, *Blo;
    int64_t sBk, sBn, sBb;
    unsigned char *C, *Clo;        // Clo: split output (BF16X3, see GemmDesc)
    int64_t sCm, sCn, sCb;
    double alpha, beta;
    int fastA, fastB;              // K-contiguous, 16-byte aligned rows, K % KB == 0
    int big;                       // GemmDesc::big
};

template <int PREC> struct Tr;
template <> struct Tr<CDS_PREC_FP64> {
    typedef double E;   // element type in memory / LDS
    typedef double O;   // output type
    static constexpr int KB = 16, PLANES = 1;
};
template <> struct Tr<CDS_PREC_FP32> {
    typedef float E;
    typedef float O;
    static constexpr int KB = 32, PLANES = 1;
};
template <> struct Tr<CDS_PREC_BF16X3> {
    typedef __bf16 E;
    typedef float O;
    static constexpr int KB = 64, PLANES = 2;
};

// stage one operand tile (128 rows x KB k) into LDS (per plane)
template <int PREC>
__device__ __forceinline__ void load_tile(const Args &a, bool isA, int64_t row0, int64_t k0,
                                          int64_t batch, uint4 (&reg)[2][4], int fast)
{
    typedef typename Tr<PREC>::E E;
    const int64_t nrows = isA ? a.M : a.N;
    const int64_t srow = isA ? a.sAm : a.sBn;
    const int64_t sk = isA ? a.sAk : a.sBk;
    const int64_t sb = isA ? a.sAb : a.sBb;
    const unsigned char *base[2] = {isA ? a.A : a.B, isA ? a.Alo : a.Blo};
#pragma unroll
    for (int pl = 0; pl < Tr<PREC>::PLANES; ++pl) {
        const E *P = reinterpret_cast<const E *>(base[pl]) + batch * sb;
        if (fast) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int c = threadIdx.x + NT * i;       // 16-byte chunk id in the 128 x 128 B tile
                int r = c >> 3, q = c & 7;
                int64_t row = row0 + r;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (row < nrows)
                    v = *reinterpret_cast<const uint4 *>(P + row * srow + k0 + q * (16 / sizeof(E)));
                reg[pl][i] = v;
            }
        } else {
            // generic strided gather, element by element
            constexpr int EPC = 16 / sizeof(E);   // elements per chunk
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int c = threadIdx.x + NT * i;
                int r, q;
                if (sk != 1 && srow == 1) {           // rows contiguous: walk rows fastest
                    r = c & 127;
                    q = c >> 7;
                } else {
                    r = c >> 3;
                    q = c & 7;
                }
                int64_t row = row0 + r;
                E tmp[EPC];
#pragma unroll
                for (int e = 0; e < EPC; ++e) {
                    int64_t kk = k0 + q * EPC + e;
                    tmp[e] = (row < nrows && kk < a.K) ? P[row * srow + kk * sk] : (E)0;
                }
                reg[pl][i] = *reinterpret_cast<uint4 *>(tmp);
            }
        }
    }
}

template <int PREC>
__device__ __forceinline__ void store_tile(unsigned char *lds, const uint4 (&reg)[2][4], bool rows_fast,
                                           bool generic_rowsfast)
{
#pragma unroll
    for (int pl = 0; pl < Tr<PREC>::PLANES; ++pl)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int c = threadIdx.x + NT * i;
            int r, q;
            if (generic_rowsfast) {
                r = c & 127;
                q = c >> 7;
            } else {
                r = c >> 3;
                q = c & 7;
            }
            *reinterpret_cast<uint4 *>(lds + pl * (BM * PITCH) + r * PITCH + q * 16) = reg[pl][i];
        }
    (void)rows_fast;
}

// result element idx as a hi/lo pair of bf16 planes (x ~ hi + lo)
__device__ __forceinline__ void split_store(const Args &a, int64_t idx, float x)
{
    const __bf16 hi = (__bf16)x;
    reinterpret_cast<__bf16 *>(a.C)[idx] = hi;
    reinterpret_cast<__bf16 *>(a.Clo)[idx] = (__bf16)(x - (float)hi);
}

template <int PREC>
__global__ __launch_bounds__(NT, PREC == CDS_PREC_FP64 ? 1 : 2) void gemm_kernel(Args a)
{
    typedef typename Tr<PREC>::O O;
    constexpr int PL = Tr<PREC>::PLANES;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned char *ldsA = smem;
    unsigned char *ldsB = smem + PL * BM * PITCH;

    const int64_t n0 = (int64_t)blockIdx.x * BN;
    const int64_t m0 = (int64_t)blockIdx.y * BM;
    const int64_t batch = blockIdx.z;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int g = lane >> 4, r16 = lane & 15;
    constexpr int KB = Tr<PREC>::KB;
    const int64_t nk = cds_ceil_div(a.K, KB);

    const bool gA = !a.fastA && (a.sAk != 1 && a.sAm == 1);
    const bool gB = !a.fastB && (a.sBk != 1 && a.sBn == 1);
    // a wave whose 64 x 64 block lies wholly outside C only helps to stage the operands
    const bool live = m0 + wm < a.M && n0 + wn < a.N;

    typedef typename std::conditional<PREC == CDS_PREC_FP64, doublex4, floatx4>::type Acc;
    Acc acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

    uint4 ra[2][4], rb[2][4];
    load_tile<PREC>(a, true, m0, 0, batch, ra, a.fastA);
    load_tile<PREC>(a, false, n0, 0, batch, rb, a.fastB);

    for (int64_t kt = 0; kt < nk; ++kt) {
        __syncthreads();
        store_tile<PREC>(ldsA, ra, true, gA);
        store_tile<PREC>(ldsB, rb, true, gB);
        __syncthreads();
        if (kt + 1 < nk) {
            load_tile<PREC>(a, true, m0, (kt + 1) * KB, batch, ra, a.fastA);
            load_tile<PREC>(a, false, n0, (kt + 1) * KB, batch, rb, a.fastB);
        }
        if (!live) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int off = (g + 4 * h) * 16;
            if constexpr (PREC == CDS_PREC_FP64) {
                double2 fa[4], fb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    fa[i] = *reinterpret_cast<const double2 *>(ldsA + (wm + 16 * i + r16) * PITCH + off);
                    fb[i] = *reinterpret_cast<const double2 *>(ldsB + (wn + 16 * i + r16) * PITCH + off);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].x, fb[j].x, acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].y, fb[j].y, acc[i][j], 0, 0, 0);
                    }
            } else if constexpr (PREC == CDS_PREC_FP32) {
                float4 fa[4], fb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    fa[i] = *reinterpret_cast<const float4 *>(ldsA + (wm + 16 * i + r16) * PITCH + off);
                    fb[i] = *reinterpret_cast<const float4 *>(ldsB + (wn + 16 * i + r16) * PITCH + off);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].x, fb[j].x, acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].y, fb[j].y, acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].z, fb[j].z, acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i].w, fb[j].w, acc[i][j], 0, 0, 0);
                    }
            } else {
                bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    ah[i] = *reinterpret_cast<const bf16x8 *>(ldsA + (wm + 16 * i + r16) * PITCH + off);
                    al[i] = *reinterpret_cast<const bf16x8 *>(ldsA + BM * PITCH + (wm + 16 * i + r16) * PITCH + off);
                    bh[i] = *reinterpret_cast<const bf16x8 *>(ldsB + (wn + 16 * i + r16) * PITCH + off);
                    bl[i] = *reinterpret_cast<const bf16x8 *>(ldsB + BM * PITCH + (wn + 16 * i + r16) * PITCH + off);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                    }
            }
        }
    }

    // epilogue: C = alpha * acc + beta * C (or the split planes of alpha * acc)
    O *C = reinterpret_cast<O *>(a.C) + batch * a.sCb;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t n = n0 + wn + 16 * j + r16;
            if (n >= a.N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // f32/bf16 MFMA: lane group g holds rows 4g..4g+3; f64: rows g, g+4, g+8, g+12
                const int64_t m = m0 + wm + 16 * i + (PREC == CDS_PREC_FP64 ? g + 4 * e : 4 * g + e);
                if (m >= a.M) continue;
                if constexpr (PREC == CDS_PREC_BF16X3) {
                    if (a.Clo) {
                        split_store(a, batch * a.sCb + m * a.sCm + n * a.sCn, (float)(a.alpha * (double)acc[i][j][e]));
                        continue;
                    }
                }
                O *dst = C + m * a.sCm + n * a.sCn;
                double v = a.alpha * (double)acc[i][j][e];
                if (a.beta != 0.0) v += a.beta * (double)(*dst);
                *dst = (O)v;
            }
        }
}

// ---- large split-bf16 GEMM -------------------------------------------------------
// 256 x 256 tile per workgroup of 512 threads (8 waves in 2 x 4, 128 x 64 per wave = 8 x 4
// blocks of 16 x 16, three v_mfma_f32_16x16x32_bf16 per block and 32-k stage), for the
// products big enough to fill the chip with such tiles.  Operand tiles (two bf16 planes
// each) go straight from global memory to LDS (global_load_lds_dwordx4: lane t of a load
// writes LDS bytes 16t..16t+15 after the wave's base), double-buffered by stage; the
// 16-byte k-chunks of a row are stored XOR-swizzled by (row >> 1) & 3 (the swizzle is
// applied to the global address), so the fragment reads of 8 consecutive rows hit distinct
// banks.  The stage waits are explicit (vmcnt, then s_barrier without a memory fence, which
// would also wait for the next stage's loads).  Tiles of one XCD are contiguous in a grouped
// order (4 tile rows x all tile columns), so tiles that share operand rows run on the same
// L2.
constexpr int GB_M = 256, GB_N = 256, GB_K = 32, GB_NT = 512, GB_GM = 4;
constexpr int GB_PLANE = GB_M * GB_K * 2;       // bytes of one operand plane per stage (16 KB)
constexpr int GB_STAGE = 4 * GB_PLANE;          // A hi, A lo, B hi, B lo (64 KB)


// s_waitcnt with vmcnt = n (expcnt, lgkmcnt left alone)
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// one stage (32 k) of both operands into LDS stage buffer `buf`: 64 wave loads of 1 KB
// (16 rows x 64 bytes), 8 per wave
__device__ __forceinline__ void gb_stage(const Args &a, unsigned char *buf, int64_t m0, int64_t n0, int64_t k0,
                                         int64_t batch, int wave, int lane)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int id = wave * 8 + i;           // 0..63: operand plane (4) x row group (16)
        const int op = id >> 4, rg = id & 15;  // op: 0 A hi, 1 A lo, 2 B hi, 3 B lo
        const bool isA = op < 2;
        const int row = rg * 16 + (lane >> 2);
        const int pos = lane & 3;
        const int chunk = pos ^ ((row >> 1) & 3);
        const int64_t nrows = isA ? a.M : a.N;
        const int64_t grow = min((isA ? m0 : n0) + row, nrows - 1);
        const unsigned char *base = isA ? (op == 0 ? a.A : a.Alo) : (op == 2 ? a.B : a.Blo);
        const int64_t srow = isA ? a.sAm : a.sBn, sb = isA ? a.sAb : a.sBb;
        const __bf16 *src = reinterpret_cast<const __bf16 *>(base) + batch * sb + grow * srow + k0 + chunk * 8;
        cds_lds_dma16(src, buf + op * GB_PLANE + rg * 1024);
    }
}

__global__ __launch_bounds__(GB_NT, 1) void gemm_bf16x3_big_kernel(Args a, int64_t tiles_m, int64_t tiles_n)
{
    __shared__ __align__(16) unsigned char lds0[GB_STAGE];
    __shared__ __align__(16) unsigned char lds1[GB_STAGE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int wm = (wave >> 2) * 128, wn = (wave & 3) * 64;
    const int64_t batch = blockIdx.y;
    // tile of this workgroup: contiguous ranges per XCD (workgroups go round-robin over the 8)
    const int64_t T = tiles_m * tiles_n, bid = blockIdx.x;
    const int64_t q8 = T / 8, r8 = T % 8, xcd = bid % 8, j = bid / 8;
    const int64_t t = xcd * q8 + min(xcd, r8) + j;
    const int64_t gsz = GB_GM * tiles_n, grp = t / gsz, rem = t % gsz;
    const int64_t gm = min((int64_t)GB_GM, tiles_m - grp * GB_GM);
    const int64_t tm = grp * GB_GM + rem % gm, tn = rem / gm;
    const int64_t m0 = tm * GB_M, n0 = tn * GB_N;
    const int64_t ns = a.K / GB_K;

    floatx4 acc[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[i][jj] = floatx4{0.f, 0.f, 0.f, 0.f};

    auto compute = [&](const unsigned char *buf) {
        bf16x8 bh[4], bl[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int row = wn + 16 * jj + r16;
            const int off = row * 64 + ((g ^ ((row >> 1) & 3)) * 16);
            bh[jj] = *reinterpret_cast<const bf16x8 *>(buf + 2 * GB_PLANE + off);
            bl[jj] = *reinterpret_cast<const bf16x8 *>(buf + 3 * GB_PLANE + off);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf16x8 ah[4], al[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = wm + 16 * (4 * h + i) + r16;
                const int off = row * 64 + ((g ^ ((row >> 1) & 3)) * 16);
                ah[i] = *reinterpret_cast<const bf16x8 *>(buf + off);
                al[i] = *reinterpret_cast<const bf16x8 *>(buf + GB_PLANE + off);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    floatx4 &c = acc[4 * h + i][jj];
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[jj], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[jj], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[jj], c, 0, 0, 0);
                }
        }
    };

    gb_stage(a, lds0, m0, n0, 0, batch, wave, lane);
    for (int64_t s = 0; s < ns; ++s) {
        unsigned char *cur = (s & 1) ? lds1 : lds0;
        unsigned char *nxt = (s & 1) ? lds0 : lds1;
        if (s + 1 < ns) {
            gb_stage(a, nxt, m0, n0, (s + 1) * GB_K, batch, wave, lane);   // nxt was freed by the last barrier
            wait_vm<8>();                      // this wave's loads of stage s have landed
        } else {
            wait_vm<0>();
        }
        __builtin_amdgcn_s_barrier();          // ... and every wave's
        compute(cur);
        __builtin_amdgcn_s_waitcnt(0xC07F);    // lgkmcnt(0): this wave's reads of cur are done
        __builtin_amdgcn_s_barrier();          // cur may be refilled
    }

    float *C = reinterpret_cast<float *>(a.C) + batch * a.sCb;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int64_t n = n0 + wn + 16 * jj + r16;
            if (n >= a.N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t m = m0 + wm + 16 * i + 4 * g + e;
                if (m >= a.M) continue;
                if (a.Clo) {
                    split_store(a, batch * a.sCb + m * a.sCm + n * a.sCn, (float)(a.alpha * (double)acc[i][jj][e]));
                    continue;
                }
                float *dst = C + m * a.sCm + n * a.sCn;
                double v = a.alpha * (double)acc[i][jj][e];
                if (a.beta != 0.0) v += a.beta * (double)(*dst);
                *dst = (float)v;
            }
        }
}

bool fast_ok(const void *p, int64_t srow, int64_t sk, int64_t K, int kb, size_t esz)
{
    return sk == 1 && K % kb == 0 && cds_aligned(p, 16) && (srow * (int64_t)esz) % 16 == 0;
}

// ---- FP64 GEMM with direct-to-LDS operand stages -------------------------------------------
// For K-contiguous FP64 operands (rows 16-byte aligned, K % 16 == 0): 128 x 128 tile per
// 512-thread workgroup, 8 waves in 2 x 4 with 64 x 32 each (v_mfma_f64_16x16x4f64, 8 blocks),
// 16-k stages of both operands (128 rows x 128 bytes each) loaded straight from global memory
// into LDS with global_load_lds_dwordx4, G64_NB stages in the ring (G64_NB - 1 in flight), the
// 16-byte chunks of a row XOR-swizzled by row & 7 so the fragment reads of 8 consecutive rows hit
// distinct banks.  Two stages of 32 KB and two workgroups per CU (measured on the large workload:
// adjoint of the solve 154 ms against 169 / 164 ms for one workgroup with three / four stages;
// the 128 x 128 register-staged kernel took 222 ms).  Each output takes its K terms in the same
// order as in gemm_kernel's FP64
// path (stages of 16 in order, within a stage k pairs (2c, 2c+1) for chunk c in the order
// c = g, g + 4 of the lane groups), so the two kernels agree bit for bit.
constexpr int G64_NT = 512, G64_KS = 16, G64_SLICE = 16384, G64_STAGE = 2 * G64_SLICE, G64_NB = 2;

static_assert(G64_NB >= 2 && G64_NB <= 4, "the stage waits cover rings of 2 to 4 stages");

template <int N>
__device__ __forceinline__ void g64_wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

__global__ __launch_bounds__(G64_NT, 2) void gemm64_dma_kernel(Args a)
{
    __shared__ __align__(16) unsigned char lds[G64_NB * G64_STAGE];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, r16 = lane & 15;
    const int wr = wave >> 2, wc = wave & 3;
    const int64_t n0 = (int64_t)blockIdx.x * BN, m0 = (int64_t)blockIdx.y * BM, batch = blockIdx.z;
    const int64_t ns = a.K / G64_KS;
    // this wave's four loads per stage: slice sl (0 A, 1 B), rows 8 q + lane / 8 for q in
    // [4 (wave & 3), 4 (wave & 3) + 4), position lane % 8 holding the swizzled logical chunk
    const int sl = wave >> 2;
    const int lrow = lane >> 3, pc = lane & 7;
    const unsigned char *mat = sl ? a.B : a.A;
    const int64_t srow = sl ? a.sBn : a.sAm, sb = sl ? a.sBb : a.sAb;
    const int64_t nrows = sl ? a.N : a.M, r0g = sl ? n0 : m0;
    const unsigned char *src[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int rr = 8 * (4 * (wave & 3) + q) + lrow;
        const int64_t row = min(r0g + rr, nrows - 1);
        src[q] = mat + ((batch * sb + row * srow) * 8) + ((pc ^ (rr & 7)) * 16);
    }
    auto stage_load = [&](int buf, int64_t st) __attribute__((always_inline)) {
        unsigned char *dst = lds + buf * G64_STAGE + sl * G64_SLICE + (4 * (wave & 3)) * 1024;
#pragma unroll
        for (int q = 0; q < 4; ++q) cds_lds_dma16(src[q] + st * G64_KS * 8, dst + q * 1024);
    };
    doublex4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    auto frag = [&](const unsigned char *buf, int slc, int rr, int lc) __attribute__((always_inline)) {
        return *reinterpret_cast<const double2 *>(buf + slc * G64_SLICE + rr * 128 + ((lc ^ (rr & 7)) * 16));
    };
    // prologue: stages 0 .. NB - 2 in flight
#pragma unroll
    for (int i = 0; i < G64_NB - 1; ++i)
        if (i < ns) stage_load(i, i);
    for (int64_t st = 0; st < ns; ++st) {
        const int buf = (int)(st % G64_NB);
        // this wave's loads of stage st have landed (4 loads per later stage may still be in flight)
        const int64_t later = min((int64_t)(G64_NB - 2), ns - 1 - st);
        if (later >= 2) g64_wait_vm<8>();
        else if (later == 1) g64_wait_vm<4>();
        else g64_wait_vm<0>();
        __builtin_amdgcn_s_barrier();                      // every wave's; and stage st - 1 is read
        if (st + G64_NB - 1 < ns) stage_load((int)((st + G64_NB - 1) % G64_NB), st + G64_NB - 1);
        const unsigned char *cur = lds + buf * G64_STAGE;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int lc = g + 4 * h;
            double2 fa[4], fb[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) fa[i] = frag(cur, 0, wr * 64 + 16 * i + r16, lc);
#pragma unroll
            for (int j = 0; j < 2; ++j) fb[j] = frag(cur, 1, wc * 32 + 16 * j + r16, lc);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].x, fb[j].x, acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].y, fb[j].y, acc[i][j], 0, 0, 0);
                }
        }
        __builtin_amdgcn_s_waitcnt(0xC07F);                // lgkmcnt(0): this wave's reads are done
    }
    double *C = reinterpret_cast<double *>(a.C) + batch * a.sCb;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t n = n0 + wc * 32 + 16 * j + r16;
            if (n >= a.N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t m = m0 + wr * 64 + 16 * i + g + 4 * e;
                if (m >= a.M) continue;
                double *dst = C + m * a.sCm + n * a.sCn;
                double v = a.alpha * acc[i][j][e];
                if (a.beta != 0.0) v += a.beta * (*dst);
                *dst = v;
            }
        }
}

template <int PREC>
int launch(cds_ctx *ctx, Args &a)
{
    typedef typename Tr<PREC>::E E;
    constexpr int KB = Tr<PREC>::KB;
    a.fastA = fast_ok(a.A, a.sAm, a.sAk, a.K, KB, sizeof(E)) &&
              (PREC != CDS_PREC_BF16X3 || cds_aligned(a.Alo, 16));
    a.fastB = fast_ok(a.B, a.sBn, a.sBk, a.K, KB, sizeof(E)) &&
              (PREC != CDS_PREC_BF16X3 || cds_aligned(a.Blo, 16));
    if (PREC == CDS_PREC_BF16X3 && (!a.fastA || !a.fastB))
        return cds_fail(ctx, CDS_EINVAL, "bf16x3 GEMM needs K-contiguous 16-byte aligned operands");
    if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return CDS_OK;
    int64_t gx = cds_ceil_div(a.N, BN), gy = cds_ceil_div(a.M, BM);
    if (gy > 65535 || a.batch > 65535)
        return cds_fail(ctx, CDS_EINVAL, "GEMM grid too large (%lld x %lld x %lld)", (long long)gx,
                        (long long)gy, (long long)a.batch);
    const bool want_big = a.big == 0 ? (a.M >= 512 && a.N >= 512) : a.big == 2;
    if (PREC == CDS_PREC_BF16X3 && want_big && a.K % GB_K == 0 &&
        cds_aligned(a.A, 16) && cds_aligned(a.Alo, 16) && cds_aligned(a.B, 16) && cds_aligned(a.Blo, 16)) {
        const int64_t tm = cds_ceil_div(a.M, GB_M), tn = cds_ceil_div(a.N, GB_N);
        if (tm * tn <= 0x7fffffff) {
            hipLaunchKernelGGL(gemm_bf16x3_big_kernel, dim3((unsigned)(tm * tn), (unsigned)a.batch), dim3(GB_NT), 0,
                               ctx->stream, a, tm, tn);
            CDS_LAUNCHED(ctx);
            return CDS_OK;
        }
    }
    if (PREC == CDS_PREC_FP64 && a.fastA && a.fastB && a.K % G64_KS == 0 && cds_aligned(a.A, 16) &&
        cds_aligned(a.B, 16) && (a.sAb * 8) % 16 == 0 && (a.sBb * 8) % 16 == 0) {
        hipLaunchKernelGGL(gemm64_dma_kernel, dim3((unsigned)gx, (unsigned)gy, (unsigned)a.batch), dim3(G64_NT), 0,
                           ctx->stream, a);
        CDS_LAUNCHED(ctx);
        return CDS_OK;
    }
    size_t lds = (size_t)2 * Tr<PREC>::PLANES * BM * PITCH;
    hipLaunchKernelGGL(gemm_kernel<PREC>, dim3((unsigned)gx, (unsigned)gy, (unsigned)a.batch), dim3(NT),
                       lds, ctx->stream, a);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}

}  // namespace

namespace {
// 32 x 32 tiles through LDS (33-word pitch), every load of a thread in flight before its stores
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T *__restrict__ in, int64_t ldi, T *__restrict__ out,
                                                        int64_t ldo, int64_t rows, int64_t cols)
{
    __shared__ T t[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t r = r0 + ty + 8 * u, c = c0 + tx;
        v[u] = (r < rows && c < cols) ? in[r * ldi + c] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) t[ty + 8 * u][tx] = v[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t c = c0 + ty + 8 * u, r = r0 + tx;
        if (r < rows && c < cols) out[c * ldo + r] = t[tx][ty + 8 * u];
    }
}
}  // namespace

int cds_transpose(cds_ctx *ctx, int es, int64_t rows, int64_t cols, const void *in, int64_t ldi, void *out,
                  int64_t ldo)
{
    CDS_REQUIRE(ctx, es == 4 || es == 8, "transpose: element size %d", es);
    CDS_REQUIRE(ctx, rows >= 0 && cols >= 0 && ldi >= cols && ldo >= rows, "transpose: bad shape");
    if (rows == 0 || cols == 0) return CDS_OK;
    CDS_REQUIRE(ctx, cds_ceil_div(rows, 32) <= 65535, "transpose: too many rows");
    const dim3 g((unsigned)cds_ceil_div(cols, 32), (unsigned)cds_ceil_div(rows, 32));
    if (es == 8)
        hipLaunchKernelGGL(transpose_kernel<double>, g, dim3(256), 0, ctx->stream, (const double *)in, ldi,
                           (double *)out, ldo, rows, cols);
    else
        hipLaunchKernelGGL(transpose_kernel<float>, g, dim3(256), 0, ctx->stream, (const float *)in, ldi,
                           (float *)out, ldo, rows, cols);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}

int cds_gemm_ex(cds_ctx *ctx, int prec, const GemmDesc &d, const void *Alo, const void *Blo)
{
    Args a;
    a.M = d.M;
    a.N = d.N;
    a.K = d.K;
    a.batch = d.batch;
    a.A = (const unsigned char *)d.A;
    a.Alo = (const unsigned char *)Alo;
    a.sAm = d.sAm;
    a.sAk = d.sAk;
    a.sAb = d.sAb;
    a.B = (const unsigned char *)d.B;
    a.Blo = (const unsigned char *)Blo;
    a.sBk = d.sBk;
    a.sBn = d.sBn;
    a.sBb = d.sBb;
    a.C = (unsigned char *)d.C;
    a.Clo = (unsigned char *)d.Clo;
    if (a.Clo && (prec != CDS_PREC_BF16X3 || d.beta != 0.0))
        return cds_fail(ctx, CDS_EINVAL, "split GEMM output needs BF16X3 and beta 0");
    a.sCm = d.sCm;
    a.sCn = d.sCn;
    a.sCb = d.sCb;
    a.alpha = d.alpha;
    a.beta = d.beta;
    a.big = d.big;
    if (prec == CDS_PREC_FP64) return launch<CDS_PREC_FP64>(ctx, a);
    if (prec == CDS_PREC_FP32) return launch<CDS_PREC_FP32>(ctx, a);
    if (prec == CDS_PREC_BF16X3) return launch<CDS_PREC_BF16X3>(ctx, a);
    return cds_fail(ctx, CDS_EINVAL, "unknown precision %d", prec);
}

int cds_gemm(cds_ctx *ctx, int prec, const GemmDesc &d) { return cds_gemm_ex(ctx, prec, d, nullptr, nullptr); }
