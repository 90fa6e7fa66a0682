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
    unsigned char *C;
    int64_t sCm, sCn, sCb;
    double alpha, beta;
    int fastA, fastB;              // K-contiguous, 16-byte aligned rows, K % KB == 0
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

    // epilogue: C = alpha * acc + beta * C
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
                O *dst = C + m * a.sCm + n * a.sCn;
                double v = a.alpha * (double)acc[i][j][e];
                if (a.beta != 0.0) v += a.beta * (double)(*dst);
                *dst = (O)v;
            }
        }
}

bool fast_ok(const void *p, int64_t srow, int64_t sk, int64_t K, int kb, size_t esz)
{
    return sk == 1 && K % kb == 0 && cds_aligned(p, 16) && (srow * (int64_t)esz) % 16 == 0;
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
    size_t lds = (size_t)2 * Tr<PREC>::PLANES * BM * PITCH;
    hipLaunchKernelGGL(gemm_kernel<PREC>, dim3((unsigned)gx, (unsigned)gy, (unsigned)a.batch), dim3(NT),
                       lds, ctx->stream, a);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}

}  // namespace

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
    a.sCm = d.sCm;
    a.sCn = d.sCn;
    a.sCb = d.sCb;
    a.alpha = d.alpha;
    a.beta = d.beta;
    if (prec == CDS_PREC_FP64) return launch<CDS_PREC_FP64>(ctx, a);
    if (prec == CDS_PREC_FP32) return launch<CDS_PREC_FP32>(ctx, a);
    if (prec == CDS_PREC_BF16X3) return launch<CDS_PREC_BF16X3>(ctx, a);
    return cds_fail(ctx, CDS_EINVAL, "unknown precision %d", prec);
}

int cds_gemm(cds_ctx *ctx, int prec, const GemmDesc &d) { return cds_gemm_ex(ctx, prec, d, nullptr, nullptr); }
