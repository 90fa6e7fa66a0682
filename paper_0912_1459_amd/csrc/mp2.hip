// MP2 correlation energy from the transformed Cholesky blocks (Sec. II.A, Eq. (MP2)):
//   E = sum_{i,j occ; a,b virt} (2 (ai|bj) - (aj|bi)) (ai|bj) / (e_i + e_j - e_a - e_b),
//   (ai|bj) = sum_K B^K_ai B^K_bj  (Eq. (aomo)).
//
// The nocc x nocc block X_ab[i][j] = (ai|bj) holds both exchange partners, and
// X_ba = X_ab^T gives the same sum, so only blocks b >= a are formed:
//   E = sum_a S_aa + 2 sum_{a<b} S_ab,
//   S_ab = sum_{i<=j} R_ij / (e_i + e_j - e_a - e_b),
//   R_ij = 2 (x^2 + x'^2 - x x')  (i < j),  R_ii = x^2,   x = X_ab[i][j], x' = X_ab[j][i].
// Virtuals are processed in chunks [a0, a1): one MFMA GEMM
//   G[(a - a0) nocc + i][(b - a0) nocc + j] = sum_K Bvo[a][i][K] Bvo[b][j][K],  b >= a0,
// then one block per (a, b >= a) reduces its X_ab (32 x 32 tile pairs through LDS, as in
// the self-energy epilogue) to S_ab; a last one-block kernel sums the S_ab in fixed order.
#include "cds_internal.h"

int cds_gemm_ex(cds_ctx *ctx, int prec, const GemmDesc &d, const void *Alo, const void *Blo);

namespace {

constexpr int MP_NT = 256;
constexpr int MP_RED_NT = 1024;
constexpr size_t MP_CHUNK_BYTES = (size_t)4 << 30;   // integral chunk cap

template <typename GT>
__device__ __forceinline__ double ldg(const GT *p, int64_t i) { return (double)p[i]; }

template <typename GT>
__global__ __launch_bounds__(MP_NT) void mp2_block_kernel(const GT *__restrict__ G, int64_t ldg_, int nocc,
                                                          int a0, const double *__restrict__ eps, int nvirt,
                                                          double *__restrict__ S)
{
    __shared__ double eo[1024];
    __shared__ double t1[32][33], t2[32][33];
    __shared__ double sh[MP_NT / 64];
    const int al = blockIdx.x, bo = blockIdx.y;
    const int a = a0 + al, b = a0 + bo;
    if (b < a) return;                                     // the (b, a) block gives the same sum
    for (int i = threadIdx.x; i < nocc; i += MP_NT) eo[i] = eps[i];
    const double eab = eps[nocc + a] + eps[nocc + b];
    const int64_t base = (int64_t)al * nocc * ldg_ + (int64_t)bo * nocc;   // + i*ldg + j
    double acc = 0.0;
    const int nb = (nocc + 31) / 32;
    for (int IB = 0; IB < nb; ++IB)
        for (int JB = IB; JB < nb; ++JB) {
            // both tiles: every load in flight before the LDS stores
            constexpr int QN = 1024 / MP_NT;
            double v1[QN], v2[QN];
#pragma unroll
            for (int u = 0; u < QN; ++u) {
                const int q = threadIdx.x + MP_NT * u;
                const int r = q >> 5, c = q & 31;
                const int i1 = IB * 32 + r, j1 = JB * 32 + c;   // t1[r][c] = X[i1][j1]
                const int i2 = JB * 32 + r, j2 = IB * 32 + c;   // t2[r][c] = X[i2][j2]
                v1[u] = (i1 < nocc && j1 < nocc) ? ldg(G, base + (int64_t)i1 * ldg_ + j1) : 0.0;
                v2[u] = (i2 < nocc && j2 < nocc) ? ldg(G, base + (int64_t)i2 * ldg_ + j2) : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < QN; ++u) {
                const int q = threadIdx.x + MP_NT * u;
                t1[q >> 5][q & 31] = v1[u];
                t2[q >> 5][q & 31] = v2[u];
            }
            __syncthreads();
            for (int q = threadIdx.x; q < 1024; q += MP_NT) {
                const int r = q >> 5, c = q & 31;
                const int i = IB * 32 + r, j = JB * 32 + c;
                if (i >= nocc || j >= nocc || (IB == JB && r > c)) continue;
                const double x = t1[r][c], xt = t2[c][r];
                const double R = (i == j) ? x * x : 2.0 * (x * x + xt * xt - x * xt);
                acc += R / (eo[i] + eo[j] - eab);
            }
        }
    // block sum in fixed order
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < MP_NT / 64; ++k) s += sh[k];
        S[(int64_t)a * nvirt + b] = s;
    }
}

// E = sum_a S_aa + 2 sum_{a<b} S_ab, fixed summation order
__global__ __launch_bounds__(MP_RED_NT) void mp2_sum_kernel(const double *__restrict__ S, int nvirt,
                                                            double *__restrict__ out)
{
    __shared__ double sh[MP_RED_NT / 64];
    // each thread's terms in a fixed order (column offset b - a, then a), eight rows a of loads in
    // flight at a time
    constexpr int AU = 8;
    double acc = 0.0;
    for (int b0 = threadIdx.x; b0 < nvirt; b0 += MP_RED_NT) {     // b = a + b0: one column offset per pass
        for (int a0 = 0; a0 < nvirt; a0 += AU) {
            double v[AU];
#pragma unroll
            for (int u = 0; u < AU; ++u) {
                const int a = a0 + u, b = a + b0;
                v[u] = (a < nvirt && b < nvirt) ? S[(int64_t)a * nvirt + b] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < AU; ++u) {
                const int a = a0 + u, b = a + b0;
                if (a < nvirt && b < nvirt) acc += (b == a ? 1.0 : 2.0) * v[u];
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < MP_RED_NT / 64; ++k) s += sh[k];
        *out = s;
    }
}

}  // namespace

extern "C" int cds_mp2(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo, int32_t nocc,
                       const void *Bvo, const double *eps, double *h_energy)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, prec == CDS_PREC_FP64 || prec == CDS_PREC_FP32 || prec == CDS_PREC_BF16X3,
                "unknown precision %d", prec);
    CDS_REQUIRE(ctx, nmo >= 2 && nocc >= 1 && nocc < nmo, "need 1 <= nocc < nmo");
    CDS_REQUIRE(ctx, nocc <= 1024, "nocc must be <= 1024");
    CDS_REQUIRE(ctx, nvec >= 1 && ldk >= nvec && ldk % 64 == 0, "need 1 <= nvec <= ldk, ldk a multiple of 64");
    CDS_REQUIRE(ctx, Bvo && eps && h_energy, "NULL pointer");
    const int nvirt = nmo - nocc;
    CDS_REQUIRE(ctx, nvirt <= 65535, "nvirt must be <= 65535");
    const int64_t nvo = (int64_t)nvirt * nocc;
    const size_t es = prec == CDS_PREC_FP64 ? 8 : (prec == CDS_PREC_FP32 ? 4 : 2);
    const size_t gs = prec == CDS_PREC_FP64 ? 8 : 4;       // integral storage

    // chunks of virtuals: about 8 for the b >= a saving, more if the integrals would not fit
    int na = (nvirt + 7) / 8;
    while (na > 1 && (size_t)na * nocc * nvo * gs > MP_CHUNK_BYTES) na = (na + 1) / 2;
    CDS_REQUIRE(ctx, (size_t)na * nocc * nvo * gs <= MP_CHUNK_BYTES, "one virtual's integrals exceed the chunk cap");
    void *Gw, *Sw;
    CDS_CALL(cds_ws(ctx, WS_MP_G, (size_t)na * nocc * nvo * gs, &Gw));
    CDS_CALL(cds_ws(ctx, WS_MP_S, ((size_t)nvirt * nvirt + 1) * 8, &Sw));
    double *S = (double *)Sw;
    double *dout = S + (size_t)nvirt * nvirt;

    CdsTimer t;
    CDS_CALL(cds_timer_start(ctx, &t));
    for (int a0 = 0; a0 < nvirt; a0 += na) {
        const int n_a = std::min(na, nvirt - a0);
        const int64_t ncols = (int64_t)(nvirt - a0) * nocc;
        GemmDesc d = {};
        d.M = (int64_t)n_a * nocc;
        d.N = ncols;
        d.K = cds_ceil_div(nvec, 64) * 64;      // entries K in [nvec, this) are zero
        d.batch = 1;
        d.A = (const unsigned char *)Bvo + (size_t)a0 * nocc * ldk * es;
        d.sAm = ldk;
        d.sAk = 1;
        d.B = d.A;
        d.sBn = ldk;
        d.sBk = 1;
        d.C = Gw;
        d.sCm = ncols;
        d.sCn = 1;
        d.alpha = 1.0;
        d.beta = 0.0;
        const void *lo = nullptr;
        if (prec == CDS_PREC_BF16X3) lo = (const __bf16 *)Bvo + nvo * ldk + (int64_t)a0 * nocc * ldk;
        CDS_CALL(cds_gemm_ex(ctx, prec, d, lo, lo));
        ctx->stats.flops_mp2 += 2.0 * (double)nvec * (double)d.M * (double)d.N;
        const dim3 grid((unsigned)n_a, (unsigned)(nvirt - a0));
        if (prec == CDS_PREC_FP64)
            hipLaunchKernelGGL(mp2_block_kernel<double>, grid, dim3(MP_NT), 0, ctx->stream, (const double *)Gw,
                               ncols, nocc, a0, eps, nvirt, S);
        else
            hipLaunchKernelGGL(mp2_block_kernel<float>, grid, dim3(MP_NT), 0, ctx->stream, (const float *)Gw,
                               ncols, nocc, a0, eps, nvirt, S);
        CDS_LAUNCHED(ctx);
    }
    hipLaunchKernelGGL(mp2_sum_kernel, dim3(1), dim3(MP_RED_NT), 0, ctx->stream, (const double *)S, nvirt, dout);
    CDS_LAUNCHED(ctx);
    CDS_CALL(cds_timer_stop(ctx, &t, &ctx->stats.t_mp2_ms));
    void *hp;
    CDS_CALL(cds_pinned(ctx, 64, &hp));
    CDS_HIP(ctx, hipMemcpyAsync(hp, dout, 8, hipMemcpyDeviceToHost, ctx->stream));
    CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *h_energy = *(double *)hp;
    CDS_CALL(cds_timers_flush(ctx));
    return CDS_OK;
}
