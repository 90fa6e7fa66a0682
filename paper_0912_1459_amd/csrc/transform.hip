// AO->MO transform of the Cholesky vectors, Eq. (transformation) of the paper:
//   B^K_pq = sum_{mu,nu} C_mu,p L^K_mu,nu C_nu,q
// for the blocks the self-energy reads: B^K[sel, :] and B^K[virt, occ].
//
// Per batch of vectors K (all on the GPU, batched over K):
//   1. unpack   packed L^K -> dense symmetric Lu[K][mu][nu] (k padded to Np)
//   2. GEMM     T[K][x][mu] = sum_nu CX[x][nu] Lu[K][mu][nu]      x = occ, then sel
//   3. GEMM     Bk[K][a][i] = sum_mu Ct[nocc+a][mu] T[K][i][mu]    (virt x occ)
//      GEMM     Bk[K][s][r] = sum_mu T[K][nocc+s][mu] Ct[r][mu]    (sel x all)
//   4. transpose Bk[K][row] -> B[row][K] (K contiguous), converting to the
//      output format (double, float, or bf16 hi/lo planes).
// Working precision of steps 1-3: FP64 for CDS_PREC_FP64, FP32 for FP32, and
// split bf16 (3-term products, FP32 accumulation) for BF16X3.
#include "cds_internal.h"

#include <type_traits>

int cds_gemm_ex(cds_ctx *ctx, int prec, const GemmDesc &d, const void *Alo, const void *Blo);

namespace {

constexpr int KBATCH_MIN = 64;          // vectors per transform batch: at least this many,
constexpr int KBATCH_WG = 2048;         // enough that the smallest GEMM launches this many tiles,
constexpr size_t KBATCH_BYTES = 1ull << 30;   // and the unpacked batch stays below this size

__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)x;                       // round to nearest even
    lo = (__bf16)(x - (float)hi);
}

// store element e (double) at index idx of a working buffer of format prec
// (FP64: double; FP32: float; BF16X3: hi plane at base, lo plane at base + plane)
__device__ __forceinline__ void put(void *base, int prec, int64_t idx, int64_t plane, double v)
{
    if (prec == CDS_PREC_FP64) {
        ((double *)base)[idx] = v;
    } else if (prec == CDS_PREC_FP32) {
        ((float *)base)[idx] = (float)v;
    } else {
        __bf16 hi, lo;
        split_bf16((float)v, hi, lo);
        ((__bf16 *)base)[idx] = hi;
        ((__bf16 *)base)[plane + idx] = lo;
    }
}


// four consecutive elements idx .. idx+3 (16-byte aligned for FP64 / 8-byte for the others)
__device__ __forceinline__ void put4(void *base, int prec, int64_t idx, int64_t plane, const double (&v)[4])
{
    if (prec == CDS_PREC_FP64) {
        double4 x = {v[0], v[1], v[2], v[3]};
        *reinterpret_cast<double2 *>((double *)base + idx) = double2{x.x, x.y};
        *reinterpret_cast<double2 *>((double *)base + idx + 2) = double2{x.z, x.w};
    } else if (prec == CDS_PREC_FP32) {
        *reinterpret_cast<float4 *>((float *)base + idx) = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    } else {
        __bf16 hi[4], lo[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) split_bf16((float)v[e], hi[e], lo[e]);
        *reinterpret_cast<uint2 *>((__bf16 *)base + idx) = *reinterpret_cast<const uint2 *>(hi);
        *reinterpret_cast<uint2 *>((__bf16 *)base + plane + idx) = *reinterpret_cast<const uint2 *>(lo);
    }
}

// Lu[kb][mu][nu] = L^{k0+kb}_{mu nu} (0 for nu >= nbf), by 32 x 32 blocks: workgroup
// (kb, block pair bm >= bn) reads the block rows mu in bm, nu in bn of the lower triangle
// (contiguous in nu), writes it in place and, off the diagonal, transposed through LDS
__global__ __launch_bounds__(256) void unpack_blocks_kernel(const double *__restrict__ L, int64_t ldl, int64_t k0,
                                                            int nbf, int np_, void *out, int prec, int64_t plane)
{
    __shared__ double tile[32][33];
    const int kb = blockIdx.y;
    int bp = blockIdx.x, bm = 0;                  // block pair index -> (bm, bn), bn <= bm
    while (bp > bm) bp -= ++bm;
    const int bn = bp;
    const int r = threadIdx.x >> 3, c0 = (threadIdx.x & 7) * 4;
    const double *Lk = L + (k0 + kb) * ldl;
    const int64_t base = (int64_t)kb * nbf * np_;
    const int mu = bm * 32 + r;
    double v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int nu = bn * 32 + c0 + e;
        v[e] = 0.0;
        if (mu < nbf && nu < nbf) {
            const int a = mu < nu ? mu : nu, b = mu < nu ? nu : mu;
            v[e] = Lk[(int64_t)b * (b + 1) / 2 + a];
        }
        tile[r][c0 + e] = v[e];
    }
    if (mu < nbf) put4(out, prec, base + (int64_t)mu * np_ + bn * 32 + c0, plane, v);
    if (bm == bn) return;                         // the diagonal block holds both triangles
    __syncthreads();
    const int nu_row = bn * 32 + r;               // transposed: row nu of block bn, columns mu of bm
    if (nu_row >= nbf) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = tile[c0 + e][r];
    put4(out, prec, base + (int64_t)nu_row * np_ + bm * 32 + c0, plane, v);
}

// Ct[p][mu] = C[mu][p]; CX rows: occupied 0..nocc-1 then sel[s]; k padded to np_
__global__ void coef_kernel(const double *__restrict__ C, int nbf, int nmo, int nocc, int nsel,
                            const int32_t *__restrict__ sel, int np_, void *Ct, void *CX, int prec,
                            int64_t planeCt, int64_t planeCX)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nrow = nmo + nocc + nsel;
    if (t >= nrow * np_) return;
    int row = (int)(t / np_), mu = (int)(t - (int64_t)row * np_);
    int p;
    void *dst;
    int64_t idx, plane;
    if (row < nmo) {
        p = row;
        dst = Ct;
        idx = (int64_t)row * np_ + mu;
        plane = planeCt;
    } else {
        int x = row - nmo;
        p = x < nocc ? x : sel[x - nocc];
        dst = CX;
        idx = (int64_t)x * np_ + mu;
        plane = planeCX;
    }
    double v = mu < nbf ? C[(int64_t)mu * nmo + p] : 0.0;
    put(dst, prec, idx, plane, v);
}

// zero the byte columns [c0, c1) of nrows rows of pitch `pitch` bytes (2-byte units)
__global__ void zero_cols_kernel(unsigned char *base, int64_t nrows, int64_t pitch, int c0, int c1)
{
    const int per = (c1 - c0) / 2;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * per) return;
    const int64_t r = t / per;
    *reinterpret_cast<uint16_t *>(base + r * pitch + c0 + 2 * (t - r * per)) = 0;
}


// Bk[kb][row] (working type W) -> out[row*ldk + k0 + kb] in the output format.
// rows [0, nvo) go to Bvo, rows [nvo, nvo + nselr) to Bsel.
template <typename W>
__global__ void transpose_out_kernel(const W *__restrict__ Bk, int64_t nrows, int nkb, int64_t k0,
                                     int64_t nvo, void *Bvo, void *Bsel, int64_t ldk, int prec,
                                     int64_t plane_vo, int64_t plane_sel)
{
    __shared__ double tile[32][33];
    int64_t r0 = (int64_t)blockIdx.x * 32;
    int kb0 = blockIdx.y * 32;
    int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
    for (int j = ty; j < 32; j += 8) {
        int kb = kb0 + j;
        int64_t r = r0 + tx;
        tile[j][tx] = (kb < nkb && r < nrows) ? (double)Bk[(int64_t)kb * nrows + r] : 0.0;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        int64_t r = r0 + j;
        int kb = kb0 + tx;
        if (r >= nrows || kb >= nkb) continue;
        double v = tile[tx][j];
        if (r < nvo)
            put(Bvo, prec, r * ldk + k0 + kb, plane_vo, v);
        else
            put(Bsel, prec, (r - nvo) * ldk + k0 + kb, plane_sel, v);
    }
}

__global__ void zero_pad_kernel(int64_t nrows, int64_t ldk, int64_t nvec, void *B, int prec, int64_t plane)
{
    int64_t npad = ldk - nvec;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * npad) return;
    int64_t r = t / npad, c = nvec + (t - r * npad);
    put(B, prec, r * ldk + c, plane, 0.0);
}

size_t wsize(int prec) { return prec == CDS_PREC_FP64 ? 8 : (prec == CDS_PREC_FP32 ? 4 : 4); }

}  // namespace

extern "C" int cds_transform(cds_ctx *ctx, int32_t prec, int32_t nbf, int64_t nvec, const double *L,
                             int64_t ldl, const double *C, int32_t nmo, int32_t nocc, int32_t nsel,
                             const int32_t *h_sel, int64_t ldk, void *Bsel, void *Bvo)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, prec == CDS_PREC_FP64 || prec == CDS_PREC_FP32 || prec == CDS_PREC_BF16X3,
                "unknown precision %d", prec);
    CDS_REQUIRE(ctx, nbf >= 1 && nmo >= 1 && nmo <= nbf, "need 1 <= nmo <= nbf");
    CDS_REQUIRE(ctx, nocc >= 1 && nocc < nmo, "need 1 <= nocc < nmo");
    CDS_REQUIRE(ctx, nsel >= 1 && nsel <= nmo && h_sel, "need 1 <= nsel <= nmo and h_sel");
    CDS_REQUIRE(ctx, nvec >= 1 && ldk >= nvec, "need nvec >= 1 and ldk >= nvec");
    CDS_REQUIRE(ctx, ldl >= cds_npairs(nbf), "ldl < npairs");
    CDS_REQUIRE(ctx, L && C && Bsel && Bvo, "NULL pointer");
    for (int s = 0; s < nsel; ++s)
        CDS_REQUIRE(ctx, h_sel[s] >= 0 && h_sel[s] < nmo, "h_sel[%d]=%d out of range", s, h_sel[s]);

    CdsTimer tm;
    CDS_CALL(cds_timer_start(ctx, &tm));
    const int nvirt = nmo - nocc;
    const int nx = nocc + nsel;
    const int np_ = (int)(cds_ceil_div(nbf, 64) * 64);
    const int64_t nvo = (int64_t)nvirt * nocc, nselr = (int64_t)nsel * nmo;
    const int64_t nrows = nvo + nselr;
    // working precision of the GEMMs; the output is rounded to `prec` in the last pass
    const int wp = ctx->transform_fp64 ? CDS_PREC_FP64 : prec;
    const size_t es = wsize(wp);
    // batch: the virtual-occupied GEMM has one 128 x 128 tile group per vector and would
    // leave most of the chip idle with small batches
    const int64_t tiles_vo = cds_ceil_div(nvirt, 128) * cds_ceil_div(nocc, 128);
    int64_t kb_want = std::max<int64_t>(KBATCH_MIN, cds_ceil_div(KBATCH_WG, tiles_vo));
    kb_want = std::min<int64_t>(kb_want, std::max<int64_t>(1, (int64_t)(KBATCH_BYTES / ((size_t)nbf * np_ * es))));
    const int kbatch = (int)std::min<int64_t>(kb_want, nvec);

    // workspace: Ct + CX (+ sel list), Lu batch, T batch (+ split copy), Bk batch
    void *wcx, *wlu, *wt, *wb;
    const int64_t nCt = (int64_t)nmo * np_, nCX = (int64_t)nx * np_;
    CDS_CALL(cds_ws(ctx, WS_TR_CX, (size_t)(nCt + nCX) * es + 256 + nsel * 4, &wcx));
    const int64_t nLu = (int64_t)kbatch * nbf * np_;
    CDS_CALL(cds_ws(ctx, WS_TR_UNPACK, (size_t)nLu * es, &wlu));
    const int64_t nT = (int64_t)kbatch * nx * np_;
    CDS_CALL(cds_ws(ctx, WS_TR_T, (size_t)nT * es * (wp == CDS_PREC_BF16X3 ? 2 : 1), &wt));
    CDS_CALL(cds_ws(ctx, WS_TR_B, (size_t)kbatch * nrows * (wp == CDS_PREC_FP64 ? 8 : 4), &wb));

    unsigned char *Ct = (unsigned char *)wcx;
    unsigned char *CX = Ct + nCt * es;
    int32_t *dsel = (int32_t *)(CX + ((nCX * es + 255) / 256) * 256);
    CDS_HIP(ctx, hipMemcpyAsync(dsel, h_sel, (size_t)nsel * 4, hipMemcpyHostToDevice, ctx->stream));
    // planes for bf16: lo plane follows the hi plane of the same buffer region
    const int64_t planeCt = nCt, planeCX = nCX;
    {
        int64_t n = (int64_t)(nmo + nx) * np_;
        hipLaunchKernelGGL(coef_kernel, dim3((unsigned)cds_ceil_div(n, 256)), dim3(256), 0, ctx->stream,
                           C, nbf, nmo, nocc, nsel, dsel, np_, (void *)Ct, (void *)CX, wp, planeCt,
                           planeCX);
        CDS_LAUNCHED(ctx);
    }
    // for bf16, hi+lo planes of Ct/CX take 2 x 2 bytes = es (4) per element: place lo planes
    // right after each hi plane inside the same byte range (hi plane uses nC*2 bytes).
    // T: working float output, and (bf16) a split copy after it
    float *Tf = (float *)wt;
    __bf16 *Ts = (__bf16 *)((unsigned char *)wt + (size_t)nT * 4);
    // the first GEMM writes columns < nbf of T; the K padding [nbf, np_) must read as 0
    if (np_ > nbf) {
        const size_t tes0 = (wp == CDS_PREC_FP64) ? 8 : (wp == CDS_PREC_FP32 ? 4 : 2);
        unsigned char *tb = (wp == CDS_PREC_BF16X3) ? (unsigned char *)Ts : (unsigned char *)wt;
        const int64_t trows = (int64_t)kbatch * nx * (wp == CDS_PREC_BF16X3 ? 2 : 1);   // both planes
        const int64_t nz = trows * (int64_t)((np_ - nbf) * tes0 / 2);
        hipLaunchKernelGGL(zero_cols_kernel, dim3((unsigned)cds_ceil_div(nz, 256)), dim3(256), 0, ctx->stream, tb,
                           trows, (int64_t)np_ * (int64_t)tes0, (int)(nbf * tes0), (int)(np_ * tes0));
        CDS_LAUNCHED(ctx);
    }

    // zero padding of B beyond nvec
    if (ldk > nvec) {
        int64_t n1 = nvo * (ldk - nvec), n2 = nselr * (ldk - nvec);
        hipLaunchKernelGGL(zero_pad_kernel, dim3((unsigned)cds_ceil_div(n1, 256)), dim3(256), 0,
                           ctx->stream, nvo, ldk, nvec, Bvo, prec, nvo * ldk);
        hipLaunchKernelGGL(zero_pad_kernel, dim3((unsigned)cds_ceil_div(n2, 256)), dim3(256), 0,
                           ctx->stream, nselr, ldk, nvec, Bsel, prec, nselr * ldk);
        CDS_LAUNCHED(ctx);
    }

    const int gprec = wp;     // GEMM precision
    for (int64_t k0 = 0; k0 < nvec; k0 += kbatch) {
        const int nkb = (int)std::min<int64_t>(kbatch, nvec - k0);
        {
            const int nb = np_ / 32;
            hipLaunchKernelGGL(unpack_blocks_kernel, dim3((unsigned)(nb * (nb + 1) / 2), (unsigned)nkb), dim3(256), 0,
                               ctx->stream, L, ldl, k0, nbf, np_, wlu, wp, (int64_t)nkb * nbf * np_);
            CDS_LAUNCHED(ctx);
        }
        const int64_t planeLu = (int64_t)nkb * nbf * np_;
        // T[kb][x][mu] = sum_nu CX[x][nu] Lu[kb][mu][nu]
        GemmDesc g1 = {};
        g1.M = nx; g1.N = nbf; g1.K = np_; g1.batch = nkb;
        g1.A = CX; g1.sAm = np_; g1.sAk = 1; g1.sAb = 0;
        g1.B = wlu; g1.sBn = np_; g1.sBk = 1; g1.sBb = (int64_t)nbf * np_;
        void *Tout = (wp == CDS_PREC_FP64) ? wt : (void *)Tf;
        g1.C = Tout; g1.sCm = np_; g1.sCn = 1; g1.sCb = (int64_t)nx * np_;
        g1.alpha = 1.0; g1.beta = 0.0;
        if (wp == CDS_PREC_BF16X3) {
            // T straight into its two bf16 planes (the split of the FP32 result)
            g1.C = Ts;
            g1.Clo = Ts + (int64_t)nkb * nx * np_;
            CDS_CALL(cds_gemm_ex(ctx, gprec, g1, (const __bf16 *)CX + planeCX, (const __bf16 *)wlu + planeLu));
        } else {
            CDS_CALL(cds_gemm_ex(ctx, gprec, g1, nullptr, nullptr));
        }
        const void *Tin = (wp == CDS_PREC_BF16X3) ? (const void *)Ts : (const void *)Tout;
        const int64_t planeT = (int64_t)nkb * nx * np_;
        const size_t tes = (wp == CDS_PREC_FP64) ? 8 : (wp == CDS_PREC_FP32 ? 4 : 2);
        const size_t ces = tes;
        // Bk[kb][a][i] = sum_mu Ct[nocc+a][mu] T[kb][i][mu]
        GemmDesc g2 = {};
        g2.M = nvirt; g2.N = nocc; g2.K = np_; g2.batch = nkb;
        g2.A = (const unsigned char *)Ct + (size_t)nocc * np_ * ces; g2.sAm = np_; g2.sAk = 1; g2.sAb = 0;
        g2.B = Tin; g2.sBn = np_; g2.sBk = 1; g2.sBb = (int64_t)nx * np_;
        g2.C = wb; g2.sCm = nocc; g2.sCn = 1; g2.sCb = nrows;
        g2.alpha = 1.0; g2.beta = 0.0;
        // Bk[kb][nvo + s*nmo + r] = sum_mu T[kb][nocc+s][mu] Ct[r][mu]
        GemmDesc g3 = {};
        g3.M = nsel; g3.N = nmo; g3.K = np_; g3.batch = nkb;
        g3.A = (const unsigned char *)Tin + (size_t)nocc * np_ * tes; g3.sAm = np_; g3.sAk = 1;
        g3.sAb = (int64_t)nx * np_;
        g3.B = Ct; g3.sBn = np_; g3.sBk = 1; g3.sBb = 0;
        g3.C = (unsigned char *)wb + (size_t)nvo * (wp == CDS_PREC_FP64 ? 8 : 4);
        g3.sCm = nmo; g3.sCn = 1; g3.sCb = nrows;
        g3.alpha = 1.0; g3.beta = 0.0;
        if (wp == CDS_PREC_BF16X3) {
            CDS_CALL(cds_gemm_ex(ctx, gprec, g2, (const __bf16 *)Ct + planeCt + (int64_t)nocc * np_,
                                 Ts + planeT));
            CDS_CALL(cds_gemm_ex(ctx, gprec, g3, Ts + planeT + (int64_t)nocc * np_,
                                 (const __bf16 *)Ct + planeCt));
        } else {
            CDS_CALL(cds_gemm_ex(ctx, gprec, g2, nullptr, nullptr));
            CDS_CALL(cds_gemm_ex(ctx, gprec, g3, nullptr, nullptr));
        }
        dim3 tg((unsigned)cds_ceil_div(nrows, 32), (unsigned)cds_ceil_div(nkb, 32));
        if (wp == CDS_PREC_FP64)
            hipLaunchKernelGGL(transpose_out_kernel<double>, tg, dim3(256), 0, ctx->stream,
                               (const double *)wb, nrows, nkb, k0, nvo, Bvo, Bsel, ldk, prec, nvo * ldk,
                               nselr * ldk);
        else
            hipLaunchKernelGGL(transpose_out_kernel<float>, tg, dim3(256), 0, ctx->stream,
                               (const float *)wb, nrows, nkb, k0, nvo, Bvo, Bsel, ldk, prec, nvo * ldk,
                               nselr * ldk);
        CDS_LAUNCHED(ctx);
    }
    CDS_CALL(cds_timer_stop(ctx, &tm, &ctx->stats.t_transform_ms));
    return CDS_OK;
}

extern "C" int cds_set_transform_fp64(cds_ctx *ctx, int32_t on)
{
    if (!ctx) return CDS_EINVAL;
    if (on != 0 && on != 1) return cds_fail(ctx, CDS_EINVAL, "on must be 0 or 1");
    ctx->transform_fp64 = on;
    return CDS_OK;
}
