// Adjoints of the quasi-particle solve and of the AO->MO transform.
//
// The converged energy w* solves F(w, theta) = e_q + Sigma_qq(w; theta) - w = 0
// (Eq. (qpapp) of the paper); implicit differentiation gives
//   dw*/dtheta = P dF/dtheta,   P = 1 / (1 - Sigma'(w*))   (pole strength, Eq. (ps)).
// With g = (q r|a j) = G[s][r][a*nocc+j] (Eq. (aomo)) the self-energy Eq. (SE)
// depends on each integral through its own term and its exchange partner:
//   dSigma/dx_{a;ij} = (4 x_{a;ij} - 2 x_{a;ji}) / d_{a;ij},  same for y.
// Since G = Bsel Bvo^T:
//   Bsel_bar[s] = W[s] Bvo            (W = omega_bar P dSigma/dG)
//   Bvo_bar     = sum_s W[s]^T Bsel[s]
// and the energies enter through the denominators and e_q itself.
// Transform adjoint: B^K = C^T L^K C gives C_bar = sum_K L^K C (Bbar^K + Bbar^K^T).
#include "cds_internal.h"

#include <cmath>
#include <vector>

int cds_gemm_ex(cds_ctx *ctx, int prec, const GemmDesc &d, const void *Alo, const void *Blo);
int cds_sigma_eval_internal(cds_ctx *ctx, int prec, int64_t nvec, int64_t ldk, int nmo, int nocc,
                            int nsel, const void *Bsel, const void *Bvo, const double *eps,
                            const double *h_omega, int T, double *h_out);
int cds_contract_internal(cds_ctx *ctx, int prec, int64_t nvec, int64_t ldk, int nmo, int nocc,
                          int nsel, const void *Bsel, const void *Bvo, int s0, int nsc, void *G);
int cds_grad_epilogue_internal(cds_ctx *ctx, int prec, int nmo, int nocc, int nsc, const void *G,
                               const double *eps, const double *d_omega, const double *d_gscale,
                               void *W, double *epsA, double *epsB);
int cds_sigma_from_g_internal(cds_ctx *ctx, int prec, int nmo, int nocc, int nsc, const void *G,
                              const double *eps, const double *d_omega, double *d_out);

namespace {

// bf16 hi/lo planes -> float
__global__ void planes_to_float_kernel(const __bf16 *__restrict__ b, int64_t n, float *__restrict__ out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = (float)b[t] + (float)b[n + t];
}

template <typename T>
__global__ void zero_cols_kernel(T *__restrict__ B, int64_t nrows, int64_t ldk, int64_t c0)
{
    int64_t npad = ldk - c0;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * npad) return;
    int64_t r = t / npad;
    B[r * ldk + c0 + (t - r * npad)] = (T)0;
}

// eps_bar[r] = sum over targets and blocks of the energy partials, + P*omega_bar on e_q
// eps_bar[r]: one workgroup per orbital r; the threads take the (target, virtual) partials in a
// fixed stride, four loads in flight at a time, and the workgroup sums them in a fixed order
__global__ __launch_bounds__(256) void eps_bar_kernel(const double *__restrict__ epsA, const double *__restrict__ epsB,
                                                      int nsel, int nocc, int nvirt, const int32_t *__restrict__ sel,
                                                      const double *__restrict__ gscale, double *__restrict__ out)
{
    __shared__ double sh[4];
    const int r = blockIdx.x;
    const int64_t per = (int64_t)nvirt * (nocc + 1);
    double acc = 0.0;
    if (r < nocc) {
        const int64_t n = (int64_t)nsel * nvirt;                 // (target, virtual) pairs
        constexpr int U = 4;
        for (int64_t q0 = threadIdx.x; q0 < n; q0 += (int64_t)U * 256) {
            double va[U], vb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = q0 + (int64_t)u * 256 < n ? q0 + (int64_t)u * 256 : n - 1;
                const int64_t s = q / nvirt, a = q - s * nvirt;
                const int64_t off = s * per + a * (nocc + 1) + r;
                va[u] = epsA[off];
                vb[u] = epsB[off];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (q0 + (int64_t)u * 256 < n) acc += va[u] + vb[u];
        }
    } else {
        for (int s = threadIdx.x; s < nsel; s += 256) {
            const int64_t off = (int64_t)s * per + (int64_t)(r - nocc) * (nocc + 1) + nocc;
            acc += epsA[off] + epsB[off];
        }
    }
    for (int s = threadIdx.x; s < nsel; s += 256)
        if (sel[s] == r) acc += gscale[s];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[r] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// S[kb][p][q] = Bbar^K[p][q] + Bbar^K[q][p] (FP64), Bbar scattered from the sel and vo blocks
template <typename BT>
__global__ void sym_bar_kernel(const BT *__restrict__ bsel, const BT *__restrict__ bvo, int64_t ldk, int64_t k0,
                               int nkb, int nmo, int nocc, int nsel, const int32_t *__restrict__ sel,
                               double *__restrict__ S)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = (int64_t)nmo * nmo;
    if (t >= per * nkb) return;
    int kb = (int)(t / per);
    int64_t rem = t - kb * per;
    int p = (int)(rem / nmo), q = (int)(rem - (int64_t)p * nmo);
    int64_t K = k0 + kb;
    double v = 0.0;
    for (int s = 0; s < nsel; ++s) {
        if (sel[s] == p) v += (double)bsel[((int64_t)s * nmo + q) * ldk + K];
        if (sel[s] == q) v += (double)bsel[((int64_t)s * nmo + p) * ldk + K];
    }
    if (p >= nocc && q < nocc) v += (double)bvo[((int64_t)(p - nocc) * nocc + q) * ldk + K];
    if (q >= nocc && p < nocc) v += (double)bvo[((int64_t)(q - nocc) * nocc + p) * ldk + K];
    S[t] = v;
}

// Lu[kb][mu][nu] (nu padded to np_) in FP64
// out[e] (+)= sum_{b < nb} part[b][e], b in increasing order
__global__ void sum_parts_kernel(const double *__restrict__ part, int nb, int64_t ne, int accumulate,
                                 double *__restrict__ out)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    // in vector order, eight loads in flight at a time
    constexpr int U = 8;
    double acc = accumulate ? out[e] : 0.0;
    for (int b0 = 0; b0 < nb; b0 += U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = b0 + u < nb ? part[(int64_t)(b0 + u) * ne + e] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (b0 + u < nb) acc += v[u];
    }
    out[e] = acc;
}

__global__ void unpack64_kernel(const double *__restrict__ L, int64_t ldl, int64_t k0, int nkb, int nbf,
                                int np_, double *__restrict__ out)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = (int64_t)nbf * np_;
    if (t >= per * nkb) return;
    int kb = (int)(t / per);
    int64_t rem = t - (int64_t)kb * per;
    int mu = (int)(rem / np_), nu = (int)(rem - (int64_t)mu * np_);
    double v = 0.0;
    if (nu < nbf) {
        int a = mu < nu ? mu : nu, b = mu < nu ? nu : mu;
        v = L[(k0 + kb) * ldl + (int64_t)b * (b + 1) / 2 + a];
    }
    out[t] = v;
}

}  // namespace

extern "C" int cds_qp_adjoint(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo,
                              int32_t nocc, int32_t nsel, const int32_t *h_sel, const void *Bsel,
                              const void *Bvo, const double *eps, const double *h_omega,
                              const double *h_omega_bar, void *Bsel_bar, void *Bvo_bar, double *eps_bar)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, prec == CDS_PREC_FP64 || prec == CDS_PREC_FP32 || prec == CDS_PREC_BF16X3,
                "unknown precision %d", prec);
    CDS_REQUIRE(ctx, nmo >= 2 && nocc >= 1 && nocc < nmo && nocc <= 1024, "bad nocc/nmo");
    CDS_REQUIRE(ctx, nsel >= 1 && h_sel && h_omega && h_omega_bar, "bad targets");
    CDS_REQUIRE(ctx, nvec >= 1 && ldk >= nvec, "need nvec >= 1, ldk >= nvec");
    CDS_REQUIRE(ctx, prec != CDS_PREC_BF16X3 || ldk % 64 == 0, "BF16X3 needs ldk % 64 == 0");
    CDS_REQUIRE(ctx, Bsel && Bvo && eps && Bsel_bar && Bvo_bar && eps_bar, "NULL pointer");
    for (int s = 0; s < nsel; ++s)
        CDS_REQUIRE(ctx, h_sel[s] >= 0 && h_sel[s] < nmo, "h_sel[%d] out of range", s);
    CdsTimer tall;
    CDS_CALL(cds_timer_start(ctx, &tall));
    const int nvirt = nmo - nocc;
    const int64_t nvo = (int64_t)nvirt * nocc, nselr = (int64_t)nsel * nmo;

    // the pole strengths at the converged energies come from each chunk's integrals (below)
    std::vector<double> out((size_t)nsel * 2), hscale(nsel);

    // working copies: float operands for BF16X3 (planes -> float)
    const int gprec = prec == CDS_PREC_FP64 ? CDS_PREC_FP64 : CDS_PREC_FP32;
    const size_t es = prec == CDS_PREC_FP64 ? 8 : 4;
    const void *Bs = Bsel, *Bv = Bvo;
    void *tmp;
    size_t nB = (size_t)(nselr + nvo) * ldk;
    size_t small = (size_t)nsel * 8 * 5 + (size_t)nsel * 4 + 256;
    size_t epsbytes = (size_t)2 * nsel * nvirt * (nocc + 1) * 8;
    CDS_CALL(cds_ws(ctx, WS_AD_TMP, (prec == CDS_PREC_BF16X3 ? nB * 4 : 0) + small + epsbytes, &tmp));
    unsigned char *tp = (unsigned char *)tmp;
    if (prec == CDS_PREC_BF16X3) {
        float *fs = (float *)tp, *fv = fs + nselr * ldk;
        hipLaunchKernelGGL(planes_to_float_kernel, dim3((unsigned)cds_ceil_div(nselr * ldk, 256)), dim3(256),
                           0, ctx->stream, (const __bf16 *)Bsel, nselr * ldk, fs);
        hipLaunchKernelGGL(planes_to_float_kernel, dim3((unsigned)cds_ceil_div(nvo * ldk, 256)), dim3(256), 0,
                           ctx->stream, (const __bf16 *)Bvo, nvo * ldk, fv);
        CDS_LAUNCHED(ctx);
        Bs = fs;
        Bv = fv;
        tp += nB * 4;
    }
    double *d_omega = (double *)tp;
    double *d_scale = d_omega + nsel;
    double *d_sig = d_scale + nsel;                    // [nsel][2]: Sigma, Sigma'
    int32_t *d_sel = (int32_t *)(d_sig + 2 * nsel);
    double *epsA = (double *)(tp + small);
    double *epsB = epsA + (size_t)nsel * nvirt * (nocc + 1);
    CDS_HIP(ctx, hipMemcpyAsync(d_omega, h_omega, (size_t)nsel * 8, hipMemcpyHostToDevice, ctx->stream));
    CDS_HIP(ctx, hipMemcpyAsync(d_sel, h_sel, (size_t)nsel * 4, hipMemcpyHostToDevice, ctx->stream));

    // chunks of targets: G, W and W^T each nsc * nmo * nvo, at most 12 GiB each (few, large
    // chunks: the product over nvo below has only nsc * nmo / 128 tile rows)
    size_t per = (size_t)nmo * nvo * es;
    int csz = (int)std::max<size_t>(1, ((size_t)12 << 30) / std::max<size_t>(per, 1));
    if (ctx->target_chunk > 0) csz = std::min(csz, ctx->target_chunk);
    csz = std::min(csz, (int)nsel);
    void *G, *W;
    CDS_CALL(cds_ws(ctx, WS_SG_G, (size_t)csz * per, &G));
    CDS_CALL(cds_ws(ctx, WS_AD_G, (size_t)csz * per, &W));
    // K-contiguous copies of the operands the two products read across K (the GEMM's fast path
    // loads rows along K): Bvo^T [nvec][nvo], then per chunk W^T [nvo][nsc*nmo] and the chunk's
    // Bsel^T [nvec][nsc*nmo]
    void *BvT, *WT, *BsT;
    CDS_CALL(cds_ws(ctx, WS_AD_T1, (size_t)nvec * nvo * es, &BvT));
    CDS_CALL(cds_ws(ctx, WS_AD_T2, (size_t)csz * per, &WT));
    CDS_CALL(cds_ws(ctx, WS_AD_T3, (size_t)nvec * csz * nmo * es, &BsT));
    CDS_CALL(cds_transpose(ctx, (int)es, nvo, nvec, Bv, ldk, BvT, nvo));
    for (int s0 = 0; s0 < nsel; s0 += csz) {
        const int nsc = std::min(csz, nsel - s0);
        CDS_CALL(cds_contract_internal(ctx, prec, nvec, ldk, nmo, nocc, nsel, Bsel, Bvo, s0, nsc, G));
        // P_s = 1 / (1 - Sigma'(w*_s)) from the same integrals, then the weights' scale
        CDS_CALL(cds_sigma_from_g_internal(ctx, prec, nmo, nocc, nsc, G, eps, d_omega + s0, d_sig + 2 * s0));
        CDS_HIP(ctx, hipMemcpyAsync(out.data() + 2 * s0, d_sig + 2 * s0, (size_t)nsc * 2 * 8, hipMemcpyDeviceToHost,
                                    ctx->stream));
        CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (int s = s0; s < s0 + nsc; ++s) hscale[s] = h_omega_bar[s] / (1.0 - out[2 * s + 1]);
        CDS_HIP(ctx, hipMemcpyAsync(d_scale + s0, hscale.data() + s0, (size_t)nsc * 8, hipMemcpyHostToDevice,
                                    ctx->stream));
        CDS_CALL(cds_grad_epilogue_internal(ctx, prec, nmo, nocc, nsc, G, eps, d_omega + s0, d_scale + s0, W,
                                            epsA + (size_t)s0 * nvirt * (nocc + 1),
                                            epsB + (size_t)s0 * nvirt * (nocc + 1)));
        // Bsel_bar[s0..] = W Bvo :  (nsc*nmo) x nvec, reduction over nvo
        GemmDesc d1 = {};
        d1.M = (int64_t)nsc * nmo; d1.N = nvec; d1.K = nvo; d1.batch = 1;
        d1.A = W; d1.sAm = nvo; d1.sAk = 1;
        d1.B = BvT; d1.sBk = 1; d1.sBn = nvo;
        d1.C = (unsigned char *)Bsel_bar + (size_t)s0 * nmo * ldk * es; d1.sCm = ldk; d1.sCn = 1;
        d1.alpha = 1.0; d1.beta = 0.0;
        CDS_CALL(cds_gemm_ex(ctx, gprec, d1, nullptr, nullptr));
        // Bvo_bar += W^T Bsel[s0..] : nvo x nvec, reduction over nsc*nmo
        const int64_t kc = (int64_t)nsc * nmo;
        CDS_CALL(cds_transpose(ctx, (int)es, kc, nvo, W, nvo, WT, kc));
        CDS_CALL(cds_transpose(ctx, (int)es, kc, nvec, (const unsigned char *)Bs + (size_t)s0 * nmo * ldk * es, ldk,
                               BsT, kc));
        GemmDesc d2 = {};
        d2.M = nvo; d2.N = nvec; d2.K = kc; d2.batch = 1;
        d2.A = WT; d2.sAm = kc; d2.sAk = 1;
        d2.B = BsT; d2.sBk = 1; d2.sBn = kc;
        d2.C = Bvo_bar; d2.sCm = ldk; d2.sCn = 1;
        d2.alpha = 1.0; d2.beta = s0 == 0 ? 0.0 : 1.0;
        CDS_CALL(cds_gemm_ex(ctx, gprec, d2, nullptr, nullptr));
    }
    if (ldk > nvec) {
        if (gprec == CDS_PREC_FP64) {
            hipLaunchKernelGGL(zero_cols_kernel<double>, dim3((unsigned)cds_ceil_div(nselr * (ldk - nvec), 256)),
                               dim3(256), 0, ctx->stream, (double *)Bsel_bar, nselr, ldk, nvec);
            hipLaunchKernelGGL(zero_cols_kernel<double>, dim3((unsigned)cds_ceil_div(nvo * (ldk - nvec), 256)),
                               dim3(256), 0, ctx->stream, (double *)Bvo_bar, nvo, ldk, nvec);
        } else {
            hipLaunchKernelGGL(zero_cols_kernel<float>, dim3((unsigned)cds_ceil_div(nselr * (ldk - nvec), 256)),
                               dim3(256), 0, ctx->stream, (float *)Bsel_bar, nselr, ldk, nvec);
            hipLaunchKernelGGL(zero_cols_kernel<float>, dim3((unsigned)cds_ceil_div(nvo * (ldk - nvec), 256)),
                               dim3(256), 0, ctx->stream, (float *)Bvo_bar, nvo, ldk, nvec);
        }
        CDS_LAUNCHED(ctx);
    }
    hipLaunchKernelGGL(eps_bar_kernel, dim3((unsigned)nmo), dim3(256), 0, ctx->stream,
                       (const double *)epsA, (const double *)epsB, nsel, nocc, nvirt, (const int32_t *)d_sel,
                       (const double *)d_scale, eps_bar);
    CDS_LAUNCHED(ctx);
    CDS_CALL(cds_timer_stop(ctx, &tall, &ctx->stats.t_adjoint_ms));
    CDS_CALL(cds_timers_flush(ctx));
    return CDS_OK;
}

extern "C" int cds_transform_adjoint(cds_ctx *ctx, int32_t prec, int32_t nbf, int64_t nvec,
                                     const double *L, int64_t ldl, const double *C, int32_t nmo,
                                     int32_t nocc, int32_t nsel, const int32_t *h_sel, int64_t ldk,
                                     const void *Bsel_bar, const void *Bvo_bar, double *C_bar)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, prec == CDS_PREC_FP64 || prec == CDS_PREC_FP32 || prec == CDS_PREC_BF16X3,
                "unknown precision %d", prec);
    CDS_REQUIRE(ctx, nbf >= 1 && nmo >= 2 && nmo <= nbf && nocc >= 1 && nocc < nmo, "bad sizes");
    CDS_REQUIRE(ctx, nsel >= 1 && h_sel, "bad targets");
    CDS_REQUIRE(ctx, nvec >= 1 && ldk >= nvec && ldl >= cds_npairs(nbf), "bad nvec/ldk/ldl");
    CDS_REQUIRE(ctx, L && C && Bsel_bar && Bvo_bar && C_bar, "NULL pointer");
    for (int s = 0; s < nsel; ++s)
        CDS_REQUIRE(ctx, h_sel[s] >= 0 && h_sel[s] < nmo, "h_sel[%d] out of range", s);
    CdsTimer tall;
    CDS_CALL(cds_timer_start(ctx, &tall));
    const int np_ = (int)(cds_ceil_div(nbf, 64) * 64);
    // vectors per batch: enough that the first product launches about 2048 tiles of 128 x 128,
    // with the unpacked batch below 1 GiB (C_bar sums the vectors in order whatever the batch)
    const int64_t tiles = cds_ceil_div(nmo, 128) * cds_ceil_div(nbf, 128);
    int64_t kbw = std::max<int64_t>(64, cds_ceil_div(2048, tiles));
    kbw = std::min<int64_t>(kbw, std::max<int64_t>(1, (int64_t)((1ull << 30) / ((size_t)nbf * np_ * 8))));
    const int kb = (int)std::min<int64_t>(kbw, nvec);
    void *wl, *ws, *wk, *wsel, *wp;
    CDS_CALL(cds_ws(ctx, WS_TR_UNPACK, (size_t)kb * nbf * np_ * 8, &wl));
    CDS_CALL(cds_ws(ctx, WS_AD_TMP2, (size_t)kb * nmo * nmo * 8, &ws));
    CDS_CALL(cds_ws(ctx, WS_TR_T, (size_t)kb * nmo * np_ * 8, &wk));
    CDS_CALL(cds_ws(ctx, WS_TR_CX, (size_t)nsel * 4 + 64, &wsel));
    CDS_CALL(cds_ws(ctx, WS_AD_TMP, (size_t)kb * nbf * nmo * 8, &wp));
    CDS_HIP(ctx, hipMemcpyAsync(wsel, h_sel, (size_t)nsel * 4, hipMemcpyHostToDevice, ctx->stream));
    // Wt columns nbf..np_-1 are never written: zero once so the padded K range adds nothing
    CDS_HIP(ctx, hipMemsetAsync(wk, 0, (size_t)kb * nmo * np_ * 8, ctx->stream));
    for (int64_t k0 = 0; k0 < nvec; k0 += kb) {
        const int nkb = (int)std::min<int64_t>(kb, nvec - k0);
        int64_t n1 = (int64_t)nkb * nbf * np_;
        hipLaunchKernelGGL(unpack64_kernel, dim3((unsigned)cds_ceil_div(n1, 256)), dim3(256), 0, ctx->stream, L,
                           ldl, k0, nkb, nbf, np_, (double *)wl);
        int64_t n2 = (int64_t)nkb * nmo * nmo;
        if (prec == CDS_PREC_FP64)
            hipLaunchKernelGGL(sym_bar_kernel<double>, dim3((unsigned)cds_ceil_div(n2, 256)), dim3(256), 0,
                               ctx->stream, (const double *)Bsel_bar, (const double *)Bvo_bar, ldk, k0, nkb,
                               nmo, nocc, nsel, (const int32_t *)wsel, (double *)ws);
        else
            hipLaunchKernelGGL(sym_bar_kernel<float>, dim3((unsigned)cds_ceil_div(n2, 256)), dim3(256), 0,
                               ctx->stream, (const float *)Bsel_bar, (const float *)Bvo_bar, ldk, k0, nkb,
                               nmo, nocc, nsel, (const int32_t *)wsel, (double *)ws);
        CDS_LAUNCHED(ctx);
        // Wt[kb][p][nu] = sum_r S[kb][p][r] C[nu][r]   (S symmetric; both operands K-contiguous)
        GemmDesc g1 = {};
        g1.M = nmo; g1.N = nbf; g1.K = nmo; g1.batch = nkb;
        g1.A = ws; g1.sAm = nmo; g1.sAk = 1; g1.sAb = (int64_t)nmo * nmo;
        g1.B = C; g1.sBn = nmo; g1.sBk = 1; g1.sBb = 0;
        g1.C = wk; g1.sCm = np_; g1.sCn = 1; g1.sCb = (int64_t)nmo * np_;
        g1.alpha = 1.0; g1.beta = 0.0;
        CDS_CALL(cds_gemm_ex(ctx, CDS_PREC_FP64, g1, nullptr, nullptr));
        // part[kb][mu][p] = sum_nu Lu[kb][mu][nu] Wt[kb][p][nu]: one product per vector (the batch
        // index splits the long reduction over (kb, nu) so the tiny output still fills the chip)
        GemmDesc g2 = {};
        g2.M = nbf; g2.N = nmo; g2.K = np_; g2.batch = nkb;
        g2.A = wl; g2.sAm = np_; g2.sAk = 1; g2.sAb = (int64_t)nbf * np_;
        g2.B = wk; g2.sBn = np_; g2.sBk = 1; g2.sBb = (int64_t)nmo * np_;
        g2.C = wp; g2.sCm = nmo; g2.sCn = 1; g2.sCb = (int64_t)nbf * nmo;
        g2.alpha = 1.0; g2.beta = 0.0;
        CDS_CALL(cds_gemm_ex(ctx, CDS_PREC_FP64, g2, nullptr, nullptr));
        // C_bar (+)= sum_kb part[kb] in fixed order
        const int64_t ne = (int64_t)nbf * nmo;
        hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)cds_ceil_div(ne, 256)), dim3(256), 0, ctx->stream,
                           (const double *)wp, nkb, ne, k0 > 0 ? 1 : 0, C_bar);
        CDS_LAUNCHED(ctx);
    }
    CDS_CALL(cds_timer_stop(ctx, &tall, &ctx->stats.t_adjoint_ms));
    return CDS_OK;
}
