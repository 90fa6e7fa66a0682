// Non-diagonal second-order self-energy over selected orbitals and the Dyson pole
// search (Sec. II.B of the paper: Eqs. (Dyson), (DysonSol), (DysonSol2); Eq. (SE) is the
// diagonal of this matrix):
//   Sigma_st(w) = sum_{a,i,j} (si|aj) (2(ti|aj) - (tj|ai)) / (w + e_a - e_i - e_j)
//               + sum_{i,a,b} (sa|ib) (2(ta|ib) - (tb|ia)) / (w + e_i - e_a - e_b).
// The integrals of all selected orbitals come from one MFMA contraction
// G[s][r][a*nocc+j] = (s r|a j).  Both families are summed over unordered index pairs
// (d is symmetric in i, j and in a, b): element e = (a; i <= j) or (i; a <= b) carries
//   u_s = (si|aj), v_s = (sj|ai)   resp.   u_s = (sa|ib), v_s = (sb|ia),
// and contributes c_e (2 u_s u_t + 2 v_s v_t - u_s v_t - v_s u_t) / (w + d_e) to Sigma_st,
// with c_e = 1/2 on the diagonal (i = j, a = b) and 1 otherwise.  sigma_pairs_kernel
// stages chunks of elements (u, v of every selected orbital, weights for every trial
// energy) in LDS; each thread owns two (s <= t) pairs; per-block partial sums are reduced
// in a fixed order.
//
// The Dyson search (host loop of the library, like the quasi-particle Newton solve): one
// root per selected orbital, started at e_q with u = unit vector q; at each step the
// symmetric matrix diag(e_S) + Sigma_SS(w) is diagonalised (cyclic Jacobi), the
// eigenvector of largest overlap with the previous one is followed, and
//   w <- w + (lambda - w) P,   P = 1 / (1 - u^T Sigma'(w) u)
// until |dw| <= conv (Eq. (NR)); P is the pole strength.  With one orbital this is Eq. (iter).
#include "cds_internal.h"

#include <cmath>
#include <vector>

int cds_contract_internal(cds_ctx *ctx, int prec, int64_t nvec, int64_t ldk, int nmo, int nocc,
                          int nsel, const void *Bsel, const void *Bvo, int s0, int nsc, void *G);

namespace {

constexpr int DY_NT = 256;
constexpr int DY_CH = 64;            // elements per chunk
constexpr int DY_MAXSEL = 31;        // selected orbitals (<= 2 pairs per thread)
constexpr int DY_TT = 8;             // trial energies per launch
constexpr int DY_BLOCKS = 2048;
constexpr size_t DY_G_MAX = (size_t)16 << 30;

__device__ __forceinline__ int64_t tri_hi(int64_t x)
{
    // largest b with b(b+1)/2 <= x
    int64_t b = (int64_t)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    if (b * (b + 1) / 2 > x) --b;
    if ((b + 1) * (b + 2) / 2 <= x) ++b;
    return b;
}

template <typename GT>
__global__ __launch_bounds__(DY_NT) void sigma_pairs_kernel(const GT *__restrict__ G, int nsel, int nmo, int nocc,
                                                           int nvirt, int64_t nvo, const double *__restrict__ eps,
                                                           const double *__restrict__ omega, int T, int64_t nA,
                                                           int64_t nE, int64_t cpb, double *__restrict__ part)
{
    // rows padded by one element: lanes of a wave read one element l of different orbitals s,
    // which a pitch of DY_CH doubles would put in one bank
    __shared__ double su[DY_MAXSEL][DY_CH + 1], sv[DY_MAXSEL][DY_CH + 1];
    __shared__ double sw[DY_TT][DY_CH], swi[DY_TT][DY_CH];
    __shared__ int64_t ou[DY_CH], ov[DY_CH];
    const int npair = nsel * (nsel + 1) / 2;
    const int64_t gstride = (int64_t)nmo * nvo;
    int ps[2], pt[2];
    bool pok[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int P = threadIdx.x + h * DY_NT;
        pok[h] = P < npair;
        const int t = pok[h] ? (int)tri_hi(P) : 0;
        pt[h] = t;
        ps[h] = pok[h] ? P - t * (t + 1) / 2 : 0;
    }
    double acc[2][DY_TT][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < DY_TT; ++t) acc[h][t][0] = acc[h][t][1] = 0.0;
    const int64_t np2 = (int64_t)nocc * (nocc + 1) / 2, nv2 = (int64_t)nvirt * (nvirt + 1) / 2;
    const int64_t c0 = (int64_t)blockIdx.x * cpb;
    for (int64_t c = c0; c < c0 + cpb; ++c) {
        const int64_t e0 = c * DY_CH;
        if (e0 >= nE) break;
        __syncthreads();
        if (threadIdx.x < DY_CH) {
            const int l = threadIdx.x;
            const int64_t e = e0 + l;
            int64_t offu = 0, offv = 0;
            double d = 0.0, ce = 0.0;
            if (e < nA) {
                const int64_t a = e / np2, ij = e - a * np2;
                const int64_t j = tri_hi(ij), i = ij - j * (j + 1) / 2;
                offu = i * nvo + a * nocc + j;
                offv = j * nvo + a * nocc + i;
                d = eps[nocc + a] - eps[i] - eps[j];
                ce = i == j ? 0.5 : 1.0;
            } else if (e < nE) {
                const int64_t f = e - nA;
                const int64_t i = f / nv2, ab = f - i * nv2;
                const int64_t b = tri_hi(ab), a = ab - b * (b + 1) / 2;
                offu = (nocc + a) * nvo + b * nocc + i;
                offv = (nocc + b) * nvo + a * nocc + i;
                d = eps[i] - eps[nocc + a] - eps[nocc + b];
                ce = a == b ? 0.5 : 1.0;
            }
            ou[l] = offu;
            ov[l] = offv;
#pragma unroll
            for (int t = 0; t < DY_TT; ++t) {
                const double inv = t < T ? 1.0 / (omega[t] + d) : 0.0;
                sw[t][l] = ce * inv;
                swi[t][l] = inv;
            }
        }
        __syncthreads();
        {
            // every gathered load of a thread in flight before its LDS stores
            constexpr int QN = (DY_MAXSEL * DY_CH + DY_NT - 1) / DY_NT;
            double gu[QN], gv[QN];
#pragma unroll
            for (int u = 0; u < QN; ++u) {
                const int q = threadIdx.x + u * DY_NT;
                const int s = q / DY_CH, l = q - s * DY_CH;
                const bool ok = q < nsel * DY_CH && e0 + l < nE;
                gu[u] = ok ? (double)G[s * gstride + ou[l]] : 0.0;
                gv[u] = ok ? (double)G[s * gstride + ov[l]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < QN; ++u) {
                const int q = threadIdx.x + u * DY_NT;
                const int s = q / DY_CH, l = q - s * DY_CH;
                if (q < nsel * DY_CH) {
                    su[s][l] = gu[u];
                    sv[s][l] = gv[u];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!pok[h]) continue;
            const int s = ps[h], t2 = pt[h];
            for (int l = 0; l < DY_CH; ++l) {
                const double us = su[s][l], vs = sv[s][l], ut = su[t2][l], vt = sv[t2][l];
                const double num = 2.0 * (us * ut + vs * vt) - us * vt - vs * ut;
#pragma unroll
                for (int t = 0; t < DY_TT; ++t) {
                    const double x = num * sw[t][l];
                    acc[h][t][0] += x;
                    acc[h][t][1] -= x * swi[t][l];
                }
            }
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (!pok[h]) continue;
        const int P = threadIdx.x + h * DY_NT;
        double *dst = part + ((int64_t)blockIdx.x * npair + P) * DY_TT * 2;
#pragma unroll
        for (int t = 0; t < DY_TT; ++t) {
            dst[2 * t] = acc[h][t][0];
            dst[2 * t + 1] = acc[h][t][1];
        }
    }
}

// out[q] = sum_b part[b][q], q over pairs x DY_TT x 2: one wave per output, lane l sums
// blocks l, l+64, ... in order, then a fixed shuffle tree (deterministic)
__global__ void pairs_reduce_kernel(const double *__restrict__ part, int nblk, int64_t nq, double *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    if (q >= nq) return;                                   // whole waves leave together
    double a = 0.0;
    for (int b = l; b < nblk; b += 64) a += part[(int64_t)b * nq + q];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (l == 0) out[q] = a;
}

// cyclic Jacobi for a symmetric n x n matrix (row-major, destroyed): eigenvalues w,
// eigenvectors in the columns of V
void jacobi_eigh(int n, std::vector<double> &A, std::vector<double> &w, std::vector<double> &V)
{
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {              // columns p, q
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {              // rows p, q
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

struct DyState {
    int prec, nmo, nocc, nvirt, nsel;
    int64_t nvo;
    void *G;
    const double *eps;
    double *d_omega, *part, *out;
    int nblk;
    int64_t cpb, nA, nE;
};

int dy_setup(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo, int32_t nocc, int32_t nsel,
             const int32_t *h_sel, const void *Bsel, const void *Bvo, const double *eps, DyState &S)
{
    CDS_REQUIRE(ctx, prec == CDS_PREC_FP64 || prec == CDS_PREC_FP32 || prec == CDS_PREC_BF16X3,
                "unknown precision %d", prec);
    CDS_REQUIRE(ctx, nmo >= 2 && nocc >= 1 && nocc < nmo, "need 1 <= nocc < nmo");
    CDS_REQUIRE(ctx, nsel >= 1 && nsel <= DY_MAXSEL && h_sel, "need 1 <= nsel <= %d and h_sel", DY_MAXSEL);
    CDS_REQUIRE(ctx, nvec >= 1 && ldk >= nvec && ldk % 64 == 0, "need 1 <= nvec <= ldk, ldk a multiple of 64");
    CDS_REQUIRE(ctx, Bsel && Bvo && eps, "NULL pointer");
    for (int s = 0; s < nsel; ++s)
        CDS_REQUIRE(ctx, h_sel[s] >= 0 && h_sel[s] < nmo, "h_sel[%d] out of range", s);
    S.prec = prec;
    S.nmo = nmo;
    S.nocc = nocc;
    S.nvirt = nmo - nocc;
    S.nsel = nsel;
    S.nvo = (int64_t)S.nvirt * nocc;
    S.eps = eps;
    const size_t gs = prec == CDS_PREC_FP64 ? 8 : 4;
    const size_t gbytes = (size_t)nsel * nmo * S.nvo * gs;
    CDS_REQUIRE(ctx, gbytes <= DY_G_MAX, "integrals of the selected orbitals exceed %zu bytes", DY_G_MAX);
    CDS_CALL(cds_ws(ctx, WS_DY_G, gbytes, &S.G));
    S.nA = (int64_t)S.nvirt * ((int64_t)nocc * (nocc + 1) / 2);
    S.nE = S.nA + (int64_t)nocc * ((int64_t)S.nvirt * (S.nvirt + 1) / 2);
    const int64_t nch = cds_ceil_div(S.nE, DY_CH);
    S.nblk = (int)std::min<int64_t>(DY_BLOCKS, nch);
    S.cpb = cds_ceil_div(nch, S.nblk);
    const int npair = nsel * (nsel + 1) / 2;
    void *w;
    const size_t nq = (size_t)npair * DY_TT * 2;
    CDS_CALL(cds_ws(ctx, WS_DY_PART, ((size_t)S.nblk * nq + nq + DY_TT) * 8, &w));
    S.part = (double *)w;
    S.out = S.part + (size_t)S.nblk * nq;
    S.d_omega = S.out + nq;
    // all selected orbitals' integrals in one contraction
    CDS_CALL(cds_contract_internal(ctx, prec, nvec, ldk, nmo, nocc, nsel, Bsel, Bvo, 0, nsel, S.G));
    return CDS_OK;
}

// Sigma_SS and Sigma'_SS at up to DY_TT trial energies -> host (T x nsel x nsel each)
int dy_eval(cds_ctx *ctx, const DyState &S, int T, const double *h_w, double *h_sig, double *h_dsig)
{
    const int npair = S.nsel * (S.nsel + 1) / 2;
    const int64_t nq = (int64_t)npair * DY_TT * 2;
    void *hp;
    CDS_CALL(cds_pinned(ctx, (size_t)nq * 8 + 256, &hp));
    double *hb = (double *)hp;
    for (int t = 0; t < DY_TT; ++t) hb[t] = h_w[t < T ? t : T - 1];
    CDS_HIP(ctx, hipMemcpyAsync(S.d_omega, hb, DY_TT * 8, hipMemcpyHostToDevice, ctx->stream));
    if (S.prec == CDS_PREC_FP64)
        hipLaunchKernelGGL(sigma_pairs_kernel<double>, dim3((unsigned)S.nblk), dim3(DY_NT), 0, ctx->stream,
                           (const double *)S.G, S.nsel, S.nmo, S.nocc, S.nvirt, S.nvo, S.eps,
                           (const double *)S.d_omega, T, S.nA, S.nE, S.cpb, S.part);
    else
        hipLaunchKernelGGL(sigma_pairs_kernel<float>, dim3((unsigned)S.nblk), dim3(DY_NT), 0, ctx->stream,
                           (const float *)S.G, S.nsel, S.nmo, S.nocc, S.nvirt, S.nvo, S.eps,
                           (const double *)S.d_omega, T, S.nA, S.nE, S.cpb, S.part);
    CDS_LAUNCHED(ctx);
    hipLaunchKernelGGL(pairs_reduce_kernel, dim3((unsigned)cds_ceil_div(nq, 4)), dim3(256), 0, ctx->stream,
                       (const double *)S.part, S.nblk, nq, S.out);
    CDS_LAUNCHED(ctx);
    CDS_HIP(ctx, hipMemcpyAsync(hb, S.out, (size_t)nq * 8, hipMemcpyDeviceToHost, ctx->stream));
    CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int n = S.nsel;
    for (int P = 0; P < npair; ++P) {
        int t2 = 0;
        while ((t2 + 1) * (t2 + 2) / 2 <= P) ++t2;
        const int s = P - t2 * (t2 + 1) / 2;
        for (int t = 0; t < T; ++t) {
            const double v = hb[((size_t)P * DY_TT + t) * 2], dv = hb[((size_t)P * DY_TT + t) * 2 + 1];
            h_sig[(size_t)t * n * n + (size_t)s * n + t2] = h_sig[(size_t)t * n * n + (size_t)t2 * n + s] = v;
            h_dsig[(size_t)t * n * n + (size_t)s * n + t2] = h_dsig[(size_t)t * n * n + (size_t)t2 * n + s] = dv;
        }
    }
    return CDS_OK;
}

}  // namespace

extern "C" int cds_sigma2_matrix(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo,
                                 int32_t nocc, int32_t nsel, const int32_t *h_sel, const void *Bsel,
                                 const void *Bvo, const double *eps, int32_t T, const double *h_omega,
                                 double *h_sigma, double *h_dsigma)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, T >= 1 && T <= 1024 && h_omega && h_sigma && h_dsigma, "need 1 <= T <= 1024 and host arrays");
    DyState S;
    CdsTimer tm;
    CDS_CALL(cds_timer_start(ctx, &tm));
    CDS_CALL(dy_setup(ctx, prec, nvec, ldk, nmo, nocc, nsel, h_sel, Bsel, Bvo, eps, S));
    const size_t nn = (size_t)nsel * nsel;
    for (int t0 = 0; t0 < T; t0 += DY_TT) {
        const int nt = std::min(DY_TT, T - t0);
        CDS_CALL(dy_eval(ctx, S, nt, h_omega + t0, h_sigma + t0 * nn, h_dsigma + t0 * nn));
    }
    CDS_CALL(cds_timer_stop(ctx, &tm, &ctx->stats.t_dyson_ms));
    CDS_CALL(cds_timers_flush(ctx));
    return CDS_OK;
}

extern "C" int cds_dyson_solve(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo, int32_t nocc,
                               int32_t nsel, const int32_t *h_sel, const void *Bsel, const void *Bvo,
                               const double *eps, double conv, int32_t max_iter, double *h_omega, double *h_pole,
                               double *h_vec, int32_t *h_iters, int32_t *h_status)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, conv > 0.0 && max_iter >= 1, "need conv > 0 and max_iter >= 1");
    CDS_REQUIRE(ctx, h_omega && h_pole && h_vec && h_iters && h_status, "NULL host pointer");
    DyState S;
    CdsTimer tm;
    CDS_CALL(cds_timer_start(ctx, &tm));
    CDS_CALL(dy_setup(ctx, prec, nvec, ldk, nmo, nocc, nsel, h_sel, Bsel, Bvo, eps, S));
    const int n = nsel;
    std::vector<double> eS(n), w(n), pole(n, NAN), U((size_t)n * n, 0.0);
    {
        std::vector<double> eh(nmo);
        void *hp;
        CDS_CALL(cds_pinned(ctx, (size_t)nmo * 8, &hp));
        CDS_HIP(ctx, hipMemcpyAsync(hp, eps, (size_t)nmo * 8, hipMemcpyDeviceToHost, ctx->stream));
        CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
        std::copy((const double *)hp, (const double *)hp + nmo, eh.begin());
        for (int k = 0; k < n; ++k) {
            eS[k] = eh[h_sel[k]];
            w[k] = eS[k];
            U[(size_t)k * n + k] = 1.0;                    // row k: tracked vector of root k
        }
    }
    std::vector<int> status(n, -1), iters(n, 0);
    std::vector<double> sig((size_t)DY_TT * n * n), dsig((size_t)DY_TT * n * n), A, lam, V;
    for (int it = 1; it <= max_iter; ++it) {
        std::vector<int> act;
        for (int k = 0; k < n; ++k)
            if (status[k] < 0) act.push_back(k);
        if (act.empty()) break;
        for (size_t b0 = 0; b0 < act.size(); b0 += DY_TT) {
            const int nt = (int)std::min<size_t>(DY_TT, act.size() - b0);
            double wt[DY_TT];
            for (int t = 0; t < nt; ++t) wt[t] = w[act[b0 + t]];
            CDS_CALL(dy_eval(ctx, S, nt, wt, sig.data(), dsig.data()));
            for (int t = 0; t < nt; ++t) {
                const int k = act[b0 + t];
                A.assign(sig.begin() + (size_t)t * n * n, sig.begin() + (size_t)(t + 1) * n * n);
                for (int i = 0; i < n; ++i) A[(size_t)i * n + i] += eS[i];
                jacobi_eigh(n, A, lam, V);
                int jb = 0;
                double best = -1.0, sgn = 1.0;
                for (int j = 0; j < n; ++j) {
                    double ov = 0.0;
                    for (int i = 0; i < n; ++i) ov += V[(size_t)i * n + j] * U[(size_t)k * n + i];
                    if (std::fabs(ov) > best) {
                        best = std::fabs(ov);
                        jb = j;
                        sgn = ov >= 0.0 ? 1.0 : -1.0;
                    }
                }
                double sp = 0.0;
                const double *dS = dsig.data() + (size_t)t * n * n;
                for (int i = 0; i < n; ++i) {
                    U[(size_t)k * n + i] = sgn * V[(size_t)i * n + jb];
                }
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) sp += U[(size_t)k * n + i] * dS[(size_t)i * n + j] * U[(size_t)k * n + j];
                const double P = 1.0 / (1.0 - sp);
                const double wn = w[k] + (lam[jb] - w[k]) * P;
                pole[k] = P;
                iters[k] = it;
                if (!std::isfinite(wn) || !std::isfinite(P)) {
                    w[k] = wn;
                    status[k] = CDS_QP_NONFINITE;
                } else if (std::fabs(wn - w[k]) <= conv) {
                    w[k] = wn;
                    status[k] = CDS_QP_CONVERGED;
                } else {
                    w[k] = wn;
                }
            }
        }
    }
    for (int k = 0; k < n; ++k) {
        h_omega[k] = w[k];
        h_pole[k] = pole[k];
        h_iters[k] = iters[k];
        h_status[k] = status[k] < 0 ? CDS_QP_MAX_ITER : status[k];
        for (int i = 0; i < n; ++i) h_vec[(size_t)k * n + i] = U[(size_t)k * n + i];
    }
    CDS_CALL(cds_timer_stop(ctx, &tm, &ctx->stats.t_dyson_ms));
    CDS_CALL(cds_timers_flush(ctx));
    return CDS_OK;
}
