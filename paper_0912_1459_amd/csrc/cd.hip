// Diagonal-pivoted incomplete Cholesky decomposition of the ERI supermatrix
// (Sec. II.A of the paper: Eqs. (gs_coulomb), (CD), (stricterr)) with ERI
// columns of normalized s-Gaussians evaluated on demand (Eq. (integral),
// closed form through the Boys function F0).
//
// Device layout (HBM):
//   pair table  SoA  p[I], Px[I], Py[I], Pz[I], K[I]     5 x npairs FP64
//   L           vector-major, vector k at L + k*ldl        FP64
//   D           residual diagonal                           FP64[npairs]
//   mask        1 on pivot pairs                            u8[npairs]
//   part        partial GEMV sums, split s at part + s*npad FP64
//
// One step k (three launches, no host round trip):
//   cd_partial   grid (row tiles x j-splits): part[s][I] = sum_{j in split s} L[j][I] L[j][p]
//   cd_finalize  grid (row tiles): c_I = V_Ip - sum_s part[s][I]; L[k][I] = c_I / sqrt(D_p)
//                (0 on earlier pivots, sqrt(D_p) on p); D_I -= L[k][I]^2; per-tile max/min
//   cd_select    one block: D_max, status, next pivot = lowest index with D_I >= D_max - tau
// The partial kernel streams k*npairs*8 bytes of L per step: it is HBM-bound.
#include "cds_internal.h"

#include <cfloat>
#include <climits>

namespace {

constexpr int CD_BLOCK = 256;           // threads of the partial/finalize kernels
constexpr int CD_JCHUNK = 128;          // vectors per j-split of the partial GEMV
constexpr int CD_FIN_TILE = 256;        // rows per finalize tile (one per thread)
constexpr int CD_SEL_BLOCK = 1024;

struct PairTable {
    double *p, *Px, *Py, *Pz, *K;
};

struct CdState {
    int64_t k;       // vectors made so far
    int64_t p;       // pivot of the next vector
    double dp;       // residual diagonal of that pivot
    double dmax;     // largest non-pivot residual diagonal
    int32_t done;    // 1 once a termination rule fired
    int32_t status;  // CDS_CD_* once done
};

__device__ __forceinline__ double boys_f0(double T)
{
    if (T < 1e-12) return 1.0 - T / 3.0 + T * T / 10.0;
    return 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
}

// (rho_I | V | rho_J) for two s-Gaussian product densities
__device__ __forceinline__ double eri_pp(double p, double Px, double Py, double Pz, double Kp,
                                         double q, double Qx, double Qy, double Qz, double Kq)
{
    const double two_pi_52 = 2.0 * 17.493418327624862;   // 2 pi^(5/2)
    double dx = Px - Qx, dy = Py - Qy, dz = Pz - Qz;
    double r2 = dx * dx + dy * dy + dz * dz;
    double s = p + q;
    double T = p * q / s * r2;
    return Kp * Kq * two_pi_52 / (p * q * sqrt(s)) * boys_f0(T);
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
__device__ __forceinline__ double block_min(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    v = (threadIdx.x < NT / 64) ? sh[threadIdx.x] : INFINITY;
    if (w == 0)
        for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if (threadIdx.x == 0) sh[0] = v;
    __syncthreads();
    return sh[0];
}

template <int NT>
__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t *sh)
{
    for (int o = 32; o > 0; o >>= 1) {
        int64_t u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    v = (threadIdx.x < NT / 64) ? sh[threadIdx.x] : INT64_MAX;
    if (w == 0)
        for (int o = 32; o > 0; o >>= 1) {
            int64_t u = __shfl_xor(v, o, 64);
            v = u < v ? u : v;
        }
    __syncthreads();
    if (threadIdx.x == 0) sh[0] = v;
    __syncthreads();
    return sh[0];
}

// ---- CD kernels ------------------------------------------------------------------
__global__ void mark_pivots_kernel(int64_t n, const int64_t *__restrict__ piv, int64_t npairs,
                                   unsigned char *__restrict__ mask)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) {
        int64_t p = piv[j];
        if (p >= 0 && p < npairs) mask[p] = 1;
    }
}

// per-tile max and min of non-pivot residual diagonals (start / resume)
__global__ __launch_bounds__(CD_FIN_TILE) void tile_stats_kernel(
    int64_t npairs, const double *__restrict__ D, const unsigned char *__restrict__ mask,
    double *__restrict__ tmax, double *__restrict__ tmin)
{
    __shared__ double sh[CD_FIN_TILE / 64];
    int64_t I = (int64_t)blockIdx.x * CD_FIN_TILE + threadIdx.x;
    double mx = -INFINITY, mn = INFINITY;
    if (I < npairs && !mask[I]) mx = mn = D[I];
    mx = block_max<CD_FIN_TILE>(mx, sh);
    mn = block_min<CD_FIN_TILE>(mn, sh);
    if (threadIdx.x == 0) {
        tmax[blockIdx.x] = mx;
        tmin[blockIdx.x] = mn;
    }
}

// part[s][I..I+VW-1] = sum_{j in split s} L[j][I] * L[j][p]
template <int VW>
__global__ __launch_bounds__(CD_BLOCK) void cd_partial_kernel(
    const double *__restrict__ L, int64_t ldl, int64_t npairs, int64_t npad,
    const CdState *__restrict__ st, double *__restrict__ part)
{
    __shared__ double prow[CD_JCHUNK];
    if (st->done) return;
    const int64_t k = st->k, p = st->p;
    const int64_t j0 = (int64_t)blockIdx.y * CD_JCHUNK;
    const int64_t j1 = min(j0 + (int64_t)CD_JCHUNK, k);
    const int nj = (int)(j1 - j0);
    for (int t = threadIdx.x; t < nj; t += CD_BLOCK) prow[t] = L[(j0 + t) * ldl + p];
    __syncthreads();
    const int64_t I = ((int64_t)blockIdx.x * CD_BLOCK + threadIdx.x) * VW;
    if (I >= npairs) return;
    const double *Lp = L + j0 * ldl + I;
    if constexpr (VW == 2) {
        double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
        int j = 0;
        for (; j + 4 <= nj; j += 4) {
            double2 v0 = *reinterpret_cast<const double2 *>(Lp + (int64_t)(j + 0) * ldl);
            double2 v1 = *reinterpret_cast<const double2 *>(Lp + (int64_t)(j + 1) * ldl);
            double2 v2 = *reinterpret_cast<const double2 *>(Lp + (int64_t)(j + 2) * ldl);
            double2 v3 = *reinterpret_cast<const double2 *>(Lp + (int64_t)(j + 3) * ldl);
            a0 = fma(v0.x, prow[j], a0);
            a1 = fma(v0.y, prow[j], a1);
            b0 = fma(v1.x, prow[j + 1], b0);
            b1 = fma(v1.y, prow[j + 1], b1);
            a0 = fma(v2.x, prow[j + 2], a0);
            a1 = fma(v2.y, prow[j + 2], a1);
            b0 = fma(v3.x, prow[j + 3], b0);
            b1 = fma(v3.y, prow[j + 3], b1);
        }
        for (; j < nj; ++j) {
            double2 v = *reinterpret_cast<const double2 *>(Lp + (int64_t)j * ldl);
            a0 = fma(v.x, prow[j], a0);
            a1 = fma(v.y, prow[j], a1);
        }
        double2 r;
        r.x = a0 + b0;
        r.y = a1 + b1;
        *reinterpret_cast<double2 *>(part + (int64_t)blockIdx.y * npad + I) = r;
    } else {
        double a0 = 0.0, b0 = 0.0;
        int j = 0;
        for (; j + 2 <= nj; j += 2) {
            a0 = fma(Lp[(int64_t)j * ldl], prow[j], a0);
            b0 = fma(Lp[(int64_t)(j + 1) * ldl], prow[j + 1], b0);
        }
        for (; j < nj; ++j) a0 = fma(Lp[(int64_t)j * ldl], prow[j], a0);
        part[(int64_t)blockIdx.y * npad + I] = a0 + b0;
    }
}

// new vector k, residual diagonal update, per-tile max/min of the updated D
template <bool DENSE>
__global__ __launch_bounds__(CD_FIN_TILE) void cd_finalize_kernel(
    PairTable pt, const double *__restrict__ V, int64_t ldv, double *__restrict__ L, int64_t ldl,
    int64_t npairs, int64_t npad, const double *__restrict__ part, int nsplit,
    double *__restrict__ D, unsigned char *__restrict__ mask, const CdState *__restrict__ st,
    double *__restrict__ tmax, double *__restrict__ tmin)
{
    __shared__ double sh[CD_FIN_TILE / 64];
    if (st->done) return;
    const int64_t k = st->k, p = st->p;
    const double sq = sqrt(st->dp);
    const int64_t I = (int64_t)blockIdx.x * CD_FIN_TILE + threadIdx.x;
    double mx = -INFINITY, mn = INFINITY;
    if (I < npairs) {
        double l;
        if (mask[I]) {
            l = 0.0;                          // earlier pivot: exactly zero
        } else if (I == p) {
            l = sq;                           // the pivot's own entry
        } else {
            double c;
            if constexpr (DENSE) {
                c = V[p * ldv + I];
            } else {
                c = eri_pp(pt.p[I], pt.Px[I], pt.Py[I], pt.Pz[I], pt.K[I], pt.p[p], pt.Px[p],
                           pt.Py[p], pt.Pz[p], pt.K[p]);
            }
            double acc = 0.0;
            for (int s = 0; s < nsplit; ++s) acc += part[(int64_t)s * npad + I];
            c -= acc;
            l = c / sq;
            double d = D[I] - l * l;
            D[I] = d;
            mx = mn = d;
        }
        L[k * ldl + I] = l;
        if (I == p) {
            D[I] = 0.0;
            mask[I] = 1;
        }
    }
    mx = block_max<CD_FIN_TILE>(mx, sh);
    mn = block_min<CD_FIN_TILE>(mn, sh);
    if (threadIdx.x == 0) {
        tmax[blockIdx.x] = mx;
        tmin[blockIdx.x] = mn;
    }
}

// termination tests and the next pivot (one block)
__global__ __launch_bounds__(CD_SEL_BLOCK) void cd_select_kernel(
    int after_step, int64_t ntiles, const double *__restrict__ tmax,
    const double *__restrict__ tmin, const double *__restrict__ D,
    const unsigned char *__restrict__ mask, int64_t npairs, double delta, double tau,
    double psd_tol, int64_t max_vec, CdState *st, int64_t *__restrict__ piv)
{
    __shared__ double shd[CD_SEL_BLOCK / 64];
    __shared__ int64_t shi[CD_SEL_BLOCK / 64];
    if (st->done) return;
    int64_t k = st->k;
    if (after_step) {
        if (threadIdx.x == 0) piv[k] = st->p;
        k += 1;
    }
    double mx = -INFINITY, mn = INFINITY;
    for (int64_t t = threadIdx.x; t < ntiles; t += CD_SEL_BLOCK) {
        mx = fmax(mx, tmax[t]);
        mn = fmin(mn, tmin[t]);
    }
    mx = block_max<CD_SEL_BLOCK>(mx, shd);
    mn = block_min<CD_SEL_BLOCK>(mn, shd);
    int status = -100;
    if (mn < -psd_tol) status = CDS_CD_NOTPSD;
    else if (mx == -INFINITY) status = CDS_CD_FULLRANK;
    else if (mx <= delta) status = CDS_CD_CONVERGED;
    else if (k >= max_vec) status = CDS_CD_CAP;
    if (status != -100) {
        if (threadIdx.x == 0) {
            st->k = k;
            st->dmax = mx;
            st->status = status;
            st->done = 1;
        }
        return;
    }
    const double thresh = mx - tau;
    int64_t ft = INT64_MAX;
    for (int64_t t = threadIdx.x; t < ntiles; t += CD_SEL_BLOCK)
        if (tmax[t] >= thresh && t < ft) ft = t;
    ft = block_min_i64<CD_SEL_BLOCK>(ft, shi);
    int64_t cand = INT64_MAX;
    if (ft != INT64_MAX && threadIdx.x < CD_FIN_TILE) {
        int64_t I = ft * CD_FIN_TILE + threadIdx.x;
        if (I < npairs && !mask[I] && D[I] >= thresh) cand = I;
    }
    cand = block_min_i64<CD_SEL_BLOCK>(cand, shi);
    if (cand == INT64_MAX) {
        // no candidate although D_max > delta: only possible with non-finite residuals
        if (threadIdx.x == 0) {
            st->k = k;
            st->dmax = mx;
            st->status = CDS_CD_NOTPSD;
            st->done = 1;
        }
        return;
    }
    if (threadIdx.x == 0) {
        st->k = k;
        st->p = cand;
        st->dp = D[cand];
        st->dmax = mx;
    }
}

__global__ void max_reduce_kernel(int64_t n, const double *__restrict__ x, double *__restrict__ out)
{
    __shared__ double sh[CD_SEL_BLOCK / 64];
    double m = -INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += CD_SEL_BLOCK) m = fmax(m, x[i]);
    m = block_max<CD_SEL_BLOCK>(m, sh);
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

int cholesky_impl(cds_ctx *ctx, bool dense, int32_t nbf, const double *centres,
                  const double *alpha, int64_t npairs, const double *V, int64_t ldv, double delta,
                  double tau, double psd_tol, int64_t max_vec, double *L, int64_t ldl,
                  int64_t *piv, double *D, int64_t nvec_in, int64_t *h_nvec, double *h_dmax,
                  int32_t *h_status)
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
    const int64_t rows_per_block = (int64_t)CD_BLOCK * vw;
    const int64_t ntile_part = cds_ceil_div(npairs, rows_per_block);
    const int64_t npad = ntile_part * rows_per_block;
    const int64_t ntile_fin = cds_ceil_div(npairs, CD_FIN_TILE);
    const int64_t max_split = cds_ceil_div(max_vec, CD_JCHUNK);

    void *w_part, *w_tile, *w_mask, *w_state;
    CDS_CALL(cds_ws(ctx, WS_CD_PART, (size_t)std::max<int64_t>(max_split, 1) * npad * 8 + npairs * 8,
                    &w_part));
    CDS_CALL(cds_ws(ctx, WS_CD_TILE, (size_t)2 * ntile_fin * 8 + 64, &w_tile));
    CDS_CALL(cds_ws(ctx, WS_CD_MASK, (size_t)npairs, &w_mask));
    CDS_CALL(cds_ws(ctx, WS_CD_STATE, sizeof(CdState), &w_state));
    double *part = (double *)w_part;
    double *tmax = (double *)w_tile, *tmin = tmax + ntile_fin;
    double *dscratch = tmin + ntile_fin;       // one double: max diagonal
    unsigned char *mask = (unsigned char *)w_mask;
    CdState *st = (CdState *)w_state;

    // largest ERI diagonal (for the default tie window / PSD tolerance)
    double *diag = part + (size_t)std::max<int64_t>(max_split, 1) * npad;
    if (dense)
        hipLaunchKernelGGL(dense_diag_kernel, dim3(nb), dim3(256), 0, ctx->stream, npairs, V, ldv,
                           diag);
    else
        hipLaunchKernelGGL(eri_diag_kernel, dim3(nb), dim3(256), 0, ctx->stream, npairs, pt, diag);
    CDS_LAUNCHED(ctx);
    hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(CD_SEL_BLOCK), 0, ctx->stream, npairs,
                       diag, dscratch);
    CDS_LAUNCHED(ctx);
    void *hp;
    CDS_CALL(cds_pinned(ctx, 256, &hp));
    CDS_HIP(ctx, hipMemcpyAsync(hp, dscratch, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const double vmax = *(double *)hp;
    if (tau < 0) tau = 1e-10 * vmax;
    if (psd_tol < 0) psd_tol = 1e3 * DBL_EPSILON * vmax;

    CdsTimer tall;
    CDS_CALL(cds_timer_start(ctx, &tall));
    CDS_HIP(ctx, hipMemsetAsync(mask, 0, (size_t)npairs, ctx->stream));
    CdState st0 = {};
    st0.k = nvec_in;
    *(CdState *)hp = st0;
    CDS_HIP(ctx, hipMemcpyAsync(st, hp, sizeof(CdState), hipMemcpyHostToDevice, ctx->stream));
    if (nvec_in == 0) {
        CDS_HIP(ctx, hipMemcpyAsync(D, diag, (size_t)npairs * 8, hipMemcpyDeviceToDevice, ctx->stream));
    } else {
        hipLaunchKernelGGL(mark_pivots_kernel, dim3((unsigned)cds_ceil_div(nvec_in, 256)), dim3(256),
                           0, ctx->stream, nvec_in, piv, npairs, mask);
        CDS_LAUNCHED(ctx);
    }
    hipLaunchKernelGGL(tile_stats_kernel, dim3((unsigned)ntile_fin), dim3(CD_FIN_TILE), 0, ctx->stream,
                       npairs, D, mask, tmax, tmin);
    CDS_LAUNCHED(ctx);
    hipLaunchKernelGGL(cd_select_kernel, dim3(1), dim3(CD_SEL_BLOCK), 0, ctx->stream, 0, ntile_fin,
                       tmax, tmin, D, mask, npairs, delta, tau, psd_tol, max_vec, st, piv);
    CDS_LAUNCHED(ctx);

    int64_t k = nvec_in;
    int batch = 8;
    CdState hs = {};
    for (;;) {
        CDS_HIP(ctx, hipMemcpyAsync(hp, st, sizeof(CdState), hipMemcpyDeviceToHost, ctx->stream));
        CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
        hs = *(CdState *)hp;
        if (hs.done) break;
        if (hs.k != k)
            return cds_fail(ctx, CDS_EDEVICE, "CD state out of step (device k=%lld host k=%lld)",
                            (long long)hs.k, (long long)k);
        for (int b = 0; b < batch && k < max_vec; ++b, ++k) {
            const int nsplit = (int)cds_ceil_div(k, CD_JCHUNK);
            if (nsplit > 0) {
                CdsTimer tk;
                if (ctx->kernel_timing) CDS_CALL(cds_timer_start(ctx, &tk));
                dim3 grid((unsigned)ntile_part, (unsigned)nsplit);
                if (vw == 2)
                    hipLaunchKernelGGL(cd_partial_kernel<2>, grid, dim3(CD_BLOCK), 0, ctx->stream, L,
                                       ldl, npairs, npad, st, part);
                else
                    hipLaunchKernelGGL(cd_partial_kernel<1>, grid, dim3(CD_BLOCK), 0, ctx->stream, L,
                                       ldl, npairs, npad, st, part);
                CDS_LAUNCHED(ctx);
                if (ctx->kernel_timing) CDS_CALL(cds_timer_stop(ctx, &tk, &ctx->stats.t_cd_kernel_ms));
            }
            if (dense)
                hipLaunchKernelGGL(cd_finalize_kernel<true>, dim3((unsigned)ntile_fin),
                                   dim3(CD_FIN_TILE), 0, ctx->stream, pt, V, ldv, L, ldl, npairs, npad,
                                   part, nsplit, D, mask, st, tmax, tmin);
            else
                hipLaunchKernelGGL(cd_finalize_kernel<false>, dim3((unsigned)ntile_fin),
                                   dim3(CD_FIN_TILE), 0, ctx->stream, pt, V, ldv, L, ldl, npairs, npad,
                                   part, nsplit, D, mask, st, tmax, tmin);
            CDS_LAUNCHED(ctx);
            hipLaunchKernelGGL(cd_select_kernel, dim3(1), dim3(CD_SEL_BLOCK), 0, ctx->stream, 1,
                               ntile_fin, tmax, tmin, D, mask, npairs, delta, tau, psd_tol, max_vec,
                               st, piv);
            CDS_LAUNCHED(ctx);
        }
        if (batch < 64) batch *= 2;
    }
    CDS_CALL(cds_timer_stop(ctx, &tall, &ctx->stats.t_cd_ms));
    // algorithmic bytes of the steps made: L read (8 npairs k) + column/D/pair traffic
    for (int64_t j = nvec_in; j < hs.k; ++j)
        ctx->stats.bytes_cd += 8.0 * (double)npairs * (double)j + 64.0 * (double)npairs;
    ctx->stats.n_cd_steps += hs.k - nvec_in;
    CDS_CALL(cds_timers_flush(ctx));
    *h_nvec = hs.k;
    *h_dmax = hs.dmax;
    *h_status = hs.status;
    if (hs.status == CDS_CD_CAP)
        return cds_fail(ctx, CDS_ECAP, "max_vec=%lld reached with D_max=%g > delta=%g",
                        (long long)max_vec, hs.dmax, delta);
    if (hs.status == CDS_CD_NOTPSD)
        return cds_fail(ctx, CDS_ENOTPSD, "residual diagonal below -%g", psd_tol);
    return CDS_OK;
}

}  // namespace

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

int cds_set_kernel_timing(cds_ctx *ctx, int32_t on)
{
    if (!ctx) return CDS_EINVAL;
    ctx->kernel_timing = on != 0;
    return CDS_OK;
}

}  // extern "C"
