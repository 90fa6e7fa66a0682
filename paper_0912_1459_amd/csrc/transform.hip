// AO->MO transform of the Cholesky vectors, Eq. (transformation) of the paper:
//   B^K_pq = sum_{mu,nu} C_mu,p L^K_mu,nu C_nu,q
// for the blocks the self-energy reads: B^K[sel, :] and B^K[virt, occ].
//
// Per batch of vectors K (all on the GPU):
//   1. unpack   packed L^K -> dense symmetric Lu[K][mu][nu] (k padded to Np)
//   2. GEMM     T[x][K][mu] = sum_nu CX[x][nu] Lu[K][mu][nu]      (batched over K)
//      with x = the occupied orbitals, then the selected orbitals that are not occupied
//      (an occupied target's row of T is its occupied row)
//   3. GEMM     W[a][(i,K)] = sum_mu Ct[nocc+a][mu] T[i][K][mu]     (virt x occ, one product)
//      GEMM     W[r][(s,K)] = sum_mu Ct[r][mu] T[x_s][K][mu]        (all x sel, one product
//                                                                   per run of consecutive x_s)
//   4. copy     W -> B[row][K] (K contiguous: each (row, batch) segment is contiguous in W),
//      converting to the output format (double, float, or bf16 hi/lo planes).
// Working precision of steps 1-3: FP64 for CDS_PREC_FP64, FP32 for FP32, and
// split bf16 (3-term products, FP32 accumulation) for BF16X3.
#include "cds_internal.h"

#include <array>
#include <type_traits>
#include <vector>

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

// Ct[p][mu] = C[mu][p]; CX rows: occupied 0..nocc-1 then the MOs ext[0..nx-nocc); k padded to np_
__global__ void coef_kernel(const double *__restrict__ C, int nbf, int nmo, int nocc, int nx,
                            const int32_t *__restrict__ ext, int np_, void *Ct, void *CX, int prec,
                            int64_t planeCt, int64_t planeCX)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nrow = nmo + nx;
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
        p = x < nocc ? x : ext[x - nocc];
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


// W (working type) -> out[row*ldk + k0 + kb] in the output format, one thread per (row, kb).
// Rows [0, nvo) = (a, i) go to Bvo from W[(a*nocc + i)*nkb + kb]; rows nvo + s*nmo + r go to
// Bsel from W[nvo*nkb + r*nsel*nkb + s*nkb + kb].  Reads and writes run along kb.
template <typename W>
__global__ __launch_bounds__(256) void copy_out_kernel(const W *__restrict__ Wb, int64_t nvo, int nmo, int nsel,
                                                       int nkb, int64_t k0, void *Bvo, void *Bsel, int64_t ldk,
                                                       int prec, int64_t plane_vo, int64_t plane_sel)
{
    const int64_t nrows = nvo + (int64_t)nsel * nmo;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * nkb) return;
    const int64_t row = t / nkb;
    const int kb = (int)(t - row * nkb);
    if (row < nvo) {
        put(Bvo, prec, row * ldk + k0 + kb, plane_vo, (double)Wb[t]);
    } else {
        const int64_t rs = row - nvo;
        const int sidx = (int)(rs / nmo), r = (int)(rs - (int64_t)sidx * nmo);
        const double v = (double)Wb[nvo * nkb + ((int64_t)r * nsel + sidx) * nkb + kb];
        put(Bsel, prec, rs * ldk + k0 + kb, plane_sel, v);
    }
}

// The same copy from the single product W[r][x * nkb + kb] = sum_mu Ct[r][mu] T[x][kb][mu] over
// every MO r and every row x of T: B_vo[a][i] from row nocc + a, column i; B_sel[s][r] from row r,
// column xs[s].
__global__ __launch_bounds__(256) void copy_out_all_kernel(const double *__restrict__ Wb, int64_t nvo, int nmo,
                                                           int nocc, int nx, int nsel, const int32_t *__restrict__ xs,
                                                           int nkb, int64_t k0, void *Bvo, void *Bsel, int64_t ldk,
                                                           int prec, int64_t plane_vo, int64_t plane_sel)
{
    const int64_t nrows = nvo + (int64_t)nsel * nmo;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * nkb) return;
    const int64_t row = t / nkb;
    const int kb = (int)(t - row * nkb);
    if (row < nvo) {
        const int64_t a = row / nocc, i = row - a * nocc;
        put(Bvo, prec, row * ldk + k0 + kb, plane_vo, Wb[((nocc + a) * nx + i) * nkb + kb]);
    } else {
        const int64_t rs = row - nvo;
        const int sidx = (int)(rs / nmo), r = (int)(rs - (int64_t)sidx * nmo);
        put(Bsel, prec, rs * ldk + k0 + kb, plane_sel, Wb[((int64_t)r * nx + xs[sidx]) * nkb + kb]);
    }
}

__global__ void zero_pad_kernel(int64_t nrows, int64_t ldk, int64_t nvec, int64_t kend, void *B, int prec,
                                int64_t plane)
{
    int64_t npad = kend - nvec;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * npad) return;
    int64_t r = t / npad, c = nvec + (t - r * npad);
    put(B, prec, r * ldk + c, plane, 0.0);
}

size_t wsize(int prec) { return prec == CDS_PREC_FP64 ? 8 : (prec == CDS_PREC_FP32 ? 4 : 4); }

// One transform: sizes, working precision, workspace and the launches of each stage.
struct TrPlan {
    int prec, wp, nbf, nmo, nocc, nsel, nvirt, nx, np_, kbatch;
    int64_t nvo, nselr, nrows, ldl, ldk;
    const double *L, *C;
    void *Bsel, *Bvo;
    std::vector<int32_t> ext;                 // CX rows past the occupied ones: these MOs
    std::vector<int> xs;                      // row of T (x) of each selected orbital
    std::vector<std::array<int, 3>> runs;     // (s0, count, x0): consecutive s with consecutive x
    unsigned char *Ct, *CX;
    int32_t *dext, *dxs;
    bool comb;                                // one product over all MOs and all rows of T
    void *wlu, *wt, *wb;
    float *Tf;
    __bf16 *Ts;
    int64_t planeCt, planeCX;
};

int tr_check(cds_ctx *ctx, int32_t prec, int32_t nbf, int64_t nvec, const double *L, int64_t ldl,
             const double *C, int32_t nmo, int32_t nocc, int32_t nsel, const int32_t *h_sel, int64_t ldk,
             void *Bsel, void *Bvo)
{
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
    return CDS_OK;
}

// sizes and workspace for batches of at most max(1, min(kb_cap, adaptive size)) vectors
// the buffers of one batch (unpacked L^K, T and its split planes, the products) from three slots
int tr_alloc_batch(cds_ctx *ctx, TrPlan &p, CdsSlot slu, CdsSlot st, CdsSlot sb)
{
    const size_t es = wsize(p.wp);
    const int64_t nLu = (int64_t)p.kbatch * p.nbf * p.np_;
    CDS_CALL(cds_ws(ctx, slu, (size_t)nLu * es, &p.wlu));
    const int64_t nT = (int64_t)p.kbatch * p.nx * p.np_;
    CDS_CALL(cds_ws(ctx, st, (size_t)nT * es * (p.wp == CDS_PREC_BF16X3 ? 2 : 1), &p.wt));
    const int64_t wrows = p.comb ? (int64_t)p.nmo * p.nx : p.nrows;
    CDS_CALL(cds_ws(ctx, sb, (size_t)p.kbatch * wrows * (p.wp == CDS_PREC_FP64 ? 8 : 4), &p.wb));
    // T: working float output, and (bf16) its two planes after it
    p.Tf = (float *)p.wt;
    p.Ts = (__bf16 *)((unsigned char *)p.wt + (size_t)nT * 4);
    return CDS_OK;
}

int tr_alloc(cds_ctx *ctx, TrPlan &p, int32_t prec, int32_t nbf, const double *L, int64_t ldl, const double *C,
             int32_t nmo, int32_t nocc, int32_t nsel, const int32_t *h_sel, int64_t ldk, void *Bsel, void *Bvo,
             int64_t kb_cap)
{
    p.prec = prec;
    p.nbf = nbf;
    p.nmo = nmo;
    p.nocc = nocc;
    p.nsel = nsel;
    p.nvirt = nmo - nocc;
    // an occupied target reads the occupied row of T; other targets get a row of their own
    p.ext.clear();
    p.xs.assign(nsel, 0);
    for (int s = 0; s < nsel; ++s) {
        const int q = h_sel[s];
        if (q < nocc) {
            p.xs[s] = q;
            continue;
        }
        int j = 0;
        while (j < (int)p.ext.size() && p.ext[j] != q) ++j;
        if (j == (int)p.ext.size()) p.ext.push_back(q);
        p.xs[s] = nocc + j;
    }
    p.runs.clear();
    for (int s = 0; s < nsel; ++s) {
        if (!p.runs.empty() && p.runs.back()[0] + p.runs.back()[1] == s &&
            p.runs.back()[2] + p.runs.back()[1] == p.xs[s])
            ++p.runs.back()[1];
        else
            p.runs.push_back({s, 1, p.xs[s]});
    }
    p.nx = nocc + (int)p.ext.size();
    p.np_ = (int)(cds_ceil_div(nbf, 64) * 64);
    p.nvo = (int64_t)p.nvirt * nocc;
    p.nselr = (int64_t)nsel * nmo;
    p.nrows = p.nvo + p.nselr;
    p.L = L;
    p.ldl = ldl;
    p.C = C;
    p.ldk = ldk;
    p.Bsel = Bsel;
    p.Bvo = Bvo;
    // working precision of the GEMMs; the output is rounded to `prec` in the last pass
    p.wp = ctx->transform_fp64 ? CDS_PREC_FP64 : prec;
    // FP64: one product Ct^T T over every MO and every row of T (one launch that fills the chip)
    // when it computes at most 15 % more than the two blocks need
    p.comb = p.wp == CDS_PREC_FP64 && (int64_t)nmo * p.nx * 100 <= p.nrows * 115;
    const size_t es = wsize(p.wp);
    // batch: enough 128 x 128 tiles of the virtual-occupied product per launch to fill the
    // chip (that product has one tile group of nvirt x nocc per vector)
    const int64_t tiles_vo = cds_ceil_div(p.nvirt, 128) * cds_ceil_div(nocc, 128);
    int64_t kb_want = std::max<int64_t>(KBATCH_MIN, cds_ceil_div(KBATCH_WG, tiles_vo));
    kb_want = std::min<int64_t>(kb_want, std::max<int64_t>(1, (int64_t)(KBATCH_BYTES / ((size_t)nbf * p.np_ * es))));
    p.kbatch = (int)std::max<int64_t>(1, std::min<int64_t>(kb_want, kb_cap));

    // workspace: Ct + CX (+ sel list), Lu batch, T batch (+ split copy), Bk batch
    void *wcx;
    const int64_t nCt = (int64_t)nmo * p.np_, nCX = (int64_t)p.nx * p.np_;
    CDS_CALL(cds_ws(ctx, WS_TR_CX, (size_t)(nCt + nCX) * es + 256 + nsel * 8, &wcx));
    CDS_CALL(tr_alloc_batch(ctx, p, WS_TR_UNPACK, WS_TR_T, WS_TR_B));
    p.Ct = (unsigned char *)wcx;
    p.CX = p.Ct + nCt * es;
    p.dext = (int32_t *)(p.CX + ((nCX * es + 255) / 256) * 256);
    p.dxs = p.dext + nsel;
    // for bf16 the hi and lo planes of Ct / CX take 2 x 2 bytes = es per element: each lo
    // plane follows its hi plane inside the same byte range
    p.planeCt = nCt;
    p.planeCX = nCX;
    return CDS_OK;
}

// the K padding [nbf, np_) of a batch buffer set's T reads as 0 (the first GEMM writes columns
// < nbf only)
int tr_zero_tpad(cds_ctx *ctx, const TrPlan &p)
{
    if (p.np_ > p.nbf) {
        const size_t tes0 = (p.wp == CDS_PREC_FP64) ? 8 : (p.wp == CDS_PREC_FP32 ? 4 : 2);
        unsigned char *tb = (p.wp == CDS_PREC_BF16X3) ? (unsigned char *)p.Ts : (unsigned char *)p.wt;
        const int64_t trows = (int64_t)p.kbatch * p.nx * (p.wp == CDS_PREC_BF16X3 ? 2 : 1);   // both planes
        const int64_t nz = trows * (int64_t)((p.np_ - p.nbf) * tes0 / 2);
        hipLaunchKernelGGL(zero_cols_kernel, dim3((unsigned)cds_ceil_div(nz, 256)), dim3(256), 0, ctx->stream, tb,
                           trows, (int64_t)p.np_ * (int64_t)tes0, (int)(p.nbf * tes0), (int)(p.np_ * tes0));
        CDS_LAUNCHED(ctx);
    }
    return CDS_OK;
}

// coefficient copies and the zero K padding of T (once per transform)
int tr_setup(cds_ctx *ctx, const TrPlan &p)
{
    if (!p.ext.empty())
        CDS_HIP(ctx, hipMemcpyAsync(p.dext, p.ext.data(), p.ext.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    if (p.comb)
        CDS_HIP(ctx, hipMemcpyAsync(p.dxs, p.xs.data(), p.xs.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    {
        int64_t n = (int64_t)(p.nmo + p.nx) * p.np_;
        hipLaunchKernelGGL(coef_kernel, dim3((unsigned)cds_ceil_div(n, 256)), dim3(256), 0, ctx->stream,
                           p.C, p.nbf, p.nmo, p.nocc, p.nx, p.dext, p.np_, (void *)p.Ct, (void *)p.CX, p.wp,
                           p.planeCt, p.planeCX);
        CDS_LAUNCHED(ctx);
    }
    return tr_zero_tpad(ctx, p);
}

// zero entries K in [nvec, kend) of both output blocks, kend <= ldk
int tr_pad(cds_ctx *ctx, const TrPlan &p, int64_t nvec, int64_t kend)
{
    if (kend > nvec) {
        int64_t n1 = p.nvo * (kend - nvec), n2 = p.nselr * (kend - nvec);
        hipLaunchKernelGGL(zero_pad_kernel, dim3((unsigned)cds_ceil_div(n1, 256)), dim3(256), 0, ctx->stream, p.nvo,
                           p.ldk, nvec, kend, p.Bvo, p.prec, p.nvo * p.ldk);
        hipLaunchKernelGGL(zero_pad_kernel, dim3((unsigned)cds_ceil_div(n2, 256)), dim3(256), 0, ctx->stream,
                           p.nselr, p.ldk, nvec, kend, p.Bsel, p.prec, p.nselr * p.ldk);
        CDS_LAUNCHED(ctx);
    }
    return CDS_OK;
}

// vectors [k0, k0 + nkb), nkb <= kbatch: unpack, three GEMMs, transposed output
int tr_batch(cds_ctx *ctx, const TrPlan &p, int64_t k0, int nkb)
{
    const int np_ = p.np_, nx = p.nx, nocc = p.nocc, nmo = p.nmo, nsel = p.nsel, nbf = p.nbf;
    {
        const int nb = np_ / 32;
        hipLaunchKernelGGL(unpack_blocks_kernel, dim3((unsigned)(nb * (nb + 1) / 2), (unsigned)nkb), dim3(256), 0,
                           ctx->stream, p.L, p.ldl, k0, nbf, np_, p.wlu, p.wp, (int64_t)nkb * nbf * np_);
        CDS_LAUNCHED(ctx);
    }
    const int64_t planeLu = (int64_t)nkb * nbf * np_;
    const int gprec = p.wp;
    // T[x][kb][mu] = sum_nu CX[x][nu] Lu[kb][mu][nu]   (row (x, kb) of T at (x*nkb + kb)*np_)
    GemmDesc g1 = {};
    g1.M = nx; g1.N = nbf; g1.K = np_; g1.batch = nkb;
    g1.A = p.CX; g1.sAm = np_; g1.sAk = 1; g1.sAb = 0;
    g1.B = p.wlu; g1.sBn = np_; g1.sBk = 1; g1.sBb = (int64_t)nbf * np_;
    void *Tout = (p.wp == CDS_PREC_FP64) ? p.wt : (void *)p.Tf;
    g1.C = Tout; g1.sCm = (int64_t)nkb * np_; g1.sCn = 1; g1.sCb = np_;
    g1.alpha = 1.0; g1.beta = 0.0;
    g1.big = 1;
    if (p.wp == CDS_PREC_BF16X3) {
        // T straight into its two bf16 planes (the split of the FP32 result)
        g1.C = p.Ts;
        g1.Clo = p.Ts + (int64_t)nkb * nx * np_;
        CDS_CALL(cds_gemm_ex(ctx, gprec, g1, (const __bf16 *)p.CX + p.planeCX, (const __bf16 *)p.wlu + planeLu));
    } else {
        CDS_CALL(cds_gemm_ex(ctx, gprec, g1, nullptr, nullptr));
    }
    const unsigned char *Tin = (const unsigned char *)((p.wp == CDS_PREC_BF16X3) ? (const void *)p.Ts : Tout);
    const int64_t planeT = (int64_t)nkb * nx * np_;
    const size_t tes = (p.wp == CDS_PREC_FP64) ? 8 : (p.wp == CDS_PREC_FP32 ? 4 : 2);
    const size_t wes = (p.wp == CDS_PREC_FP64) ? 8 : 4;
    if (p.comb) {
        // W[r][x*nkb + kb] = sum_mu Ct[r][mu] T[x][kb][mu] for every MO r and row x of T: both
        // blocks from one launch (each entry the same sum as in the two products below)
        GemmDesc gc = {};
        gc.M = nmo; gc.N = (int64_t)nx * nkb; gc.K = np_; gc.batch = 1;
        gc.A = p.Ct; gc.sAm = np_; gc.sAk = 1;
        gc.B = Tout; gc.sBn = np_; gc.sBk = 1;
        gc.C = p.wb; gc.sCm = (int64_t)nx * nkb; gc.sCn = 1;
        gc.alpha = 1.0; gc.beta = 0.0;
        gc.big = nmo >= 512 ? 2 : 1;
        CDS_CALL(cds_gemm_ex(ctx, gprec, gc, nullptr, nullptr));
        const int64_t nel = p.nrows * nkb;
        hipLaunchKernelGGL(copy_out_all_kernel, dim3((unsigned)cds_ceil_div(nel, 256)), dim3(256), 0, ctx->stream,
                           (const double *)p.wb, p.nvo, nmo, nocc, nx, nsel, (const int32_t *)p.dxs, nkb, k0, p.Bvo,
                           p.Bsel, p.ldk, p.prec, p.nvo * p.ldk, p.nselr * p.ldk);
        CDS_LAUNCHED(ctx);
        return CDS_OK;
    }
    // the 256 x 256 split-bf16 tiles are chosen from the per-vector shapes only, so that a
    // vector's blocks do not depend on the batching
    // W[a][i*nkb + kb] = sum_mu Ct[nocc+a][mu] T[i][kb][mu]
    GemmDesc g2 = {};
    g2.M = p.nvirt; g2.N = (int64_t)nocc * nkb; g2.K = np_; g2.batch = 1;
    g2.A = p.Ct + (size_t)nocc * np_ * tes; g2.sAm = np_; g2.sAk = 1;
    g2.B = Tin; g2.sBn = np_; g2.sBk = 1;
    g2.C = p.wb; g2.sCm = (int64_t)nocc * nkb; g2.sCn = 1;
    g2.alpha = 1.0; g2.beta = 0.0;
    g2.big = p.nvirt >= 512 ? 2 : 1;
    if (p.wp == CDS_PREC_BF16X3)
        CDS_CALL(cds_gemm_ex(ctx, gprec, g2, (const __bf16 *)p.Ct + p.planeCt + (int64_t)nocc * np_,
                             p.Ts + planeT));
    else
        CDS_CALL(cds_gemm_ex(ctx, gprec, g2, nullptr, nullptr));
    // W[nvo*nkb + r*nsel*nkb + s*nkb + kb] = sum_mu Ct[r][mu] T[x_s][kb][mu], one product per run
    for (const auto &run : p.runs) {
        const int s0 = run[0], cnt = run[1], x0 = run[2];
        GemmDesc g3 = {};
        g3.M = nmo; g3.N = (int64_t)cnt * nkb; g3.K = np_; g3.batch = 1;
        g3.A = p.Ct; g3.sAm = np_; g3.sAk = 1;
        g3.B = Tin + (size_t)x0 * nkb * np_ * tes; g3.sBn = np_; g3.sBk = 1;
        g3.C = (unsigned char *)p.wb + ((size_t)p.nvo * nkb + (size_t)s0 * nkb) * wes;
        g3.sCm = (int64_t)nsel * nkb; g3.sCn = 1;
        g3.alpha = 1.0; g3.beta = 0.0;
        g3.big = nmo >= 512 ? 2 : 1;
        if (p.wp == CDS_PREC_BF16X3)
            CDS_CALL(cds_gemm_ex(ctx, gprec, g3, (const __bf16 *)p.Ct + p.planeCt,
                                 p.Ts + planeT + (int64_t)x0 * nkb * np_));
        else
            CDS_CALL(cds_gemm_ex(ctx, gprec, g3, nullptr, nullptr));
    }
    const int64_t nel = p.nrows * nkb;
    const dim3 cg((unsigned)cds_ceil_div(nel, 256));
    if (p.wp == CDS_PREC_FP64)
        hipLaunchKernelGGL(copy_out_kernel<double>, cg, dim3(256), 0, ctx->stream, (const double *)p.wb, p.nvo, nmo,
                           nsel, nkb, k0, p.Bvo, p.Bsel, p.ldk, p.prec, p.nvo * p.ldk, p.nselr * p.ldk);
    else
        hipLaunchKernelGGL(copy_out_kernel<float>, cg, dim3(256), 0, ctx->stream, (const float *)p.wb, p.nvo, nmo,
                           nsel, nkb, k0, p.Bvo, p.Bsel, p.ldk, p.prec, p.nvo * p.ldk, p.nselr * p.ldk);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}

// vectors [k0, k1) in batches of at most kbatch
int tr_range(cds_ctx *ctx, const TrPlan &p, int64_t k0, int64_t k1)
{
    for (; k0 < k1; k0 += p.kbatch) CDS_CALL(tr_batch(ctx, p, k0, (int)std::min<int64_t>(p.kbatch, k1 - k0)));
    return CDS_OK;
}

// launches of the calling thread go to stream s until the scope ends
struct StreamScope {
    cds_ctx *c;
    hipStream_t old;
    StreamScope(cds_ctx *c_, hipStream_t s) : c(c_), old(c_->stream) { c->stream = s; }
    ~StreamScope() { c->stream = old; }
};

// Transform of the decomposition's vectors while it runs, on the side stream.  With look-ahead
// blocks, once OVL_PIECE vectors are known to be final and not yet queued, the next block's
// pass is followed (through an event) by a piece of OVL_PIECE of them, so the piece runs in
// the block's single-workgroup and row-update kernels, where most of the device is idle,
// rather than beside the passes (on c60's decomposition, pieces of 112 measured better than 64,
// 80, 96 and 104; on the path with the wider candidate set, whose blocks are longer and fewer,
// pieces of 56 leave less of the transform after it; batches queued as soon as vectors are
// final slowed the decomposition).  Without blocks (per-step launches), the vectors made since
// the last batch go at each read of the state, at least OVL_MIN of them.
constexpr int64_t OVL_MIN = 128;
constexpr int64_t OVL_PIECE = 112;
constexpr int64_t OVL_PIECE_WIDE = 56;
constexpr int64_t OVL_CAP = 512;    // batch size the workspace holds

struct Overlap {
    cds_ctx *ctx;
    TrPlan *p;
    int64_t kdone = 0;    // vectors queued on the side stream
    int64_t kfinal = 0;   // vectors known to be final
    bool started = false;
    bool gated = false;   // pieces follow the blocks (the decomposition runs look-ahead blocks)
};

int overlap_queue(Overlap &o, int64_t k1)
{
    StreamScope sc(o.ctx, o.ctx->stream2);
    if (!o.started) {
        CDS_CALL(tr_setup(o.ctx, *o.p));
        CDS_HIP(o.ctx, hipEventRecord(o.ctx->trset, o.ctx->stream));
        o.started = true;
    }
    CDS_CALL(tr_range(o.ctx, *o.p, o.kdone, k1));
    o.kdone = k1;
    return CDS_OK;
}

int overlap_committed(void *user, int64_t k)
{
    Overlap &o = *(Overlap *)user;
    o.kfinal = k;
    if (o.gated || k - o.kdone < OVL_MIN) return CDS_OK;
    return overlap_queue(o, k);
}

// a piece of the final vectors, started on the side stream once the block's pass is done
int overlap_block(void *user, int wide)
{
    Overlap &o = *(Overlap *)user;
    o.gated = true;
    const int64_t piece = wide ? OVL_PIECE_WIDE : OVL_PIECE;
    if (o.kfinal - o.kdone < piece) return CDS_OK;
    CDS_HIP(o.ctx, hipEventRecord(o.ctx->gate, o.ctx->stream));
    CDS_HIP(o.ctx, hipStreamWaitEvent(o.ctx->stream2, o.ctx->gate, 0));
    return overlap_queue(o, std::min<int64_t>(o.kfinal, o.kdone + piece));
}

}  // namespace

extern "C" int cds_transform(cds_ctx *ctx, int32_t prec, int32_t nbf, int64_t nvec, const double *L,
                             int64_t ldl, const double *C, int32_t nmo, int32_t nocc, int32_t nsel,
                             const int32_t *h_sel, int64_t ldk, void *Bsel, void *Bvo)
{
    CDS_CALL(cds_enter(ctx));
    CDS_CALL(tr_check(ctx, prec, nbf, nvec, L, ldl, C, nmo, nocc, nsel, h_sel, ldk, Bsel, Bvo));
    CdsTimer tm;
    CDS_CALL(cds_timer_start(ctx, &tm));
    TrPlan p;
    CDS_CALL(tr_alloc(ctx, p, prec, nbf, L, ldl, C, nmo, nocc, nsel, h_sel, ldk, Bsel, Bvo, nvec));
    CDS_CALL(tr_setup(ctx, p));
    CDS_CALL(tr_pad(ctx, p, nvec, p.ldk));
    CDS_CALL(tr_range(ctx, p, 0, nvec));
    CDS_CALL(cds_timer_stop(ctx, &tm, &ctx->stats.t_transform_ms));
    return CDS_OK;
}

extern "C" int cds_cholesky_transform_sgauss(cds_ctx *ctx, int32_t nbf, const double *centres, const double *alpha,
                                             double delta, double tau, double psd_tol, int64_t max_vec, double *L,
                                             int64_t ldl, int64_t *piv, double *D, int32_t prec, const double *C,
                                             int32_t nmo, int32_t nocc, int32_t nsel, const int32_t *h_sel,
                                             int64_t ldk, void *Bsel, void *Bvo, int64_t *h_nvec, double *h_dmax,
                                             int32_t *h_status)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, nbf >= 1 && centres && alpha, "need nbf >= 1, centres and alpha");
    CDS_REQUIRE(ctx, max_vec >= 1, "max_vec must be >= 1");
    CDS_CALL(tr_check(ctx, prec, nbf, max_vec, L, ldl, C, nmo, nocc, nsel, h_sel, ldk, Bsel, Bvo));
    if (!ctx->stream2) {
        CDS_HIP(ctx, hipStreamCreateWithFlags(&ctx->stream2, hipStreamNonBlocking));
        CDS_HIP(ctx, hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming));
        CDS_HIP(ctx, hipEventCreateWithFlags(&ctx->gate, hipEventDisableTiming));
        CDS_HIP(ctx, hipEventCreateWithFlags(&ctx->trset, hipEventDisableTiming));
    }
    // everything the side stream uses is allocated before any work is queued
    TrPlan p;
    CDS_CALL(tr_alloc(ctx, p, prec, nbf, L, ldl, C, nmo, nocc, nsel, h_sel, ldk, Bsel, Bvo,
                      std::min<int64_t>(OVL_CAP, max_vec)));
    TrPlan p2 = p;                  // the last vectors' batch buffers (the caller's stream)
    CDS_CALL(tr_alloc_batch(ctx, p2, WS_TR_UNPACK2, WS_TR_T2, WS_TR_B2));
    // the side stream starts after everything queued before this call
    CDS_HIP(ctx, hipEventRecord(ctx->join, ctx->stream));
    CDS_HIP(ctx, hipStreamWaitEvent(ctx->stream2, ctx->join, 0));
    Overlap ov;
    ov.ctx = ctx;
    ov.p = &p;
    CdHook hook = {overlap_committed, overlap_block, &ov};
    const int rc = cds_cholesky_hooked(ctx, nbf, centres, alpha, delta, tau, psd_tol, max_vec, L, ldl, piv, D,
                                       h_nvec, h_dmax, h_status, &hook);
    int rt = CDS_OK;
    // transform time exposed after the decomposition: from its end to the join
    CdsTimer tm;
    const bool timed = rc == CDS_OK || rc == CDS_ECAP || rc == CDS_ENOTPSD;
    if (timed) rt = cds_timer_start(ctx, &tm);
    if (rt == CDS_OK && timed) {
        const std::string err = ctx->err;
        if (ov.started && *h_nvec > ov.kdone) {
            // the rest of the vectors on the caller's stream, with a second set of batch
            // buffers, beside the batches the side stream has not finished (they write other
            // entries K of the blocks); the coefficient copies are the side stream's
            rt = tr_zero_tpad(ctx, p2);
            if (rt == CDS_OK && hipStreamWaitEvent(ctx->stream, ctx->trset, 0) != hipSuccess)
                rt = cds_fail(ctx, CDS_EDEVICE, "hipStreamWaitEvent failed");
            if (rt == CDS_OK) rt = tr_range(ctx, p2, ov.kdone, *h_nvec);
        } else {
            // no batch queued yet: everything on the side stream
            StreamScope sc(ctx, ctx->stream2);
            if (!ov.started) rt = tr_setup(ctx, p);
            if (rt == CDS_OK && *h_nvec > ov.kdone) rt = tr_range(ctx, p, ov.kdone, *h_nvec);
        }
        // ldk was sized for max_vec: only the entries up to the next multiple of 64, the last any
        // consumer of the blocks reads, are cleared
        if (rt == CDS_OK) rt = tr_pad(ctx, p, *h_nvec, std::min<int64_t>(p.ldk, cds_ceil_div(*h_nvec, 64) * 64));
        if (rt == CDS_OK) ctx->err = err;
    }
    // the caller's stream waits for the side stream
    CDS_HIP(ctx, hipEventRecord(ctx->join, ctx->stream2));
    CDS_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->join, 0));
    if (rt == CDS_OK && timed) {
        const std::string err = ctx->err;
        rt = cds_timer_stop(ctx, &tm, &ctx->stats.t_transform_ms);
        if (rt == CDS_OK) ctx->err = err;
    }
    return rt != CDS_OK ? rt : rc;
}

namespace {

// Rows [r0, r1) of a row-major array of 16-byte chunks move from ld16 chunks per row to ldn16,
// keeping the first ldn16 of each.  The caller sizes the batch so that every destination lies
// below every source of the batch (r1 ldn16 <= r0 ld16) and only over rows already moved, so
// its rows move in one launch in any order.
__global__ __launch_bounds__(256) void restride_kernel(uint4 *B, int64_t r0, int64_t r1, int64_t ld16,
                                                       int64_t ldn16)
{
    const int64_t n = (r1 - r0) * ldn16;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
        const int64_t r = r0 + q / ldn16, c = q % ldn16;
        B[r * ldn16 + c] = B[r * ld16 + c];
    }
}

}  // namespace

extern "C" int cds_restride_blocks(cds_ctx *ctx, int32_t prec, int64_t rows, int64_t ldk, int64_t ldk_new, void *B)
{
    CDS_CALL(cds_enter(ctx));
    CDS_REQUIRE(ctx, prec == CDS_PREC_FP64 || prec == CDS_PREC_FP32 || prec == CDS_PREC_BF16X3, "unknown prec %d",
                (int)prec);
    CDS_REQUIRE(ctx, rows >= 0, "rows must be >= 0");
    CDS_REQUIRE(ctx, ldk_new >= 1 && 2 * ldk_new <= ldk, "need 1 <= ldk_new <= ldk / 2 (ldk %lld, ldk_new %lld)",
                (long long)ldk, (long long)ldk_new);
    const int64_t es = prec == CDS_PREC_FP64 ? 8 : prec == CDS_PREC_FP32 ? 4 : 2;
    CDS_REQUIRE(ctx, (ldk * es) % 16 == 0 && (ldk_new * es) % 16 == 0,
                "rows of ldk and ldk_new entries must be multiples of 16 bytes");
    if (rows == 0) return CDS_OK;
    CDS_REQUIRE(ctx, B && ((uintptr_t)B & 15) == 0, "B must be a 16-byte aligned device pointer");
    // the two bf16 planes are one array of 2 rows rows
    const int64_t R = prec == CDS_PREC_BF16X3 ? 2 * rows : rows;
    const int64_t ld16 = ldk * es / 16, ldn16 = ldk_new * es / 16;
    CdsTimer tm;
    CDS_CALL(cds_timer_start(ctx, &tm));
    // row 0 stays; a batch starting at row a can end at a ldk / ldk_new >= 2 a
    for (int64_t a = 1; a < R;) {
        const int64_t b = std::min<int64_t>(R, a * ldk / ldk_new);
        const int64_t nb = std::min<int64_t>(cds_ceil_div((b - a) * ldn16, 256), 8192);
        hipLaunchKernelGGL(restride_kernel, dim3((unsigned)nb), dim3(256), 0, ctx->stream, (uint4 *)B, a, b, ld16,
                           ldn16);
        CDS_LAUNCHED(ctx);
        a = b;
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
