// Second-order self-energy and quasi-particle solves (Sec. II.B of the paper):
//   Eq. (SE)   Sigma_qq(w) = sum_{a,i,j} (2(qi|aj) - (qj|ai)) (qi|aj) / (w + e_a - e_i - e_j)
//                          + sum_{i,a,b} (2(qa|ib) - (qb|ia)) (qa|ib) / (w + e_i - e_a - e_b)
//   Eq. (aomo) (pq|rs) = sum_K B^K_pq B^K_rs
//   Eqs. (qpapp), (iter), (ps), (NR): Newton solve of w = e_q + Sigma_qq(w).
//
// Contraction: one MFMA GEMM per chunk of targets,
//   G[s][r][a*nocc + j] = sum_K Bsel[s][r][K] Bvo[a][j][K] = (q r | a j),
// so (qi|aj) = G[s][i][a*nocc+j] and (qa|ib) = (qa|bi) = G[s][nocc+a][b*nocc+i].
// Epilogue kernels then form the numerators, divide by the denominators and
// reduce deterministically (per-block partials, fixed-order final sums):
//   part A (2h1p): one block per (s, a), elements (i, j) of X^a
//   part B (2p1h): one block per (s, a), elements (b, i) of row a of the Y^i
// Residue mode stores the pair-symmetrised numerators
//   R = U_uv + U_vu = 2 (g_uv^2 + g_vu^2 - g_uv g_vu)  (u < v),  R = g_uu^2
// once; each later Newton step is one pass over R.
#include "cds_internal.h"

#include <cmath>
#include <cstring>
#include <vector>

int cds_gemm_ex(cds_ctx *ctx, int prec, const GemmDesc &d, const void *Alo, const void *Blo);

namespace {

constexpr int EP_NT = 256;
constexpr int TMAX = 16;

enum EpMode { EP_SIGMA = 0, EP_RESIDUE = 1, EP_GRAD = 2 };

struct EpArgs {
    const void *G;          // integrals of this chunk: [sc][nmo][nvo] (double or float)
    int nmo, nocc, nvirt, nsc;
    int64_t nvo;
    const double *eps;      // device orbital energies
    const double *omega;    // [sc][T] trial energies (chunk-relative)
    int T;
    double *part;           // partial sums [sc][nblk][T][2]
    int nblkA, nblkB;       // blocks per target in part A / part B
    void *R;                // residues [sc][nres] (RESIDUE mode)
    int64_t nres, offB;     // residues per target; start of part B within a target
    // gradient mode
    const double *gscale;   // [sc] omega_bar * P per target
    void *W;                // weights dSigma/dG scaled, same layout as G
    double *epsA;           // [sc][nvirt][nocc + 1] part A energy partials
    double *epsB;           // [sc][nvirt][nocc + 1] part B energy partials
};

template <typename GT>
__device__ __forceinline__ double ld(const void *p, int64_t i) { return (double)((const GT *)p)[i]; }

template <int NTH>
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NTH / 64; ++k) s += sh[k];   // fixed order
    __syncthreads();
    if (threadIdx.x == 0) sh[0] = s;
    __syncthreads();
    return sh[0];
}

// reduce per-thread sums acc[t][0..1] over the block and store to part
template <int NTH>
__device__ __forceinline__ void flush_partials(double (*acc)[2], int T, double *dst, double *sh)
{
    for (int t = 0; t < T; ++t)
        for (int c = 0; c < 2; ++c) {
            double v = block_sum<NTH>(acc[t][c], sh);
            if (threadIdx.x == 0) dst[t * 2 + c] = v;
        }
}

// ---------------------------------------------------------------------------
// Pair-symmetrised epilogues.  Both exchange partners of Eq. (SE) share one
// denominator (d is symmetric in i, j and in a, b), so each unordered pair
// contributes R/d with R = U_uv + U_vu = 2(g_uv^2 + g_vu^2 - g_uv g_vu) (u != v)
// or R = g_uu^2.  SIGMA mode accumulates sum_t R/d_t and -R/d_t^2 for TT trial
// energies; RESIDUE mode stores R once (residue layout: part A [a][j(j+1)/2+i],
// part B [a][(b-a)*nocc + i], b >= a).
// ---------------------------------------------------------------------------

// part A (2h1p), block (a = blockIdx.x, s = blockIdx.y): X^a[i][j] = G[s][i][a*nocc + j].
// 32 x 32 tile pairs (IB <= JB) of X^a and its transpose are staged in LDS so both
// partners are read with coalesced loads.  d = w + e_a - e_i - e_j.
template <typename GT, int MODE, int TT>
__global__ __launch_bounds__(EP_NT) void pair_a_kernel(EpArgs e)
{
    __shared__ double sh[EP_NT / 64];
    __shared__ double eo[1024];
    __shared__ double t1[32][33], t2[32][33];
    const int a = blockIdx.x, s = blockIdx.y, nocc = e.nocc;
    for (int i = threadIdx.x; i < nocc; i += EP_NT) eo[i] = e.eps[i];
    const double ea = e.eps[nocc + a];
    const int64_t gbase = (int64_t)s * e.nmo * e.nvo + (int64_t)a * nocc;   // + i*nvo + j
    double acc[TT > 0 ? TT : 1][2];
    double w[TT > 0 ? TT : 1];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
        acc[t][0] = acc[t][1] = 0.0;
        w[t] = e.omega[s * e.T + (t < e.T ? t : e.T - 1)];
    }
    const int nb = (nocc + 31) / 32;
    for (int IB = 0; IB < nb; ++IB)
        for (int JB = IB; JB < nb; ++JB) {
            // both tiles: every load in flight before the LDS stores (a loop of loads would
            // wait on each)
            constexpr int QN = 1024 / EP_NT;
            double v1[QN], v2[QN];
#pragma unroll
            for (int u = 0; u < QN; ++u) {
                const int q = threadIdx.x + EP_NT * u;
                const int r = q >> 5, c = q & 31;
                const int i1 = IB * 32 + r, j1 = JB * 32 + c;   // t1[r][c] = X[i1][j1]
                const int i2 = JB * 32 + r, j2 = IB * 32 + c;   // t2[r][c] = X[i2][j2]
                v1[u] = (i1 < nocc && j1 < nocc) ? ld<GT>(e.G, gbase + (int64_t)i1 * e.nvo + j1) : 0.0;
                v2[u] = (i2 < nocc && j2 < nocc) ? ld<GT>(e.G, gbase + (int64_t)i2 * e.nvo + j2) : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < QN; ++u) {
                const int q = threadIdx.x + EP_NT * u;
                t1[q >> 5][q & 31] = v1[u];
                t2[q >> 5][q & 31] = v2[u];
            }
            __syncthreads();
            // element (i, j) = (IB*32 + ci, JB*32 + cj), ci fastest over the threads: the
            // residues of consecutive i are consecutive in the packed layout
            for (int q = threadIdx.x; q < 1024; q += EP_NT) {
                const int cj = q >> 5, ci = q & 31;
                const int i = IB * 32 + ci, j = JB * 32 + cj;
                if (i >= nocc || j >= nocc || (IB == JB && ci > cj)) continue;
                const double x = t1[ci][cj], xt = t2[cj][ci];
                const double R = (i == j) ? x * x : 2.0 * (x * x + xt * xt - x * xt);
                if constexpr (MODE == EP_SIGMA) {
                    const double dd = ea - eo[i] - eo[j];
#pragma unroll
                    for (int t = 0; t < TT; ++t) {
                        const double id = 1.0 / (w[t] + dd);
                        const double ri = R * id;
                        acc[t][0] += ri;
                        acc[t][1] -= ri * id;
                    }
                } else {
                    const int64_t pp = (int64_t)j * (j + 1) / 2 + i;
                    ((GT *)e.R)[(int64_t)s * e.nres + (int64_t)a * (nocc * (nocc + 1) / 2) + pp] = (GT)R;
                }
            }
        }
    if constexpr (MODE == EP_SIGMA) {
        double *dst = e.part + (((int64_t)s * (e.nblkA + e.nblkB) + a) * e.T) * 2;
#pragma unroll
        for (int t = 0; t < TT; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double v = block_sum<EP_NT>(acc[t][c], sh);
                if (threadIdx.x == 0 && t < e.T) dst[t * 2 + c] = v;
            }
    }
}

// part B (2p1h): y_{i;ab} = G[s][nocc+a][b*nocc+i], partner y_{i;ba} = G[s][nocc+b][a*nocc+i];
// d = w + e_i - e_a - e_b.  Block blk handles a = blk and a = nvirt-1-blk over b >= a
// (equal work per block); both partners are contiguous in i.
template <typename GT, int MODE, int TT>
__global__ __launch_bounds__(EP_NT) void pair_b_kernel(EpArgs e)
{
    __shared__ double sh[EP_NT / 64];
    __shared__ double eo[1024];
    const int s = blockIdx.y, nocc = e.nocc, nvirt = e.nvirt, blk = blockIdx.x;
    for (int i = threadIdx.x; i < nocc; i += EP_NT) eo[i] = e.eps[i];
    __syncthreads();
    const double *ev = e.eps + nocc;
    const int64_t gs0 = (int64_t)s * e.nmo * e.nvo;
    double acc[TT > 0 ? TT : 1][2];
    double w[TT > 0 ? TT : 1];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
        acc[t][0] = acc[t][1] = 0.0;
        w[t] = e.omega[s * e.T + (t < e.T ? t : e.T - 1)];
    }
    for (int pass = 0; pass < 2; ++pass) {
        const int a = pass == 0 ? blk : nvirt - 1 - blk;
        if (pass == 1 && a == blk) break;
        const double ea = ev[a];
        const int64_t base_a = gs0 + (int64_t)(nocc + a) * e.nvo;
        const int64_t nitem = (int64_t)(nvirt - a) * nocc;
        const int64_t roff = (int64_t)s * e.nres + e.offB +
                             (int64_t)nocc * ((int64_t)a * nvirt - (int64_t)a * (a - 1) / 2);
        // four items per thread and round: their loads are all in flight before the first use
        constexpr int UB = 4;
        for (int64_t q0 = threadIdx.x; q0 < nitem; q0 += (int64_t)UB * EP_NT) {
            double yv[UB], ytv[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int64_t q = q0 + (int64_t)u * EP_NT;
                const int64_t qc = q < nitem ? q : nitem - 1;
                const int bo = (int)(qc / nocc), i = (int)(qc - (int64_t)bo * nocc);
                const int b = a + bo;
                yv[u] = ld<GT>(e.G, base_a + (int64_t)b * nocc + i);
                ytv[u] = ld<GT>(e.G, gs0 + (int64_t)(nocc + b) * e.nvo + (int64_t)a * nocc + i);
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int64_t q = q0 + (int64_t)u * EP_NT;
                if (q >= nitem) break;
                const int bo = (int)(q / nocc), i = (int)(q - (int64_t)bo * nocc);
                const int b = a + bo;
                const double y = yv[u], yt = ytv[u];
                const double R = (bo == 0) ? y * y : 2.0 * (y * y + yt * yt - y * yt);
                if constexpr (MODE == EP_SIGMA) {
                    const double dd = eo[i] - ea - ev[b];
#pragma unroll
                    for (int t = 0; t < TT; ++t) {
                        const double id = 1.0 / (w[t] + dd);
                        const double ri = R * id;
                        acc[t][0] += ri;
                        acc[t][1] -= ri * id;
                    }
                } else {
                    ((GT *)e.R)[roff + q] = (GT)R;
                }
            }
        }
    }
    if constexpr (MODE == EP_SIGMA) {
        double *dst = e.part + (((int64_t)s * (e.nblkA + e.nblkB) + e.nblkA + blk) * e.T) * 2;
#pragma unroll
        for (int t = 0; t < TT; ++t)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double v = block_sum<EP_NT>(acc[t][c], sh);
                if (threadIdx.x == 0 && t < e.T) dst[t * 2 + c] = v;
            }
    }
}

// Gradient weights, part A (block per (a, s)): W = gscale (4 x_ij - 2 x_ji) / d for every
// ordered element; thread i owns e-bar_i (row sums), the block sums e-bar_a.
template <typename GT>
__global__ __launch_bounds__(EP_NT) void grad_a_kernel(EpArgs e)
{
    __shared__ double sh[EP_NT / 64];
    __shared__ double eo[1024];
    const int a = blockIdx.x, s = blockIdx.y, nocc = e.nocc;
    for (int i = threadIdx.x; i < nocc; i += EP_NT) eo[i] = e.eps[i];
    __syncthreads();
    const double ea = e.eps[nocc + a];
    const int64_t gbase = (int64_t)s * e.nmo * e.nvo + (int64_t)a * nocc;
    const double w0 = e.omega[s];
    const double gs = e.gscale[s];
    double sa = 0.0;
    for (int i = threadIdx.x; i < nocc; i += EP_NT) {
        double si = 0.0;
        // JU columns at a time, their loads in flight before the first use (same order of terms)
        constexpr int JU = 4;
        for (int j0 = 0; j0 < nocc; j0 += JU) {
            double xv[JU], xtv[JU];
#pragma unroll
            for (int u = 0; u < JU; ++u) {
                const int j = j0 + u < nocc ? j0 + u : nocc - 1;
                xv[u] = ld<GT>(e.G, gbase + (int64_t)i * e.nvo + j);
                xtv[u] = ld<GT>(e.G, gbase + (int64_t)j * e.nvo + i);
            }
#pragma unroll
            for (int u = 0; u < JU; ++u) {
                const int j = j0 + u;
                if (j >= nocc) break;
                const double x = xv[u], xt = xtv[u];
                double d = w0 + ea - eo[i] - eo[j];
                double uu = (2.0 * x - xt) * x, ut = (2.0 * xt - x) * xt;
                double id = 1.0 / d;
                ((GT *)e.W)[gbase + (int64_t)i * e.nvo + j] = (GT)(gs * (4.0 * x - 2.0 * xt) * id);
                si += (uu + ut) * id * id;     // d symmetric in (i, j)
                sa -= uu * id * id;
            }
        }
        e.epsA[((int64_t)s * e.nvirt + a) * (nocc + 1) + i] = gs * si;
    }
    sa = block_sum<EP_NT>(sa, sh);
    if (threadIdx.x == 0) e.epsA[((int64_t)s * e.nvirt + a) * (nocc + 1) + nocc] = gs * sa;
}

// Gradient weights, part B (block per (a, s)) over all (b, i); per-i sums are owned by
// fixed threads (i = tid % nocc) and combined in a fixed order.
template <typename GT>
__global__ __launch_bounds__(EP_NT) void grad_b_kernel(EpArgs e)
{
    __shared__ double sh[EP_NT / 64];
    __shared__ double eo[1024];
    __shared__ double acc_i[1024];
    const int s = blockIdx.y, nocc = e.nocc, nvirt = e.nvirt, a = blockIdx.x;
    for (int i = threadIdx.x; i < nocc; i += EP_NT) {
        eo[i] = e.eps[i];
        acc_i[i] = 0.0;
    }
    __syncthreads();
    const double *ev = e.eps + nocc;
    const int64_t gs0 = (int64_t)s * e.nmo * e.nvo;
    const double ea = ev[a];
    const int64_t base_a = gs0 + (int64_t)(nocc + a) * e.nvo;
    const double gsc = e.gscale[s];
    const double w0 = e.omega[s];
    const int per = EP_NT / nocc > 0 ? EP_NT / nocc : 1;
    const int i0 = threadIdx.x % nocc, bsub = threadIdx.x / nocc;
    double sa = 0.0, si = 0.0;
    if (bsub < per) {
        for (int i = i0; i < nocc; i += (nocc > EP_NT ? EP_NT : nocc)) {
            double sii = 0.0;
            for (int b = bsub; b < nvirt; b += per) {
                double y = ld<GT>(e.G, base_a + (int64_t)b * nocc + i);
                double yt = ld<GT>(e.G, gs0 + (int64_t)(nocc + b) * e.nvo + (int64_t)a * nocc + i);
                double d = w0 + eo[i] - ea - ev[b];
                double id = 1.0 / d;
                double u = (2.0 * y - yt) * y, ut = (2.0 * yt - y) * yt;
                ((GT *)e.W)[base_a + (int64_t)b * nocc + i] = (GT)(gsc * (4.0 * y - 2.0 * yt) * id);
                sii -= u * id * id;           // role i of element (a, b, i)
                sa += (u + ut) * id * id;     // roles a of (a,b,i) and b of (b,a,i)
            }
            si = sii;
            if (nocc > EP_NT) e.epsB[((int64_t)s * nvirt + a) * (nocc + 1) + i] = gsc * si;
        }
    }
    if (nocc <= EP_NT) {
        for (int k = 0; k < per; ++k) {
            __syncthreads();
            if (bsub == k && bsub < per) acc_i[i0] += si;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nocc; i += EP_NT)
            e.epsB[((int64_t)s * nvirt + a) * (nocc + 1) + i] = gsc * acc_i[i];
    }
    sa = block_sum<EP_NT>(sa, sh);
    if (threadIdx.x == 0) e.epsB[((int64_t)s * nvirt + a) * (nocc + 1) + nocc] = gsc * sa;
}

// Newton sweep over stored residues: Sigma(w) = sum R / (w - pole), one energy per target.
// Blocks [0, nvirt) sum part A of a = blockIdx.x; blocks [nvirt, nvirt + ceil(nvirt/2)) the
// balanced part-B pairs, in the residue layout written above.
template <typename RT>
__global__ __launch_bounds__(EP_NT) void sweep_kernel(EpArgs e, const int *__restrict__ active)
{
    __shared__ double sh[EP_NT / 64];
    __shared__ double eo[1024];
    const int s = active[blockIdx.y], nocc = e.nocc, nvirt = e.nvirt;
    for (int i = threadIdx.x; i < nocc; i += EP_NT) eo[i] = e.eps[i];
    __syncthreads();
    const double *ev = e.eps + nocc;
    const double w = e.omega[s];
    const RT *R = (const RT *)e.R + (int64_t)s * e.nres;
    constexpr int SU = 4;
    double s0 = 0.0, s1 = 0.0;
    const int blk = blockIdx.x;
    if (blk < nvirt) {
        const int a = blk;
        const int npair = nocc * (nocc + 1) / 2;
        const RT *Ra = R + (int64_t)a * npair;
        const double ea = ev[a];
        // SU residues per thread and round, loaded before the first use (same order of terms)
        for (int p0 = threadIdx.x; p0 < npair; p0 += SU * EP_NT) {
            double rv[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int p = p0 + u * EP_NT;
                rv[u] = (double)Ra[p < npair ? p : npair - 1];
            }
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int p = p0 + u * EP_NT;
                if (p >= npair) break;
                // p = j(j+1)/2 + i, i <= j (float square root, then exact integer correction)
                int j = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
                if (j * (j + 1) / 2 > p) --j;
                if ((j + 1) * (j + 2) / 2 <= p) ++j;
                const int i = p - j * (j + 1) / 2;
                const double id = 1.0 / (w + ea - eo[i] - eo[j]);
                const double ri = rv[u] * id;
                s0 += ri;
                s1 -= ri * id;
            }
        }
    } else {
        const int pb = blk - nvirt;
        for (int pass = 0; pass < 2; ++pass) {
            const int a = pass == 0 ? pb : nvirt - 1 - pb;
            if (pass == 1 && a == pb) break;
            const int64_t nitem = (int64_t)(nvirt - a) * nocc;
            const RT *Rb = R + e.offB + (int64_t)nocc * ((int64_t)a * nvirt - (int64_t)a * (a - 1) / 2);
            const double ea = ev[a];
            for (int64_t q0 = threadIdx.x; q0 < nitem; q0 += (int64_t)SU * EP_NT) {
                double rv[SU];
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int64_t q = q0 + (int64_t)u * EP_NT;
                    rv[u] = (double)Rb[q < nitem ? q : nitem - 1];
                }
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    const int64_t q = q0 + (int64_t)u * EP_NT;
                    if (q >= nitem) break;
                    const int bo = (int)(q / nocc), i = (int)(q - (int64_t)bo * nocc);
                    const double id = 1.0 / (w + eo[i] - ea - ev[a + bo]);
                    const double ri = rv[u] * id;
                    s0 += ri;
                    s1 -= ri * id;
                }
            }
        }
    }
    s0 = block_sum<EP_NT>(s0, sh);
    s1 = block_sum<EP_NT>(s1, sh);
    if (threadIdx.x == 0) {
        double *dst = e.part + ((int64_t)blockIdx.y * (e.nblkA + e.nblkB) + blk) * 2;
        dst[0] = s0;
        dst[1] = s1;
    }
}

// Sum of part[s][b][t][c] over the blocks b of one output (s, t, c), by one workgroup of 256
// threads in a fixed order: thread j adds blocks j, j + 256, ... in turn, the 64 lanes of a wave
// are combined by a butterfly and the four waves in order (deterministic, and the same in both
// kernels below).
__device__ __forceinline__ double reduce_blocks(const double *__restrict__ part, int s, int tc, int nblk, int T)
{
    __shared__ double sh[4];
    double acc = 0.0;
    constexpr int U = 4;
    for (int b0 = threadIdx.x; b0 < nblk; b0 += U * 256) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * 256;
            v[u] = b < nblk ? part[((int64_t)s * nblk + b) * T * 2 + tc] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (b0 + u * 256 < nblk) acc += v[u];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// out[s][t][c]: one workgroup per output (grid nsc * T * 2)
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double *__restrict__ part, int nsc, int nblk,
                                                              int T, double *__restrict__ out)
{
    const int idx = blockIdx.x, s = idx / (T * 2), tc = idx - s * T * 2;
    const double v = reduce_blocks(part, s, tc, nblk, T);
    if (threadIdx.x == 0) out[idx] = v;
}

// Newton's iteration on the device (residue mode, fused path): the solve's state per target
// (energy, its own orbital energy, pole strength, status, steps) and the list of targets still
// iterating, so that several iterations go without a round trip to the host.
struct NewtonDev {
    double *om, *qe, *pole;
    int *act, *status, *iters, *sel;
    int *cnt;                               // [0] targets still iterating, [1] last step made
};

__global__ void newton_init_kernel(int nsel, const double *__restrict__ eps, int have_w0, NewtonDev d)
{
    for (int s = threadIdx.x; s < nsel; s += blockDim.x) {
        const double q = eps[d.sel[s]];
        d.qe[s] = q;
        if (!have_w0) d.om[s] = q;
        d.act[s] = s;
        d.status[s] = -1;
        d.iters[s] = 0;
        d.pole[s] = __builtin_nan("");
    }
    if (threadIdx.x == 0) {
        d.cnt[0] = nsel;
        d.cnt[1] = 0;
    }
}

// Sigma and Sigma' of the k-th target still iterating (out[2k], out[2k+1]), T = 1; rows past
// the count return
__global__ __launch_bounds__(256) void reduce_active_kernel(const double *__restrict__ part, int nblk,
                                                            const int *__restrict__ cnt, double *__restrict__ out)
{
    if ((int)blockIdx.x >= 2 * cnt[0]) return;
    const int idx = blockIdx.x, s = idx / 2, tc = idx - s * 2;
    const double v = reduce_blocks(part, s, tc, nblk, 1);
    if (threadIdx.x == 0) out[idx] = v;
}

// step `it` of Eq. (NR) for every target still iterating, in list order, with the operations of
// the host loop: P = 1 / (1 - Sigma'), w' = w + (e_q + Sigma - w) P, converged at |w' - w| <= conv
__global__ void newton_step_kernel(const double *__restrict__ out, double conv, int it, NewtonDev d)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0) return;
    const int n = d.cnt[0];
    if (n == 0) return;
    d.cnt[1] = it;
    int m = 0;
    for (int k = 0; k < n; ++k) {
        const int s = d.act[k];
        const double sg = out[2 * k], ds = out[2 * k + 1];
        d.iters[s] = it;
        if (!isfinite(sg) || !isfinite(ds)) {            // a denominator vanished
            d.status[s] = CDS_QP_NONFINITE;
            continue;
        }
        const double P = 1.0 / (1.0 - ds);
        const double w = d.om[s];
        const double wn = w + (d.qe[s] + sg - w) * P;
        d.pole[s] = P;
        d.om[s] = wn;
        if (!isfinite(wn) || !isfinite(P)) {
            d.status[s] = CDS_QP_NONFINITE;
            continue;
        }
        if (fabs(wn - w) <= conv) {
            d.status[s] = CDS_QP_CONVERGED;
            continue;
        }
        d.act[m++] = s;
    }
    d.cnt[0] = m;
}

// sig[s][t] and dsig[s][t] (the two components written apart); same order as above
__global__ __launch_bounds__(256) void reduce_split_kernel(const double *__restrict__ part, int nsc, int nblk, int T,
                                                           double *__restrict__ sig, double *__restrict__ dsig)
{
    const int idx = blockIdx.x, s = idx / (T * 2), tc = idx - s * T * 2;
    const double v = reduce_blocks(part, s, tc, nblk, T);
    if (threadIdx.x == 0) (tc & 1 ? dsig : sig)[s * T + (tc >> 1)] = v;
}

struct SigmaShape {
    int prec;
    int64_t nvec, ldk;
    int nmo, nocc, nvirt, nsel;
    int64_t nvo, nselr;
};

int check_shape(cds_ctx *ctx, const SigmaShape &sh, const int32_t *h_sel, const void *Bsel,
                const void *Bvo, const double *eps)
{
    CDS_REQUIRE(ctx, sh.prec == CDS_PREC_FP64 || sh.prec == CDS_PREC_FP32 || sh.prec == CDS_PREC_BF16X3,
                "unknown precision %d", sh.prec);
    CDS_REQUIRE(ctx, sh.nmo >= 2 && sh.nocc >= 1 && sh.nocc < sh.nmo, "need 1 <= nocc < nmo");
    CDS_REQUIRE(ctx, sh.nocc <= 1024, "nocc must be <= 1024");
    CDS_REQUIRE(ctx, sh.nsel >= 1 && sh.nsel <= 65535 && h_sel, "need 1 <= nsel and h_sel");
    CDS_REQUIRE(ctx, sh.nvec >= 1 && sh.ldk >= sh.nvec, "need nvec >= 1, ldk >= nvec");
    CDS_REQUIRE(ctx, sh.prec != CDS_PREC_BF16X3 || sh.ldk % 64 == 0, "BF16X3 needs ldk % 64 == 0");
    CDS_REQUIRE(ctx, Bsel && Bvo && eps, "NULL pointer");
    for (int s = 0; s < sh.nsel; ++s)
        CDS_REQUIRE(ctx, h_sel[s] >= 0 && h_sel[s] < sh.nmo, "h_sel[%d] out of range", s);
    return CDS_OK;
}

// targets per chunk so that G stays below ~4 GiB (and at most the context's target chunk)
int chunk_targets(const cds_ctx *ctx, const SigmaShape &sh)
{
    size_t es = sh.prec == CDS_PREC_FP64 ? 8 : 4;
    size_t per = (size_t)sh.nmo * sh.nvo * es;
    size_t lim = (size_t)4 << 30;
    int n = (int)std::max<size_t>(1, lim / std::max<size_t>(per, 1));
    if (ctx->target_chunk > 0) n = std::min(n, ctx->target_chunk);
    return std::min(n, sh.nsel);
}

// split-bf16 lo planes of the blocks (NULL for the other precisions)
void lo_planes(const SigmaShape &sh, const void *Bsel, const void *Bvo, const void **Slo, const void **Vlo)
{
    *Slo = *Vlo = nullptr;
    if (sh.prec == CDS_PREC_BF16X3) {
        *Slo = (const __bf16 *)Bsel + sh.nselr * sh.ldk;
        *Vlo = (const __bf16 *)Bvo + sh.nvo * sh.ldk;
    }
}

// targets per launch of the fused kernel (all unless the context caps it)
int fused_chunk(const cds_ctx *ctx, const SigmaShape &sh)
{
    return ctx->target_chunk > 0 ? std::min(ctx->target_chunk, sh.nsel) : sh.nsel;
}

__global__ void iota_kernel(int *__restrict__ p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

// device list 0 .. nsel-1 of target slots (slot s0 + j of a launch is entry s0 + j)
int target_slots(cds_ctx *ctx, int nsel, int **d_tsel)
{
    void *p;
    CDS_CALL(cds_ws(ctx, WS_SG_TSEL, (size_t)nsel * 4, &p));
    hipLaunchKernelGGL(iota_kernel, dim3((unsigned)cds_ceil_div(nsel, 256)), dim3(256), 0, ctx->stream, (int *)p, nsel);
    CDS_LAUNCHED(ctx);
    *d_tsel = (int *)p;
    return CDS_OK;
}

// G for targets [s0, s0+nsc)
int contract_chunk(cds_ctx *ctx, const SigmaShape &sh, const void *Bsel, const void *Bvo, int s0,
                   int nsc, void *G)
{
    const size_t es = sh.prec == CDS_PREC_FP64 ? 8 : (sh.prec == CDS_PREC_FP32 ? 4 : 2);
    GemmDesc d = {};
    d.M = (int64_t)nsc * sh.nmo;
    d.N = sh.nvo;
    // entries K in [nvec, this) are zero: the sum stops at the first multiple of 64 past nvec
    d.K = std::min<int64_t>(sh.ldk, cds_ceil_div(sh.nvec, 64) * 64);
    d.batch = 1;
    d.A = (const unsigned char *)Bsel + (size_t)s0 * sh.nmo * sh.ldk * es;
    d.sAm = sh.ldk;
    d.sAk = 1;
    d.B = Bvo;
    d.sBn = sh.ldk;
    d.sBk = 1;
    d.C = G;
    d.sCm = sh.nvo;
    d.sCn = 1;
    d.alpha = 1.0;
    d.beta = 0.0;
    const void *Alo = nullptr, *Blo = nullptr;
    if (sh.prec == CDS_PREC_BF16X3) {
        Alo = (const __bf16 *)Bsel + sh.nselr * sh.ldk + (int64_t)s0 * sh.nmo * sh.ldk;
        Blo = (const __bf16 *)Bvo + sh.nvo * sh.ldk;
    }
    CdsTimer t;
    CDS_CALL(cds_timer_start(ctx, &t));
    CDS_CALL(cds_gemm_ex(ctx, sh.prec, d, Alo, Blo));
    CDS_CALL(cds_timer_stop(ctx, &t, &ctx->stats.t_contract_ms));
    ctx->stats.flops_contract += 2.0 * (double)sh.nvec * nsc * sh.nmo * (double)sh.nvo;
    ctx->stats.n_contract += 1;
    return CDS_OK;
}

template <typename GT, int MODE, int TT>
void launch_pairs(cds_ctx *ctx, const SigmaShape &sh, EpArgs &e)
{
    dim3 ga((unsigned)sh.nvirt, (unsigned)e.nsc);
    dim3 gb((unsigned)((sh.nvirt + 1) / 2), (unsigned)e.nsc);
    hipLaunchKernelGGL((pair_a_kernel<GT, MODE, TT>), ga, dim3(EP_NT), 0, ctx->stream, e);
    hipLaunchKernelGGL((pair_b_kernel<GT, MODE, TT>), gb, dim3(EP_NT), 0, ctx->stream, e);
}

template <typename GT, int MODE>
int launch_epilogue_t(cds_ctx *ctx, const SigmaShape &sh, EpArgs &e)
{
    if (MODE == EP_RESIDUE) launch_pairs<GT, EP_RESIDUE, 0>(ctx, sh, e);
    else if (e.T <= 1) launch_pairs<GT, EP_SIGMA, 1>(ctx, sh, e);
    else if (e.T <= 2) launch_pairs<GT, EP_SIGMA, 2>(ctx, sh, e);
    else if (e.T <= 4) launch_pairs<GT, EP_SIGMA, 4>(ctx, sh, e);
    else if (e.T <= 8) launch_pairs<GT, EP_SIGMA, 8>(ctx, sh, e);
    else launch_pairs<GT, EP_SIGMA, 16>(ctx, sh, e);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}

template <int MODE>
int launch_epilogue(cds_ctx *ctx, const SigmaShape &sh, EpArgs &e, bool fp64)
{
    if (MODE == EP_GRAD) {
        dim3 g((unsigned)sh.nvirt, (unsigned)e.nsc);
        if (fp64) {
            hipLaunchKernelGGL(grad_a_kernel<double>, g, dim3(EP_NT), 0, ctx->stream, e);
            hipLaunchKernelGGL(grad_b_kernel<double>, g, dim3(EP_NT), 0, ctx->stream, e);
        } else {
            hipLaunchKernelGGL(grad_a_kernel<float>, g, dim3(EP_NT), 0, ctx->stream, e);
            hipLaunchKernelGGL(grad_b_kernel<float>, g, dim3(EP_NT), 0, ctx->stream, e);
        }
        CDS_LAUNCHED(ctx);
        return CDS_OK;
    }
    return fp64 ? launch_epilogue_t<double, MODE>(ctx, sh, e) : launch_epilogue_t<float, MODE>(ctx, sh, e);
}

// Sigma, Sigma' for all targets at T energies each (device omega [nsel][T]) -> host out [nsel][T][2]
int eval_sigma(cds_ctx *ctx, const SigmaShape &sh, const void *Bsel, const void *Bvo,
               const double *eps, const double *d_omega, int T, double *h_out)
{
    const void *Slo, *Vlo;
    lo_planes(sh, Bsel, Bvo, &Slo, &Vlo);
    CdsFusedPlan fp;
    if (cds_fused_plan(sh.prec, sh.nvec, sh.ldk, sh.nmo, sh.nocc, Bsel, Bvo, Slo, Vlo, &fp)) {
        // integrals formed and reduced over the denominators in one kernel (never stored)
        const int csz = fused_chunk(ctx, sh);
        int *tsel;
        CDS_CALL(target_slots(ctx, sh.nsel, &tsel));
        void *part, *out;
        CDS_CALL(cds_ws(ctx, WS_SG_PART, (size_t)csz * fp.tpt * T * 2 * 8, &part));
        CDS_CALL(cds_ws(ctx, WS_SG_OUT, (size_t)sh.nsel * T * 2 * 8, &out));
        for (int s0 = 0; s0 < sh.nsel; s0 += csz) {
            const int nsc = std::min(csz, sh.nsel - s0);
            CdsTimer t;
            CDS_CALL(cds_timer_start(ctx, &t));
            CDS_CALL(cds_fused_sigma(ctx, sh.prec, fp, sh.ldk, sh.nmo, sh.nocc, nsc, tsel + s0, Bsel, Bvo, Slo, Vlo,
                                     eps, d_omega + (int64_t)s0 * T, T, (double *)part));
            CDS_CALL(cds_timer_stop(ctx, &t, &ctx->stats.t_contract_ms));
            ctx->stats.flops_contract += 2.0 * (double)sh.nvec * nsc * sh.nmo * (double)sh.nvo;
            ctx->stats.n_contract += 1;
            CdsTimer t2;
            CDS_CALL(cds_timer_start(ctx, &t2));
            const int nout = nsc * T * 2;
            hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)nout), dim3(256), 0,
                               ctx->stream, (const double *)part, nsc, (int)fp.tpt, T,
                               (double *)out + (int64_t)s0 * T * 2);
            CDS_LAUNCHED(ctx);
            CDS_CALL(cds_timer_stop(ctx, &t2, &ctx->stats.t_epilogue_ms));
        }
        CDS_HIP(ctx, hipMemcpyAsync(h_out, out, (size_t)sh.nsel * T * 2 * 8, hipMemcpyDeviceToHost, ctx->stream));
        CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
        return CDS_OK;
    }
    // blocks the fused kernel cannot read (K padding or alignment): integrals through HBM
    const int csz = chunk_targets(ctx, sh);
    const size_t es = sh.prec == CDS_PREC_FP64 ? 8 : 4;
    void *G, *part, *out;
    CDS_CALL(cds_ws(ctx, WS_SG_G, (size_t)csz * sh.nmo * sh.nvo * es, &G));
    const int nblk = sh.nvirt + (sh.nvirt + 1) / 2;
    CDS_CALL(cds_ws(ctx, WS_SG_PART, (size_t)csz * nblk * T * 2 * 8, &part));
    CDS_CALL(cds_ws(ctx, WS_SG_OUT, (size_t)sh.nsel * T * 2 * 8, &out));
    for (int s0 = 0; s0 < sh.nsel; s0 += csz) {
        const int nsc = std::min(csz, sh.nsel - s0);
        CDS_CALL(contract_chunk(ctx, sh, Bsel, Bvo, s0, nsc, G));
        EpArgs e = {};
        e.G = G;
        e.nmo = sh.nmo;
        e.nocc = sh.nocc;
        e.nvirt = sh.nvirt;
        e.nsc = nsc;
        e.nvo = sh.nvo;
        e.eps = eps;
        e.omega = d_omega + (int64_t)s0 * T;
        e.T = T;
        e.part = (double *)part;
        e.nblkA = sh.nvirt;
        e.nblkB = (sh.nvirt + 1) / 2;
        CdsTimer t;
        CDS_CALL(cds_timer_start(ctx, &t));
        CDS_CALL(launch_epilogue<EP_SIGMA>(ctx, sh, e, sh.prec == CDS_PREC_FP64));
        int n = nsc * T * 2;
        hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)n), dim3(256), 0,
                           ctx->stream, (const double *)part, nsc, nblk, T,
                           (double *)out + (int64_t)s0 * T * 2);
        CDS_LAUNCHED(ctx);
        CDS_CALL(cds_timer_stop(ctx, &t, &ctx->stats.t_epilogue_ms));
    }
    CDS_HIP(ctx, hipMemcpyAsync(h_out, out, (size_t)sh.nsel * T * 2 * 8, hipMemcpyDeviceToHost, ctx->stream));
    CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return CDS_OK;
}

}  // namespace

// shared with the adjoint translation unit
int cds_sigma_eval_internal(cds_ctx *ctx, int prec, int64_t nvec, int64_t ldk, int nmo, int nocc,
                            int nsel, const void *Bsel, const void *Bvo, const double *eps,
                            const double *h_omega, int T, double *h_out)
{
    SigmaShape sh = {prec, nvec, ldk, nmo, nocc, nmo - nocc, nsel,
                     (int64_t)(nmo - nocc) * nocc, (int64_t)nsel * nmo};
    void *om;
    CDS_CALL(cds_ws(ctx, WS_SG_OMEGA, (size_t)nsel * T * 8, &om));
    CDS_HIP(ctx, hipMemcpyAsync(om, h_omega, (size_t)nsel * T * 8, hipMemcpyHostToDevice, ctx->stream));
    return eval_sigma(ctx, sh, Bsel, Bvo, eps, (const double *)om, T, h_out);
}

// G for targets [s0, s0+nsc) into buffer G (adjoint)
int cds_contract_internal(cds_ctx *ctx, int prec, int64_t nvec, int64_t ldk, int nmo, int nocc,
                          int nsel, const void *Bsel, const void *Bvo, int s0, int nsc, void *G)
{
    SigmaShape sh = {prec, nvec, ldk, nmo, nocc, nmo - nocc, nsel,
                     (int64_t)(nmo - nocc) * nocc, (int64_t)nsel * nmo};
    return contract_chunk(ctx, sh, Bsel, Bvo, s0, nsc, G);
}

// Sigma and Sigma' of a chunk's targets at one energy each (device d_omega[nsc]) from its formed
// integrals G -> device d_out[nsc][2] (adjoint: the pole strengths at the converged energies)
int cds_sigma_from_g_internal(cds_ctx *ctx, int prec, int nmo, int nocc, int nsc, const void *G,
                              const double *eps, const double *d_omega, double *d_out)
{
    SigmaShape sh = {prec, 0, 0, nmo, nocc, nmo - nocc, nsc,
                     (int64_t)(nmo - nocc) * nocc, (int64_t)nsc * nmo};
    const int nblk = sh.nvirt + (sh.nvirt + 1) / 2;
    void *part;
    CDS_CALL(cds_ws(ctx, WS_SG_PART, (size_t)nsc * nblk * 2 * 8, &part));
    EpArgs e = {};
    e.G = G;
    e.nmo = nmo;
    e.nocc = nocc;
    e.nvirt = sh.nvirt;
    e.nsc = nsc;
    e.nvo = sh.nvo;
    e.eps = eps;
    e.omega = d_omega;
    e.T = 1;
    e.part = (double *)part;
    e.nblkA = sh.nvirt;
    e.nblkB = (sh.nvirt + 1) / 2;
    CDS_CALL(launch_epilogue<EP_SIGMA>(ctx, sh, e, prec == CDS_PREC_FP64));
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)(nsc * 2)), dim3(256), 0, ctx->stream,
                       (const double *)part, nsc, nblk, 1, d_out);
    CDS_LAUNCHED(ctx);
    return CDS_OK;
}

// gradient-weight epilogue for a chunk (adjoint)
int cds_grad_epilogue_internal(cds_ctx *ctx, int prec, int nmo, int nocc, int nsc, const void *G,
                               const double *eps, const double *d_omega, const double *d_gscale,
                               void *W, double *epsA, double *epsB)
{
    SigmaShape sh = {prec, 0, 0, nmo, nocc, nmo - nocc, nsc,
                     (int64_t)(nmo - nocc) * nocc, (int64_t)nsc * nmo};
    EpArgs e = {};
    e.G = G;
    e.nmo = nmo;
    e.nocc = nocc;
    e.nvirt = nmo - nocc;
    e.nsc = nsc;
    e.nvo = sh.nvo;
    e.eps = eps;
    e.omega = d_omega;
    e.T = 1;
    e.gscale = d_gscale;
    e.W = W;
    e.epsA = epsA;
    e.epsB = epsB;
    return launch_epilogue<EP_GRAD>(ctx, sh, e, prec == CDS_PREC_FP64);
}

extern "C" int cds_set_target_chunk(cds_ctx *ctx, int32_t n)
{
    if (!ctx) return CDS_EINVAL;
    if (n < 0 || n > 65535) return cds_fail(ctx, CDS_EINVAL, "target chunk must be in [0, 65535]");
    ctx->target_chunk = n;
    return CDS_OK;
}

extern "C" int cds_sigma2(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo,
                          int32_t nocc, int32_t nsel, const int32_t *h_sel, const void *Bsel,
                          const void *Bvo, const double *eps, int32_t T, const double *h_omega,
                          double *h_sigma, double *h_dsigma)
{
    CDS_CALL(cds_enter(ctx));
    SigmaShape sh = {prec, nvec, ldk, nmo, nocc, nmo - nocc, nsel,
                     (int64_t)(nmo - nocc) * nocc, (int64_t)nsel * nmo};
    CDS_CALL(check_shape(ctx, sh, h_sel, Bsel, Bvo, eps));
    CDS_REQUIRE(ctx, T >= 1 && T <= TMAX, "T must be in [1, %d]", TMAX);
    CDS_REQUIRE(ctx, h_omega && h_sigma && h_dsigma, "NULL host pointer");
    std::vector<double> out((size_t)nsel * T * 2);
    CDS_CALL(cds_sigma_eval_internal(ctx, prec, nvec, ldk, nmo, nocc, nsel, Bsel, Bvo, eps, h_omega, T,
                                     out.data()));
    for (int64_t k = 0; k < (int64_t)nsel * T; ++k) {
        h_sigma[k] = out[2 * k];
        h_dsigma[k] = out[2 * k + 1];
    }
    CDS_CALL(cds_timers_flush(ctx));
    return CDS_OK;
}

extern "C" int cds_qp_solve(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo,
                            int32_t nocc, int32_t nsel, const int32_t *h_sel, const void *Bsel,
                            const void *Bvo, const double *eps, const double *h_omega0, double conv,
                            int32_t max_iter, int32_t mode, double *h_omega, double *h_pole,
                            int32_t *h_iters, int32_t *h_status)
{
    CDS_CALL(cds_enter(ctx));
    SigmaShape sh = {prec, nvec, ldk, nmo, nocc, nmo - nocc, nsel,
                     (int64_t)(nmo - nocc) * nocc, (int64_t)nsel * nmo};
    CDS_CALL(check_shape(ctx, sh, h_sel, Bsel, Bvo, eps));
    CDS_REQUIRE(ctx, max_iter >= 1, "max_iter must be >= 1");
    CDS_REQUIRE(ctx, conv >= 0.0 && std::isfinite(conv), "conv must be finite and >= 0");
    CDS_REQUIRE(ctx, mode == CDS_QP_RECOMPUTE || mode == CDS_QP_RESIDUES, "unknown mode %d", mode);
    CDS_REQUIRE(ctx, h_omega && h_pole && h_iters && h_status, "NULL host pointer");

    CdsTimer tall;
    CDS_CALL(cds_timer_start(ctx, &tall));
    const void *Slo, *Vlo;
    lo_planes(sh, Bsel, Bvo, &Slo, &Vlo);
    CdsFusedPlan fp;
    const bool fused = cds_fused_plan(prec, nvec, ldk, nmo, nocc, Bsel, Bvo, Slo, Vlo, &fp);
    // residues from the fused contraction: the iteration runs on the device (no orbital energies
    // on the host, no round trip per step)
    const bool dev = mode == CDS_QP_RESIDUES && fused;
    std::vector<double> heps;
    if (!dev) {
        heps.resize(nmo);
        CDS_HIP(ctx, hipMemcpyAsync(heps.data(), eps, (size_t)nmo * 8, hipMemcpyDeviceToHost, ctx->stream));
        CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }

    std::vector<double> w(nsel), pole(nsel, NAN);
    std::vector<int> active, status(nsel, -1), iters(nsel, 0);
    if (!dev)
        for (int s = 0; s < nsel; ++s) w[s] = h_omega0 ? h_omega0[s] : heps[h_sel[s]];

    // residue mode: one contraction per target chunk, residues kept on the device
    const int64_t npairA = (int64_t)nocc * (nocc + 1) / 2;
    const int64_t nres = (int64_t)sh.nvirt * npairA + (int64_t)nocc * sh.nvirt * (sh.nvirt + 1) / 2;
    const size_t res_es = prec == CDS_PREC_FP64 ? 8 : 4;
    void *R = nullptr, *om = nullptr, *part = nullptr, *outd = nullptr, *act = nullptr;
    const int nblkA = sh.nvirt, nblkB = (sh.nvirt + 1) / 2;
    NewtonDev nd = {};
    int64_t nblk_sweep = nblkA + nblkB;
    void *hp;
    CDS_CALL(cds_pinned(ctx, (size_t)nsel * (2 * 8 + 8 + 4) + 64, &hp));
    double *h_out = (double *)hp;
    double *h_w = h_out + (size_t)nsel * 2;
    int *h_act = (int *)(h_w + nsel);
    bool first_done = false;              // the first evaluation came with the residues
    if (mode == CDS_QP_RESIDUES && fused) {
        // residues formed by the fused contraction (no integrals in HBM), swept per task; the
        // contraction also sums them at the starting energies (the first Newton evaluation)
        CDS_CALL(cds_ws(ctx, WS_SG_RES, (size_t)nsel * fp.nres * res_es, &R));
        nblk_sweep = fp.tpt;
        CDS_CALL(cds_ws(ctx, WS_SG_PART, (size_t)nsel * nblk_sweep * 2 * 8, &part));
        // sums, the active list, then the solve's state: w and P (double), status and steps
        // (int), read back in one copy; then e_q (double), the targets' orbitals (int), the two
        // counters
        const size_t off_state = (((size_t)nsel * 2 * 8 + 32 + (size_t)nsel * 4) + 255) / 256 * 256;
        CDS_CALL(cds_ws(ctx, WS_SG_OUT, off_state + (size_t)nsel * (8 + 8 + 4 + 4 + 8 + 4) + 64, &outd));
        act = (unsigned char *)outd + (size_t)nsel * 2 * 8 + 32;
        unsigned char *stb = (unsigned char *)outd + off_state;
        nd.om = (double *)stb;
        nd.pole = nd.om + nsel;
        nd.status = (int *)(nd.pole + nsel);
        nd.iters = nd.status + nsel;
        nd.qe = (double *)(nd.iters + nsel);
        nd.sel = (int *)(nd.qe + nsel);
        nd.cnt = nd.sel + nsel;
        nd.act = (int *)act;
        om = nd.om;
        CDS_HIP(ctx, hipMemcpyAsync(nd.sel, h_sel, (size_t)nsel * 4, hipMemcpyHostToDevice, ctx->stream));
        if (h_omega0)
            CDS_HIP(ctx, hipMemcpyAsync(om, h_omega0, (size_t)nsel * 8, hipMemcpyHostToDevice, ctx->stream));
        hipLaunchKernelGGL(newton_init_kernel, dim3(1), dim3(256), 0, ctx->stream, nsel, eps, h_omega0 ? 1 : 0, nd);
        CDS_LAUNCHED(ctx);
        const int csz = fused_chunk(ctx, sh);
        int *tsel;
        CDS_CALL(target_slots(ctx, nsel, &tsel));
        for (int s0 = 0; s0 < nsel; s0 += csz) {
            const int nsc = std::min(csz, nsel - s0);
            CdsTimer t;
            CDS_CALL(cds_timer_start(ctx, &t));
            CDS_CALL(cds_fused_residues(ctx, prec, fp, ldk, nmo, nocc, nsc, tsel + s0, Bsel, Bvo, Slo, Vlo, eps,
                                        (unsigned char *)R + (size_t)s0 * fp.nres * res_es, (const double *)om + s0,
                                        (double *)part + (size_t)s0 * nblk_sweep * 2));
            CDS_CALL(cds_timer_stop(ctx, &t, &ctx->stats.t_contract_ms));
            ctx->stats.flops_contract += 2.0 * (double)nvec * nsc * nmo * (double)sh.nvo;
            ctx->stats.n_contract += 1;
        }
        first_done = true;
    } else if (mode == CDS_QP_RESIDUES) {
        // blocks the fused kernel cannot read: integrals through HBM, then the residue epilogue
        CDS_CALL(cds_ws(ctx, WS_SG_RES, (size_t)nsel * nres * res_es + (size_t)nsel * 4, &R));
        const int csz = chunk_targets(ctx, sh);
        void *G;
        CDS_CALL(cds_ws(ctx, WS_SG_G, (size_t)csz * nmo * sh.nvo * res_es, &G));
        for (int s0 = 0; s0 < nsel; s0 += csz) {
            const int nsc = std::min(csz, nsel - s0);
            CDS_CALL(contract_chunk(ctx, sh, Bsel, Bvo, s0, nsc, G));
            EpArgs e = {};
            e.G = G;
            e.nmo = nmo;
            e.nocc = nocc;
            e.nvirt = sh.nvirt;
            e.nsc = nsc;
            e.nvo = sh.nvo;
            e.eps = eps;
            e.R = (unsigned char *)R + (size_t)s0 * nres * res_es;
            e.nres = nres;
            e.offB = (int64_t)sh.nvirt * npairA;
            CdsTimer t;
            CDS_CALL(cds_timer_start(ctx, &t));
            CDS_CALL(launch_epilogue<EP_RESIDUE>(ctx, sh, e, prec == CDS_PREC_FP64));
            CDS_CALL(cds_timer_stop(ctx, &t, &ctx->stats.t_epilogue_ms));
        }
        CDS_CALL(cds_ws(ctx, WS_SG_OMEGA, (size_t)nsel * 8, &om));
        CDS_CALL(cds_ws(ctx, WS_SG_PART, (size_t)nsel * (nblkA + nblkB) * 2 * 8, &part));
        CDS_CALL(cds_ws(ctx, WS_SG_OUT, (size_t)nsel * 2 * 8 + (size_t)nsel * 4 + 64, &outd));
        act = (unsigned char *)outd + (size_t)nsel * 2 * 8 + 32;
    }

    if (dev) {
        // chunks of NEWTON_CHUNK steps between reads of the count of targets still iterating;
        // a step with none left launches kernels that return at once
        constexpr int NEWTON_CHUNK = 3;
        int *h_cnt = (int *)h_out;
        for (int it = 1; it <= max_iter;) {
            const int last = std::min(max_iter, it + NEWTON_CHUNK - 1);
            for (; it <= last; ++it) {
                if (!(first_done && it == 1))
                    CDS_CALL(cds_fused_sweep(ctx, prec, fp, nmo, nocc, nsel, (const int *)act, eps,
                                             (const double *)om, R, (double *)part, nd.cnt));
                hipLaunchKernelGGL(reduce_active_kernel, dim3((unsigned)(2 * nsel)), dim3(256), 0, ctx->stream,
                                   (const double *)part, (int)nblk_sweep, (const int *)nd.cnt, (double *)outd);
                hipLaunchKernelGGL(newton_step_kernel, dim3(1), dim3(64), 0, ctx->stream, (const double *)outd, conv,
                                   it, nd);
                CDS_LAUNCHED(ctx);
            }
            CDS_HIP(ctx, hipMemcpyAsync(h_cnt, nd.cnt, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
            if (h_cnt[0] == 0) break;
        }
        ctx->stats.n_newton_iter += h_cnt[1];
        // w, P, status and steps in one copy (24 bytes per target; the pinned buffer holds 28)
        CDS_HIP(ctx, hipMemcpyAsync(hp, nd.om, (size_t)nsel * 24, hipMemcpyDeviceToHost, ctx->stream));
        CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
        const double *hw = (const double *)hp, *hpo = hw + nsel;
        const int *hs = (const int *)(hpo + nsel), *hi = hs + nsel;
        for (int s = 0; s < nsel; ++s) {
            h_omega[s] = hw[s];
            h_pole[s] = hpo[s];
            h_status[s] = hs[s] < 0 ? CDS_QP_MAX_ITER : hs[s];
            h_iters[s] = hi[s];
        }
        CDS_CALL(cds_timer_stop(ctx, &tall, &ctx->stats.t_newton_ms));
        CDS_CALL(cds_timers_flush(ctx));
        return CDS_OK;
    }
    for (int s = 0; s < nsel; ++s) active.push_back(s);
    std::vector<double> out_all((size_t)nsel * 2);
    for (int it = 1; it <= max_iter && !active.empty(); ++it) {
        if (mode == CDS_QP_RESIDUES) {
            // the first evaluation of the fused path came with the residues (all targets active)
            if (!(first_done && it == 1)) {
                for (int s = 0; s < nsel; ++s) h_w[s] = w[s];
                for (size_t k = 0; k < active.size(); ++k) h_act[k] = active[k];
                CDS_HIP(ctx, hipMemcpyAsync(om, h_w, (size_t)nsel * 8, hipMemcpyHostToDevice, ctx->stream));
                CDS_HIP(ctx, hipMemcpyAsync(act, h_act, active.size() * 4, hipMemcpyHostToDevice, ctx->stream));
                if (fused) {
                    CDS_CALL(cds_fused_sweep(ctx, prec, fp, nmo, nocc, (int)active.size(), (const int *)act, eps,
                                             (const double *)om, R, (double *)part));
                } else {
                    EpArgs e = {};
                    e.nmo = nmo;
                    e.nocc = nocc;
                    e.nvirt = sh.nvirt;
                    e.nvo = sh.nvo;
                    e.eps = eps;
                    e.omega = (const double *)om;
                    e.T = 1;
                    e.R = R;
                    e.nres = nres;
                    e.offB = (int64_t)sh.nvirt * npairA;
                    e.part = (double *)part;
                    e.nblkA = nblkA;
                    e.nblkB = nblkB;
                    dim3 g((unsigned)(nblkA + nblkB), (unsigned)active.size());
                    if (prec == CDS_PREC_FP64)
                        hipLaunchKernelGGL(sweep_kernel<double>, g, dim3(EP_NT), 0, ctx->stream, e, (const int *)act);
                    else
                        hipLaunchKernelGGL(sweep_kernel<float>, g, dim3(EP_NT), 0, ctx->stream, e, (const int *)act);
                    CDS_LAUNCHED(ctx);
                }
            }
            int n = (int)active.size() * 2;
            hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)n), dim3(256), 0,
                               ctx->stream, (const double *)part, (int)active.size(), (int)nblk_sweep, 1,
                               (double *)outd);
            CDS_LAUNCHED(ctx);
            CDS_HIP(ctx, hipMemcpyAsync(h_out, outd, (size_t)active.size() * 2 * 8, hipMemcpyDeviceToHost,
                                        ctx->stream));
            CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
            for (size_t k = 0; k < active.size(); ++k) {
                out_all[2 * active[k]] = h_out[2 * k];
                out_all[2 * active[k] + 1] = h_out[2 * k + 1];
            }
        } else {
            // recompute the integrals for every target at its current energy (T = 1)
            CDS_CALL(cds_sigma_eval_internal(ctx, prec, nvec, ldk, nmo, nocc, nsel, Bsel, Bvo, eps,
                                             w.data(), 1, out_all.data()));
        }
        ctx->stats.n_newton_iter += 1;
        std::vector<int> still;
        for (int s : active) {
            const double q_eps = heps[h_sel[s]];
            const double sg = out_all[2 * s], ds = out_all[2 * s + 1];
            iters[s] = it;
            if (!std::isfinite(sg) || !std::isfinite(ds)) {   // a denominator vanished
                status[s] = CDS_QP_NONFINITE;
                continue;
            }
            const double P = 1.0 / (1.0 - ds);
            const double wn = w[s] + (q_eps + sg - w[s]) * P;
            pole[s] = P;
            if (!std::isfinite(wn) || !std::isfinite(P)) {
                w[s] = wn;
                status[s] = CDS_QP_NONFINITE;
                continue;
            }
            if (std::fabs(wn - w[s]) <= conv) {
                w[s] = wn;
                status[s] = CDS_QP_CONVERGED;
                continue;
            }
            w[s] = wn;
            still.push_back(s);
        }
        active.swap(still);
    }
    for (int s : active) status[s] = CDS_QP_MAX_ITER;
    for (int s = 0; s < nsel; ++s) {
        h_omega[s] = w[s];
        h_pole[s] = pole[s];
        h_iters[s] = iters[s];
        h_status[s] = status[s];
    }
    CDS_CALL(cds_timer_stop(ctx, &tall, &ctx->stats.t_newton_ms));
    CDS_CALL(cds_timers_flush(ctx));
    return CDS_OK;
}

// ---- allocation-free self-energy -----------------------------------------------------------
// Device memory of cds_sigma2_noalloc: one array per GPU, held from the library's load until
// the process ends.  Host code must not use the array's name as an address: its device address
// comes from hipGetSymbolAddress (cds_noalloc_scratch_address, called by cds_create with the
// context's device current) and is kept in the context.
static __device__ __align__(256) unsigned char scratch[CDS_NOALLOC_SCRATCH_BYTES];

int cds_noalloc_scratch_address(void **out)
{
    *out = nullptr;
    return hipGetSymbolAddress(out, HIP_SYMBOL(scratch)) == hipSuccess && *out ? CDS_OK : CDS_EDEVICE;
}

extern "C" int cds_sigma2_noalloc(cds_ctx *ctx, int32_t prec, int64_t nvec, int64_t ldk, int32_t nmo,
                                  int32_t nocc, int32_t nsel, const int32_t *h_sel, const void *Bsel,
                                  const void *Bvo, const double *eps, int32_t T, const double *h_omega,
                                  double *h_sigma, double *h_dsigma)
{
    CDS_CALL(cds_enter(ctx));
    SigmaShape sh = {prec, nvec, ldk, nmo, nocc, nmo - nocc, nsel,
                     (int64_t)(nmo - nocc) * nocc, (int64_t)nsel * nmo};
    CDS_CALL(check_shape(ctx, sh, h_sel, Bsel, Bvo, eps));
    CDS_REQUIRE(ctx, T >= 1 && T <= TMAX, "T must be in [1, %d]", TMAX);
    CDS_REQUIRE(ctx, h_omega && h_sigma && h_dsigma, "NULL host pointer");
    const void *Slo, *Vlo;
    lo_planes(sh, Bsel, Bvo, &Slo, &Vlo);
    CdsFusedPlan fp;
    CDS_REQUIRE(ctx, cds_fused_plan(prec, nvec, ldk, nmo, nocc, Bsel, Bvo, Slo, Vlo, &fp),
                "allocation-free path needs 16-byte aligned blocks with ldk >= nvec rounded up to the "
                "K stage (16 FP64, 32 FP32 / BF16X3) and ldk * element size a multiple of 16");
    if (!ctx->scratch) return cds_fail(ctx, CDS_ESTATE, "no device address for the scratch array");
    // scratch layout: partials [csz][tpt][T][2], sigma [nsel][T], dsigma [nsel][T],
    // trial energies [nsel][T], target slots [nsel]
    const int csz = fused_chunk(ctx, sh);
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t b_part = up((size_t)csz * fp.tpt * T * 2 * 8), b_nt = up((size_t)nsel * T * 8);
    const size_t need = b_part + 3 * b_nt + up((size_t)nsel * 4);
    CDS_REQUIRE(ctx, need <= (size_t)CDS_NOALLOC_SCRATCH_BYTES,
                "allocation-free path: %zu bytes of scratch needed, %d available (fewer targets per "
                "launch, see cds_set_target_chunk, or fewer trial energies)",
                need, CDS_NOALLOC_SCRATCH_BYTES);
    unsigned char *sp = (unsigned char *)ctx->scratch;
    double *part = (double *)sp;
    double *sig = (double *)(sp + b_part), *dsig = (double *)(sp + b_part + b_nt);
    double *om = (double *)(sp + b_part + 2 * b_nt);
    int *tsel = (int *)(sp + b_part + 3 * b_nt);
    CDS_HIP(ctx, hipMemcpyAsync(om, h_omega, (size_t)nsel * T * 8, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(iota_kernel, dim3((unsigned)cds_ceil_div(nsel, 256)), dim3(256), 0, ctx->stream, tsel, nsel);
    CDS_LAUNCHED(ctx);
    for (int s0 = 0; s0 < nsel; s0 += csz) {
        const int nsc = std::min(csz, nsel - s0);
        CDS_CALL(cds_fused_sigma(ctx, prec, fp, ldk, nmo, nocc, nsc, tsel + s0, Bsel, Bvo, Slo, Vlo, eps,
                                 om + (int64_t)s0 * T, T, part));
        const int nout = nsc * T * 2;
        hipLaunchKernelGGL(reduce_split_kernel, dim3((unsigned)nout), dim3(256), 0, ctx->stream,
                           (const double *)part, nsc, (int)fp.tpt, T, sig + (int64_t)s0 * T,
                           dsig + (int64_t)s0 * T);
        CDS_LAUNCHED(ctx);
    }
    CDS_HIP(ctx, hipMemcpyAsync(h_sigma, sig, (size_t)nsel * T * 8, hipMemcpyDeviceToHost, ctx->stream));
    CDS_HIP(ctx, hipMemcpyAsync(h_dsigma, dsig, (size_t)nsel * T * 8, hipMemcpyDeviceToHost, ctx->stream));
    CDS_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return CDS_OK;
}
