/*
 * ORACLE — test infrastructure only.  Plain, slow, FP64 reference for the
 * two-electron integrals and the diagonal-pivoted incomplete Cholesky
 * decomposition of the ERI supermatrix.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library; the product
 * path never does.  It shares no code with the HIP library.
 *
 * Paper: Vysotskiy & Cederbaum, "On the Cholesky Decomposition for electron
 * propagator methods" (arXiv:0912.1459), Sec. II.A.
 *
 *   - basis: real primitive s-Gaussians chi_mu(r) = N_mu exp(-a_mu |r-A_mu|^2),
 *     N_mu = (2 a_mu / pi)^(3/4); product densities rho_I = chi_mu chi_nu with
 *     I = (mu, nu), mu <= nu (Sec. II.A, definition of the product-density set).
 *     Pair index I = nu(nu+1)/2 + mu (0-based, LAPACK 'U' packed order).
 *   - ERI (mu nu | lam sig) = (rho_I | V | rho_J), Eq. (integral).  For
 *     s-Gaussians the closed form is the textbook Boys-function result
 *       V_IJ = K_I K_J 2 pi^(5/2) / (p q sqrt(p+q)) F0(pq/(p+q) |P-Q|^2)
 *     with p = a_mu + a_nu, P = (a_mu A_mu + a_nu A_nu)/p,
 *     K_I = N_mu N_nu exp(-a_mu a_nu |A_mu - A_nu|^2 / p) (Gaussian product
 *     theorem) and F0(T) = 1/2 sqrt(pi/T) erf(sqrt T); below T = 1e-12 the
 *     series 1 - T/3 + T^2/10 is used (truncation < 1e-25).
 *   - Pivoted Cholesky, Eqs. (gs_coulomb), (CD), (stricterr): vectors are
 *     added one at a time; each new vector is the residual ERI column of the
 *     pivot pair divided by the square root of its residual diagonal.  The
 *     procedure continues while the largest residual diagonal exceeds delta
 *     and stops once it is <= delta, so that every residual diagonal is then
 *     <= delta.  Pivot rule (the paper is silent): among non-pivot pairs with
 *     D_I >= D_max - tau, take the lowest index.  Entries of later vectors on
 *     earlier pivot rows are exactly zero (lower-trapezoidal L, Eq. (CD)).
 *
 * Storage: L row-major, L[I*ldl + k] = L^k_I (row of pair I contiguous).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Boys function of order zero. */
double orc_boys_f0(double T)
{
    if (T < 1e-12)
        return 1.0 - T / 3.0 + T * T / 10.0;
    double s = sqrt(T);
    return 0.5 * sqrt(M_PI / T) * erf(s);
}

static double snorm(double a) { return pow(2.0 * a / M_PI, 0.75); }

/* (mu nu | lam sig) for four normalized primitive s-Gaussians, Eq. (integral). */
double orc_eri4(const double *A, double a, const double *B, double b,
                const double *C, double c, const double *D, double d)
{
    double p = a + b, q = c + d;
    double ab2 = 0.0, cd2 = 0.0, pq2 = 0.0;
    double P[3], Q[3];
    for (int x = 0; x < 3; ++x) {
        ab2 += (A[x] - B[x]) * (A[x] - B[x]);
        cd2 += (C[x] - D[x]) * (C[x] - D[x]);
        P[x] = (a * A[x] + b * B[x]) / p;
        Q[x] = (c * C[x] + d * D[x]) / q;
    }
    for (int x = 0; x < 3; ++x)
        pq2 += (P[x] - Q[x]) * (P[x] - Q[x]);
    double KI = snorm(a) * snorm(b) * exp(-a * b * ab2 / p);
    double KJ = snorm(c) * snorm(d) * exp(-c * d * cd2 / q);
    double T = p * q / (p + q) * pq2;
    return KI * KJ * 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * orc_boys_f0(T);
}

/* Pair I -> (mu, nu), mu <= nu, I = nu(nu+1)/2 + mu. */
void orc_pair_index(int64_t I, int64_t *mu, int64_t *nu)
{
    int64_t n = (int64_t)((sqrt(8.0 * (double)I + 1.0) - 1.0) / 2.0);
    while (n * (n + 1) / 2 > I) --n;
    while ((n + 1) * (n + 2) / 2 <= I) ++n;
    *nu = n;
    *mu = I - n * (n + 1) / 2;
}

double orc_eri_pairs(int64_t I, int64_t J, const double *centres, const double *alpha)
{
    int64_t m, n, l, s;
    orc_pair_index(I, &m, &n);
    orc_pair_index(J, &l, &s);
    return orc_eri4(centres + 3 * m, alpha[m], centres + 3 * n, alpha[n],
                    centres + 3 * l, alpha[l], centres + 3 * s, alpha[s]);
}

/* Dense ERI supermatrix V[I*npairs + J] over all pairs (symmetric). */
void orc_eri_matrix(int32_t nbf, const double *centres, const double *alpha, double *V)
{
    int64_t np = (int64_t)nbf * (nbf + 1) / 2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t I = 0; I < np; ++I)
        for (int64_t J = I; J < np; ++J) {
            double v = orc_eri_pairs(I, J, centres, alpha);
            V[I * np + J] = v;
            V[J * np + I] = v;
        }
}

/* Diagonal V_II over all pairs. */
void orc_eri_diagonal(int32_t nbf, const double *centres, const double *alpha, double *out)
{
    int64_t np = (int64_t)nbf * (nbf + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t I = 0; I < np; ++I)
        out[I] = orc_eri_pairs(I, I, centres, alpha);
}

/* ERI columns V[:, cols[c]] -> out[c*npairs + I]. */
void orc_eri_columns(int32_t nbf, const double *centres, const double *alpha,
                     int64_t ncol, const int64_t *cols, double *out)
{
    int64_t np = (int64_t)nbf * (nbf + 1) / 2;
    for (int64_t c = 0; c < ncol; ++c) {
#pragma omp parallel for schedule(static)
        for (int64_t I = 0; I < np; ++I)
            out[c * np + I] = orc_eri_pairs(I, cols[c], centres, alpha);
    }
}

/*
 * Diagonal-pivoted incomplete Cholesky of V (dense if V != NULL, otherwise ERI
 * columns evaluated on demand from the basis).
 *
 * In/out: L (npairs x ldl, row-major), piv[max_vec], D[npairs] (residual
 * diagonal; pivots hold 0), *nvec.  When *nvec > 0 on entry the call resumes
 * from that state (L, piv and D as a previous call left them).
 * allowed: NULL, or npairs flags; only pairs with allowed[I] != 0 may become
 * pivots (every non-pivot row is still updated) -- the inner projection of
 * Eq. (int_approx) onto the allowed products, as in the atomic CD.
 * reverse: 0 sums the residual column over earlier vectors in the order j = 0, 1, ...; 1 in the
 * order j = k-1, ..., 0 (the same sum associated the other way: it measures how far rounding
 * alone moves a result).
 * Returns 0 when D_max <= delta, 1 when max_vec vectors were made first,
 * 2 when every allowed pair became a pivot, -4 when a non-pivot residual
 * diagonal fell below -psd_tol.  *dmax receives the final largest residual
 * diagonal among allowed non-pivots.
 */
int orc_pivoted_cd(int64_t npairs, const double *V, int32_t nbf, const double *centres,
                   const double *alpha, double delta, double tau, double psd_tol,
                   int64_t max_vec, int64_t ldl, double *L, int64_t *piv, double *D,
                   int64_t *nvec, double *dmax, const unsigned char *allowed, int reverse)
{
    unsigned char *is_piv = (unsigned char *)calloc((size_t)npairs, 1);
    double *col = (double *)malloc((size_t)npairs * sizeof(double));
    int64_t k = *nvec;
    if (k == 0) {
        /* initial residual diagonal D_I = V_II (the norm n_K before any projection) */
        for (int64_t I = 0; I < npairs; ++I)
            D[I] = V ? V[I * npairs + I] : orc_eri_pairs(I, I, centres, alpha);
    }
    for (int64_t j = 0; j < k; ++j)
        is_piv[piv[j]] = 1;
    int status = 0;
    for (;;) {
        /* largest residual diagonal among non-pivots */
        double dm = -INFINITY;
        int any = 0;
        for (int64_t I = 0; I < npairs; ++I)
            if (!is_piv[I]) {
                if (D[I] < -psd_tol) status = -4;
                if (allowed && !allowed[I]) continue;
                any = 1;
                if (D[I] > dm) dm = D[I];
            }
        *dmax = dm;
        if (status == -4) break;
        if (!any) { status = 2; break; }
        if (dm <= delta) { status = 0; break; }
        if (k >= max_vec) { status = 1; break; }
        /* pivot: lowest index within the tie window of the maximum; the window is tau
         * but at most 1% of the maximum, so it stays a tie window as delta nears tau */
        const double win = fmin(tau, 1e-2 * dm);
        int64_t p = -1;
        for (int64_t I = 0; I < npairs; ++I)
            if (!is_piv[I] && (!allowed || allowed[I]) && D[I] >= dm - win) { p = I; break; }
        double dp = D[p];
        double sq = sqrt(dp);
        /* residual column c_I = V_Ip - sum_{j<k} L_Ij L_pj */
        if (V) {
            for (int64_t I = 0; I < npairs; ++I) col[I] = V[I * npairs + p];
        } else {
#pragma omp parallel for schedule(static)
            for (int64_t I = 0; I < npairs; ++I) col[I] = orc_eri_pairs(I, p, centres, alpha);
        }
        const double *Lp = L + p * ldl;
#pragma omp parallel for schedule(static)
        for (int64_t I = 0; I < npairs; ++I) {
            double *LI = L + I * ldl;
            if (is_piv[I]) {
                LI[k] = 0.0;
            } else if (I == p) {
                LI[k] = sq;
            } else {
                double c = col[I];
                if (reverse)
                    for (int64_t j = k - 1; j >= 0; --j)
                        c -= LI[j] * Lp[j];
                else
                    for (int64_t j = 0; j < k; ++j)
                        c -= LI[j] * Lp[j];
                LI[k] = c / sq;
                D[I] -= LI[k] * LI[k];
            }
        }
        D[p] = 0.0;
        is_piv[p] = 1;
        piv[k] = p;
        ++k;
    }
    *nvec = k;
    free(col);
    free(is_piv);
    return status;
}
