/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the bivariate parsimonious-Matern
 * Gaussian log-likelihood and the cokriging predictor.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library: it has its own Gamma function,
 * its own modified Bessel function K_nu (a different method from the GPU one),
 * its own covariance builder, its own Cholesky factorisation and solves.
 *
 * What is computed (paper, Section 4 and Section 5.2):
 *   - Eq. (2) parsimonious multivariate Matern, p = 2, d = 2:
 *       C_ij(h) = rho_ij sigma_i sigma_j (h/a)^nu_ij K_nu_ij(h/a) / (2^(nu_ij-1) Gamma(nu_ij)),
 *       nu_12 = (nu_11 + nu_22)/2, rho_11 = rho_22 = 1 and rho_12 from the
 *       Gneiting-Kleiber-Schlather colocated-correlation formula (Section 4.2;
 *       the printed square root on the third Gamma factor is read as absent,
 *       otherwise rho_ii != 1 contradicts unit marginal variances).
 *   - Representation I (Section 5.2): Sigma[2l+i, 2r+j] = C_ij(||s_l - s_r||),
 *       Z = (Z_1(s_1), Z_2(s_1), Z_1(s_2), ...), 0-based l, r, i, j.
 *   - Eq. (1) l(theta) = -(p n / 2) log(2 pi) - 1/2 log|Sigma| - 1/2 Z^T Sigma^-1 Z
 *       via the Cholesky factor (Section 5.2): log|Sigma| = 2 sum log L_jj,
 *       Z^T Sigma^-1 Z = ||L^-1 Z||^2.
 *   - Eq. (3)-(4) cokriging: Zhat(s0) = c0^T Sigma^-1 Z,
 *       c0[2r+i, j] = C_ij(||s0 - s_r||).
 *   - Eq. (5) predictor MSE: E = tr{C(0) - c0^T Sigma^-1 c0}.
 *
 * Special functions (the paper names K_nu and Gamma but gives no evaluation
 * method):
 *   - 1/Gamma(1+z) for |z| <= 1/2 by its Taylor series (coefficients generated
 *     by gen_rgamma_coeffs.py); Gamma(x) by shifting into [1/2, 3/2] with
 *     Gamma(x+1) = x Gamma(x).
 *   - K_mu, K_mu+1 for |mu| <= 1/2:
 *       x <= 2: Temme's (1975) series with the auxiliary functions
 *               Gamma_1(mu) = [1/Gamma(1-mu) - 1/Gamma(1+mu)]/(2 mu),
 *               Gamma_2(mu) = [1/Gamma(1-mu) + 1/Gamma(1+mu)]/2,
 *               taken from the same Taylor series (no cancellation).
 *       x >  2: K_mu(x) = sqrt(pi) (2x)^mu e^-x U(mu+1/2, 2mu+1, 2x) (DLMF 10.39.6).
 *               The ratios U_k/U_{k-1} of U_k = U(mu+1/2+k, 2mu+1, 2x) follow
 *               from the contiguous relation DLMF 13.3.7 by backward recurrence
 *               (U_k is the minimal solution); the normalisation is
 *               sum_k C_k U_k = (2x)^(-mu-1/2) with
 *               C_k = prod_{j=1..k} ((j-1/2)^2 - mu^2) / k!,
 *               which follows from the integral representation DLMF 13.4.4 and
 *               the binomial series of (1+t)^(1/2-mu) in t/(1+t).  Then
 *               K_mu+1/K_mu = [mu + 1/2 + x + (mu^2 - 1/4) U_1/U_0] / x.
 *   - then the upward recurrence K_{v+1} = K_{v-1} + (2v/x) K_v (DLMF 10.29.1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "rgamma_coeffs.h"

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ Gamma */

/* 1/Gamma(1+z), |z| <= 1/2, Horner evaluation of the Taylor series. */
double orc_rgamma1p(double z) {
    double s = 0.0;
    for (int k = ORC_RGAMMA_NCOEF - 1; k >= 0; --k) s = s * z + orc_rgamma_coef[k];
    return s;
}

/* Gamma(x) for x > 0 (moderate x: the recurrence is unrolled). */
double orc_gamma(double x) {
    if (!(x > 0.0) || !isfinite(x)) return NAN;
    double f = 1.0;
    while (x > 1.5) { x -= 1.0; f *= x; }      /* Gamma(x) = (x-1) Gamma(x-1) */
    while (x < 0.5) { f /= x; x += 1.0; }      /* Gamma(x) = Gamma(x+1) / x   */
    return f / orc_rgamma1p(x - 1.0);
}

/* ----------------------------------------------------------- Bessel K_nu */

/* Temme's series, |mu| <= 1/2, 0 < x <= 2. */
static void orc_bessel_k_temme(double mu, double x, double *kmu, double *kmu1) {
    /* Gamma_1(mu) = -sum_{k odd} a_k mu^(k-1); Gamma_2(mu) = sum_{k even} a_k mu^k */
    double mu2 = mu * mu;
    double g1 = 0.0, g2 = 0.0;
    for (int k = ORC_RGAMMA_NCOEF - 1; k >= 0; --k) {
        if (k & 1) g1 = g1 * mu2 + orc_rgamma_coef[k];
        else       g2 = g2 * mu2 + orc_rgamma_coef[k];
    }
    g1 = -g1;
    double rg_plus = orc_rgamma1p(mu);    /* 1/Gamma(1+mu) */
    double rg_minus = orc_rgamma1p(-mu);  /* 1/Gamma(1-mu) */
    double lnx2 = log(2.0 / x);
    double sigma = mu * lnx2;
    double fact = (mu == 0.0) ? 1.0 : (ORC_PI * mu) / sin(ORC_PI * mu);
    double shs = (sigma == 0.0) ? 1.0 : sinh(sigma) / sigma;
    double f = fact * (cosh(sigma) * g1 + shs * lnx2 * g2);
    double p = 0.5 * exp(sigma) / rg_plus;    /* (1/2)(x/2)^-mu Gamma(1+mu) */
    double q = 0.5 * exp(-sigma) / rg_minus;  /* (1/2)(x/2)^+mu Gamma(1-mu) */
    double c = 1.0;
    double quarter_x2 = 0.25 * x * x;
    double sum = f;       /* sum_k c_k f_k */
    double sum1 = p;      /* sum_k c_k (p_k - k f_k) */
    for (int k = 1; k < 500; ++k) {
        double dk = (double)k;
        f = (dk * f + p + q) / (dk * dk - mu2);
        p /= (dk - mu);
        q /= (dk + mu);
        c *= quarter_x2 / dk;
        double t = c * f;
        sum += t;
        sum1 += c * (p - dk * f);
        if (fabs(t) < 1e-18 * fabs(sum)) break;
    }
    *kmu = sum;
    *kmu1 = (2.0 / x) * sum1;
}

/* Tricomi-U continued fraction by backward recurrence, |mu| <= 1/2, x > 2. */
static double orc_cf2_sum(double mu, double x, int kmax, double *r1_out) {
    double mu2 = mu * mu;
    double *r = (double *)malloc(sizeof(double) * (size_t)(kmax + 2));
    /* 1/r_k = 2(k+x) - c_{k+1} r_{k+1},  c_j = (j-1/2)^2 - mu^2,  r_{kmax+1} = 0 */
    r[kmax + 1] = 0.0;
    for (int k = kmax; k >= 1; --k) {
        double cj = (k + 0.5) * (k + 0.5) - mu2;
        r[k] = 1.0 / (2.0 * (k + x) - cj * r[k + 1]);
    }
    /* S = sum_k C_k U_k/U_0, term_k = term_{k-1} * c_k / k * r_k */
    double term = 1.0, S = 1.0;
    for (int k = 1; k <= kmax; ++k) {
        double ck = (k - 0.5) * (k - 0.5) - mu2;
        term *= ck / (double)k * r[k];
        S += term;
    }
    *r1_out = r[1];
    free(r);
    return S;
}

static void orc_bessel_k_cf2(double mu, double x, double *kmu, double *kmu1) {
    int kmax = 64;
    double r1 = 0.0;
    double S = orc_cf2_sum(mu, x, kmax, &r1);
    for (int it = 0; it < 12; ++it) {
        kmax *= 2;
        double r1n = 0.0;
        double Sn = orc_cf2_sum(mu, x, kmax, &r1n);
        int done = fabs(Sn - S) <= 1e-17 * fabs(Sn) && fabs(r1n - r1) <= 1e-17 * fabs(r1n);
        S = Sn;
        r1 = r1n;
        if (done) break;
    }
    double k0 = sqrt(ORC_PI / (2.0 * x)) * exp(-x) / S;
    *kmu = k0;
    *kmu1 = k0 * (mu + 0.5 + x + (mu * mu - 0.25) * r1) / x;
}

/* K_nu(x) for real nu and x > 0. */
double orc_bessel_k(double nu, double x) {
    if (!(x > 0.0)) return NAN;
    nu = fabs(nu);                       /* K_{-nu} = K_nu */
    int n = (int)floor(nu + 0.5);
    double mu = nu - (double)n;          /* mu in [-1/2, 1/2) */
    double kmu, kmu1;
    if (x <= 2.0) orc_bessel_k_temme(mu, x, &kmu, &kmu1);
    else          orc_bessel_k_cf2(mu, x, &kmu, &kmu1);
    if (n == 0) return kmu;
    double kprev = kmu, kcur = kmu1;     /* K_{mu}, K_{mu+1} */
    for (int j = 1; j < n; ++j) {
        double knext = kprev + 2.0 * (mu + (double)j) / x * kcur;
        kprev = kcur;
        kcur = knext;
    }
    return kcur;
}

/* Normalised Matern M(x; nu) = x^nu K_nu(x) / (2^(nu-1) Gamma(nu)), M(0) = 1. */
double orc_matern(double x, double nu) {
    if (x == 0.0) return 1.0;
    double k = orc_bessel_k(nu, x);
    if (k == 0.0) return 0.0;
    return pow(x, nu) * k / (pow(2.0, nu - 1.0) * orc_gamma(nu));
}

/* ---------------------------------------------------------------- theta */

/* theta = (sigma11^2, sigma22^2, a, nu11, nu22, beta), the paper's order. */
int orc_theta_check(const double *th) {
    if (!(th[0] > 0.0) || !isfinite(th[0])) return -1;
    if (!(th[1] > 0.0) || !isfinite(th[1])) return -2;
    if (!(th[2] > 0.0) || !isfinite(th[2])) return -3;
    if (!(th[3] > 0.0) || !isfinite(th[3])) return -4;
    if (!(th[4] > 0.0) || !isfinite(th[4])) return -5;
    if (!(fabs(th[5]) < 1.0)) return -6;   /* 2x2 beta is a PD correlation matrix */
    return 0;
}

/* rho_12 = beta [G(nu11+d/2)/G(nu11)]^1/2 [G(nu22+d/2)/G(nu22)]^1/2 G(nu12)/G(nu12+d/2), d = 2 */
double orc_rho12(const double *th) {
    const double d2 = 1.0;  /* d/2 with d = 2 */
    double nu11 = th[3], nu22 = th[4], nu12 = 0.5 * (nu11 + nu22);
    return th[5] * sqrt(orc_gamma(nu11 + d2) / orc_gamma(nu11)) *
           sqrt(orc_gamma(nu22 + d2) / orc_gamma(nu22)) *
           orc_gamma(nu12) / orc_gamma(nu12 + d2);
}

/* C_ij(h) for i, j in {0, 1}. */
double orc_cross_cov(const double *th, int i, int j, double h) {
    double nu11 = th[3], nu22 = th[4];
    double nu = (i != j) ? 0.5 * (nu11 + nu22) : (i == 0 ? nu11 : nu22);
    double rho = (i != j) ? orc_rho12(th) : 1.0;
    double si = sqrt(i == 0 ? th[0] : th[1]);
    double sj = sqrt(j == 0 ? th[0] : th[1]);
    return rho * si * sj * orc_matern(h / th[2], nu);
}

static double orc_dist(double x1, double y1, double x2, double y2) {
    double dx = x1 - x2, dy = y1 - y2;
    return sqrt(dx * dx + dy * dy);
}

/* Sigma[row, col] for arbitrary sampled entries (0-based). */
void orc_cov_entries(const double *xs, const double *ys, const double *th,
                     const int64_t *rows, const int64_t *cols, int64_t m, double *out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < m; ++t) {
        int64_t l = rows[t] / 2, r = cols[t] / 2;
        int i = (int)(rows[t] % 2), j = (int)(cols[t] % 2);
        out[t] = orc_cross_cov(th, i, j, orc_dist(xs[l], ys[l], xs[r], ys[r]));
    }
}

/* Dense 2n x 2n Sigma, row-major. */
void orc_cov_dense(const double *xs, const double *ys, int64_t n, const double *th, double *S) {
    int64_t N = 2 * n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t l = 0; l < n; ++l) {
        for (int64_t r = 0; r <= l; ++r) {
            double h = orc_dist(xs[l], ys[l], xs[r], ys[r]);
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    double c = orc_cross_cov(th, i, j, h);
                    S[(2 * l + i) * N + (2 * r + j)] = c;
                    S[(2 * r + j) * N + (2 * l + i)] = c;
                }
        }
    }
}

/* ------------------------------------------------------ linear algebra */

/* A pivot at or below this fraction of its original diagonal entry is
 * treated as a failure: the matrix is singular to working precision (a
 * duplicated location gives a pivot that is zero up to rounding, and the sign
 * of that rounding must not decide the result). */
#define ORC_SINGULAR_REL 0x1p-40

/* In-place Cholesky A = L L^T of a row-major n x n SPD matrix (lower factor;
 * the strict upper triangle is zeroed).  Column-by-column (Cholesky-Crout)
 * with dot products in index order.  Returns 0, or the 1-based index of the
 * first pivot that is not above ORC_SINGULAR_REL times its diagonal entry. */
int64_t orc_potrf(double *A, int64_t n) {
    for (int64_t j = 0; j < n; ++j) {
        double *rj = A + j * n;
        double d = rj[j];
        const double tol = ORC_SINGULAR_REL * d;
        for (int64_t k = 0; k < j; ++k) d -= rj[k] * rj[k];
        if (!(d > tol) || !(d > 0.0)) return j + 1;
        double ljj = sqrt(d);
        rj[j] = ljj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            double *ri = A + i * n;
            double s = ri[j];
            for (int64_t k = 0; k < j; ++k) s -= ri[k] * rj[k];
            ri[j] = s / ljj;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = i + 1; k < n; ++k) A[i * n + k] = 0.0;
    return 0;
}

/* b <- L^-1 b (forward substitution), row-major lower L. */
void orc_trsv_lower(const double *L, int64_t n, double *b) {
    for (int64_t i = 0; i < n; ++i) {
        double s = b[i];
        for (int64_t k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
        b[i] = s / L[i * n + i];
    }
}

/* b <- L^-T b (backward substitution with the transpose). */
void orc_trsv_lower_trans(const double *L, int64_t n, double *b) {
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int64_t k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
        b[i] = s / L[i * n + i];
    }
}

/* ------------------------------------------------------------ likelihood */

/* out = {loglik, logdet, quad}.  Returns 0, a negative theta code, or the
 * 1-based first failing pivot (then loglik = -inf). */
int64_t orc_loglik(const double *xs, const double *ys, const double *z, int64_t n,
                   const double *th, double *out) {
    int chk = orc_theta_check(th);
    if (chk) return chk;
    int64_t N = 2 * n;
    double *S = (double *)malloc(sizeof(double) * (size_t)(N * N));
    double *y = (double *)malloc(sizeof(double) * (size_t)N);
    if (!S || !y) { free(S); free(y); return -100; }
    orc_cov_dense(xs, ys, n, th, S);
    int64_t info = orc_potrf(S, N);
    if (info) {
        out[0] = -INFINITY; out[1] = NAN; out[2] = NAN;
        free(S); free(y);
        return info;
    }
    double logdet = 0.0;
    for (int64_t j = 0; j < N; ++j) logdet += log(S[j * N + j]);
    logdet *= 2.0;
    memcpy(y, z, sizeof(double) * (size_t)N);
    orc_trsv_lower(S, N, y);
    double q = 0.0;
    for (int64_t j = 0; j < N; ++j) q += y[j] * y[j];
    out[0] = -(double)n * log(2.0 * ORC_PI) - 0.5 * logdet - 0.5 * q;
    out[1] = logdet;
    out[2] = q;
    free(S); free(y);
    return 0;
}

/* Cokriging predictions zhat[2t + j] for m targets and, if mse != NULL, the
 * predictor MSE of Eq. (5) per target.  Returns as orc_loglik. */
int64_t orc_cokrige(const double *xs, const double *ys, const double *z, int64_t n,
                    const double *th, const double *x0, const double *y0, int64_t m,
                    double *zhat, double *mse) {
    int chk = orc_theta_check(th);
    if (chk) return chk;
    int64_t N = 2 * n;
    double *S = (double *)malloc(sizeof(double) * (size_t)(N * N));
    double *w = (double *)malloc(sizeof(double) * (size_t)N);
    if (!S || !w) { free(S); free(w); return -100; }
    orc_cov_dense(xs, ys, n, th, S);
    int64_t info = orc_potrf(S, N);
    if (info) { free(S); free(w); return info; }
    memcpy(w, z, sizeof(double) * (size_t)N);
    orc_trsv_lower(S, N, w);
    orc_trsv_lower_trans(S, N, w);          /* w = Sigma^-1 Z */
#pragma omp parallel
    {
        double *c0 = (double *)malloc(sizeof(double) * (size_t)N * 2);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < m; ++t) {
            for (int64_t r = 0; r < n; ++r) {
                double h = orc_dist(x0[t], y0[t], xs[r], ys[r]);
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j)
                        c0[(2 * r + i) * 2 + j] = orc_cross_cov(th, i, j, h);
            }
            for (int j = 0; j < 2; ++j) {
                double s = 0.0;
                for (int64_t k = 0; k < N; ++k) s += c0[k * 2 + j] * w[k];
                zhat[2 * t + j] = s;
            }
            if (mse) {
                /* tr{C(0) - c0^T Sigma^-1 c0} = tr C(0) - sum_j ||L^-1 c0[:, j]||^2 */
                double e = th[0] + th[1];
                double *col = (double *)malloc(sizeof(double) * (size_t)N);
                for (int j = 0; j < 2; ++j) {
                    for (int64_t k = 0; k < N; ++k) col[k] = c0[k * 2 + j];
                    orc_trsv_lower(S, N, col);
                    double s = 0.0;
                    for (int64_t k = 0; k < N; ++k) s += col[k] * col[k];
                    e -= s;
                }
                free(col);
                mse[t] = e;
            }
        }
        free(c0);
    }
    free(S); free(w);
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Vectorised helpers for the Python side. */
void orc_bessel_k_vec(double nu, const double *x, int64_t m, double *out) {
    for (int64_t t = 0; t < m; ++t) out[t] = orc_bessel_k(nu, x[t]);
}

void orc_matern_vec(double nu, const double *x, int64_t m, double *out) {
    for (int64_t t = 0; t < m; ++t) out[t] = orc_matern(x[t], nu);
}
