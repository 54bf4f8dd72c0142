/*
 * mvgeo.h -- C ABI of the MI355X (gfx950) library for the bivariate
 * parsimonious-Matern Gaussian log-likelihood, its tile-low-rank (TLR) and
 * mixed-precision variants, and the cokriging predictor built on the same
 * Cholesky factor (arxiv 2008.07437).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers named d_* are device pointers (HBM of the current HIP device);
 * pointers named h_* are host pointers.  Device inputs are owned by the caller
 * and must stay valid until the work enqueued on `hip_stream` has finished.
 * `hip_stream` is a hipStream_t passed as void* (NULL = the null stream).
 * Host outputs are valid when the call returns: the call synchronises the
 * stream before writing them.
 *
 * Locations are n_loc points (d_x[l], d_y[l]) in R^2, l = 0..n_loc-1.  The
 * observation vector follows Representation I (Section 5.2): Z has 2*n_loc
 * entries, Z[2l+i] = Z_{i+1}(s_l).  The covariance Sigma(theta) is 2n x 2n
 * with Sigma[2l+i, 2r+j] = C_ij(||s_l - s_r||) (Eq. 2).
 *
 * Return codes (LAPACK style): 0 = success; -i = argument i (1-based) is
 * invalid; > 0 = numerical failure: the 1-based global index of the first
 * Cholesky pivot that is not above 2^-40 times its original diagonal entry
 * (Sigma not positive definite, or singular to working precision, as with a
 * duplicated location); MVG_ERR_* (< -100) = runtime failure (allocation, launch).  No
 * call aborts or prints; mvg_last_error() returns the message of the last
 * failure on the calling thread.
 */
#ifndef MVGEO_H
#define MVGEO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MVG_ERR_ALLOC   (-101)
#define MVG_ERR_LAUNCH  (-102)
#define MVG_ERR_STATE   (-103)
#define MVG_ERR_LIMIT   (-104)

/* theta in the paper's order (Section 4.2): marginal variances sigma11^2 and
 * sigma22^2, shared spatial range a, smoothnesses nu11 and nu22, and the latent
 * colocated correlation beta (|beta| < 1 for p = 2).  Admissible values:
 * sigma_ii^2 > 0, a > 0, 0 < nu_ii <= 5, |beta| < 1. */
typedef struct {
    double sigma11_sq, sigma22_sq, a, nu11, nu22, beta;
} mvg_theta;

/* Arithmetic of the factorisation. */
enum {
    MVG_FP64 = 0,        /* exact dense FP64 (Section 5.2)                          */
    MVG_MIXED_FP32 = 1,  /* FP64 band tiles, FP32 off-band tiles, FP64 refinement   */
    MVG_MIXED_BF16 = 2,  /* FP64 band, off-band GEMMs on BF16 operands, FP32 accum. */
    MVG_TLR = 3,         /* tile low-rank, FP64 (Section 5.3)                       */
    MVG_DST = 4,         /* Diagonal Super Tile (Section 4.4, Experiment 2 of 6.4): */
                         /* exact FP64 with the tiles |I - J| >= band_tiles set to 0 */
    MVG_MIXED_FP32X = 5, /* FP64 tiles and panel solves; off-band trailing GEMMs on  */
                         /* FP32 MFMA (operands rounded to FP32), FP64 refinement   */
    MVG_MIXED_BF16X3 = 6 /* as MVG_MIXED_FP32X, the off-band operands split into two */
                         /* BF16 terms, three BF16 MFMAs per product, FP32 accum.   */
};

typedef struct {
    int precision;      /* MVG_FP64 / MVG_MIXED_* / MVG_TLR / MVG_DST                  */
    int nb;             /* tile size; dense and mixed: 128, 256, 512, 768 or 1024    */
                        /* (0 = 512; MVG_NB_AUTO: autotuned, see mvg_autotune_nb);     */
                        /* TLR: even, >= 64 (0 = 1200)                                 */
    int band_tiles;     /* mixed: tiles with |I - J| < band_tiles stay FP64 (0 = 2);  */
                        /* DST: tiles with |I - J| < band_tiles are kept, the others */
                        /* are annihilated (0 = 2; see mvg_dst_band)                   */
    double tlr_acc;     /* TLR: absolute singular-value threshold (0 = 1e-7)          */
    int tlr_max_rank;   /* TLR: larger ranks keep the tile dense (0 = 300)            */
    uint64_t seed;      /* TLR: seed of the randomized-SVD sketch                      */
    int ir_max_iter;    /* mixed: iterative-refinement sweeps (0 = 20)                 */
    double ir_tol;      /* mixed: stop when ||r|| <= ir_tol ||Z|| (0 = 1e-14)          */
} mvg_opts;

/* DST band for a kept fraction of tiles (Experiment 2 of Section 6.4: "DST
 * 40/60" keeps 40 % of the tiles, those nearest the diagonal): with
 * T = ceil(2 n_loc / nb) tiles per side, the smallest w in [1, T] such that
 * the T x T tiles with |I - J| < w, T + (w - 1)(2T - w) of them, number at
 * least keep_fraction * T * T (compared in FP64).  Host only, no device
 * work.  Returns w, or -1 for n_loc < 1, nb < 1 or keep_fraction outside
 * (0, 1]. */
int mvg_dst_band(int64_t n_loc, int nb, double keep_fraction);

/* Library-owned device matrix: the lower tiles of Sigma (dense, mixed, TLR or DST).
 * Freed only by mvg_mat_destroy. */
typedef struct mvg_mat mvg_mat;

/* Library-owned resident factor: the Cholesky factor L of Sigma(theta), the
 * locations it was built on, theta, and w = Sigma^-1 Z.  Freed only by
 * mvg_factor_destroy.  Used by cokrige_predict. */
typedef struct mvg_factor mvg_factor;

/* Morton (Z-order) permutation of the locations (Section 5.3 orders the
 * locations this way to lower tile ranks).  Coordinates are quantised as
 * floor(v * 2^16) clamped to [0, 65535]; x bits go to the even and y bits to
 * the odd key bits; equal keys keep input order.  d_perm (n_loc int64,
 * caller-owned) receives the sorted-to-input index map; d_xs, d_ys (nullable,
 * n_loc FP64 each, caller-owned, not aliasing d_x / d_y) receive the
 * locations in Morton order.  Requires n_loc <= 2^26.  Returns 0, -1..-6 for
 * bad arguments, MVG_ERR_*. */
int morton_order(const double *d_x, const double *d_y, int64_t n_loc,
                 int64_t *d_perm, double *d_xs, double *d_ys, void *hip_stream);

/* Generate the lower tiles of Sigma(theta) (Eq. 2, Representation I) into a
 * new library-owned matrix *out.  The layout is tile-major: nb x nb tiles,
 * column-major inside a tile, lower tiles only; 2n is padded up to a multiple
 * of nb with an identity block (log-determinant and quadratic form
 * unchanged).  Mixed precision stores off-band tiles in FP32.  TLR returns
 * dense tiles (compress with tlr_compress).  DST stores the kept tiles only;
 * every annihilated tile reads as one shared zero tile.  Returns 0, -1..-7,
 * MVG_ERR_*. */
int cov_generate(const double *d_x, const double *d_y, int64_t n_loc,
                 const mvg_theta *th, const mvg_opts *o, mvg_mat **out,
                 void *hip_stream);

/* In-place tiled Cholesky Sigma = L L^T of a matrix from cov_generate
 * (POTRF / TRSM / SYRK / GEMM tile tasks, Section 5.1).  *h_info receives 0
 * or the 1-based index of the first non-positive pivot.  DST: the factor of
 * the band matrix keeps the band (L_ij = 0 for i - j >= band_tiles), so only
 * tiles within it are updated.  Returns 0 (also when *h_info > 0), -1..-3,
 * MVG_ERR_*. */
int potrf_tiled(mvg_mat *A, const mvg_opts *o, int64_t *h_info, void *hip_stream);

/* Eq. (1) for n_theta parameter vectors on one dataset:
 *   l(theta) = -n_loc log(2 pi) - 1/2 log|Sigma| - 1/2 Z^T Sigma^-1 Z.
 * d_z: 2*n_loc FP64 in Representation I.  Host outputs (n_theta each):
 * h_loglik, h_logdet, h_quad (nullable), h_status (nullable: 0 or the pivot
 * index; a failing theta gets h_loglik = -inf).  n_theta > 1 evaluates all
 * theta on the same arena (large problems) or in one persistent launch
 * (2 n_loc <= MVG_SMALL_MAX_ROWS, FP64, see loglik_many).  keep (nullable, n_theta == 1 only) receives a resident factor for
 * cokrige_predict.  Returns 0, -1..-12 for bad arguments, MVG_ERR_*.
 *
 * Mixed precision (MVG_MIXED_FP32 / MVG_MIXED_BF16 / MVG_MIXED_FP32X /
 * MVG_MIXED_BF16X3; not in the paper): Sigma is
 * generated once in FP64 and kept for the refinement; the factor has FP64
 * tiles within band_tiles of the diagonal (all diagonal factorisations FP64)
 * and FP32 tiles elsewhere, updated on FP32 (or BF16-operand) MFMA.  The solve
 * x = Sigma^-1 Z is refined in FP64 (r = Z - Sigma x with the FP64 Sigma,
 * correction from the mixed factor) until ||r|| <= ir_tol ||Z||, or
 * |x^T r| <= 1e-10 |Z^T x| (the quadratic form has converged; not used when
 * keep is set, since predictions use x itself), ir_max_iter
 * sweeps, or stagnation; h_quad = Z^T x + x^T r (the last residual's
 * first-order correction).  h_logdet is that of the mixed factor (not
 * refined).  A theta whose mixed factor meets a non-positive pivot, or whose
 * refinement stops without meeting a criterion, is evaluated again in FP64
 * (its values, status and, with keep, factor are FP64's; mvg_ir_stats marks
 * it), so h_status > 0 means that the FP64 factor failed too.
 * Memory: the FP64 lower tiles plus the mixed copy.
 * Requires band_tiles >= 2.
 * MVG_MIXED_FP32X (not in the paper) keeps every tile in FP64 and solves every
 * panel in FP64; only the trailing updates of tiles band_tiles or more
 * tile-diagonals off the diagonal take FP32 operands (rounded from the FP64
 * panel) on FP32 MFMA, with 16-product stage sums added to the FP64 tile.
 * The log-determinant then carries only the operand rounding; memory is that
 * of two FP64 copies of Sigma.
 * MVG_MIXED_BF16X3 (not in the paper) is MVG_MIXED_FP32X with the off-band
 * operands split as a = a_hi + a_lo (a_hi: BF16 rounding of the FP32 value,
 * a_lo: BF16 rounding of the remainder) and each product formed as
 * a_hi b_hi + a_hi b_lo + a_lo b_hi on BF16 MFMA with FP32 accumulation over
 * the tile's K, added to the FP64 tile once: each operand carries at most
 * 2^-17 relative error, each product about 2^-15 at most (a_lo b_lo dropped).
 *
 * DST (MVG_DST): Eq. (1) of the Diagonal Super Tile matrix (Section 4.4),
 * Sigma with the tiles |I - J| >= band_tiles set to zero, in FP64; the
 * truncated matrix need not be positive definite (then h_status > 0). */
int loglik(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
           const mvg_theta *th, int n_theta, const mvg_opts *o,
           double *h_loglik, double *h_logdet, double *h_quad, int64_t *h_status,
           mvg_factor **keep, void *hip_stream);

/* Multivariate prediction-efficiency criteria (Section 5.4, Eq. (5)-(8),
 * Algorithm 1): for m targets s0, with c0_t, c0_a the Eq. (3)-(4) cross
 * covariances under the true theta and an approximate model's estimate
 * theta_a,
 *   E_t     = tr{C(0; theta) - c0_t^T Sigma(theta)^-1 c0_t},
 *   E_a     = tr{C(0; theta_a) - c0_a^T Sigma(theta_a)^-1 c0_a},
 *   E_{t,a} = tr{C(0; theta) - 2 c0_t^T Sigma(theta_a)^-1 c0_a
 *              + c0_a^T Sigma(theta_a)^-1 Sigma(theta) Sigma(theta_a)^-1 c0_a},
 *   LOE = E_{t,a} / E_t - 1,  MOM = E_a / E_{t,a} - 1,
 * *h_mloe / *h_mmom = their means over the targets; d_loe, d_mom (nullable,
 * device, m each) receive the per-target values.  Two dense FP64 tiled
 * factorisations (o: FP64 only, nb as for cov_generate); m <= 65535.
 * Returns 0, -1..-10, 1 or 2 if Sigma(theta) or Sigma(theta_a) is not
 * positive definite, MVG_ERR_*. */
int mloe_mmom(const double *d_x, const double *d_y, int64_t n_loc, const mvg_theta *th,
              const mvg_theta *th_a, const double *d_x0, const double *d_y0, int64_t m,
              const mvg_opts *o, double *h_mloe, double *h_mmom, double *d_loe, double *d_mom,
              void *hip_stream);

/* ------------------------------------------------------------ autotuning
 *
 * Tile size picked by measurement: for each candidate nb, one untimed
 * warm-up and one timed likelihood evaluation of this very problem (theta,
 * data, precision); the fastest candidate wins.  The choice is cached in the
 * process per (n_loc, precision, band_tiles); a cached key returns at once
 * (return value 1, h_seconds untouched).  cand: n_cand tile sizes from
 * {128, 256, 512, 768, 1024} (NULL: 256, 512, 768, 1024).  h_seconds
 * (nullable): the time of each candidate (INFINITY if it failed to run).
 * Precision FP64, DST or mixed.  Returns 0 (tuned), 1 (cached), -1..-9 for
 * bad arguments, MVG_ERR_*.
 *
 * loglik with opts.nb = MVG_NB_AUTO uses the cached choice for its key,
 * tuning first (with its first theta) when the key is new. */
#define MVG_NB_AUTO (-1)
int mvg_autotune_nb(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
                    const mvg_theta *th, const mvg_opts *o, const int *cand, int n_cand,
                    int *best_nb, double *h_seconds, void *hip_stream);

/* ------------------------------------------------------------ p variables
 *
 * The parsimonious multivariate Matern of Section 4.2 for p = 1..MVG_PMAX
 * variables (the trivariate model of the application in Section 6.4.2 is
 * p = 3): Eq. (2) for i, j = 1..p with nu_ij = (nu_ii + nu_jj) / 2 and
 * rho_ij = beta_ij sqrt(nu_ii nu_jj) / nu_ij (d = 2, rho_ii = 1), in
 * Representation I: Sigma[p l + i, p r + j] = C_ij(||s_l - s_r||), Z
 * interleaved (Z_1(s_1), .., Z_p(s_1), Z_1(s_2), ..). */
#define MVG_PMAX 4

/* theta of the p-variate model.  Admissible values: 1 <= p <= MVG_PMAX,
 * sigma_sq[i] > 0, a > 0, 0 < nu[i] <= 5, beta (row-major p x p, entries
 * i, j < p only) symmetric with unit diagonal and positive definite (checked
 * by a Cholesky factorisation on the host). */
typedef struct {
    int p;
    double sigma_sq[MVG_PMAX];
    double a;
    double nu[MVG_PMAX];
    double beta[MVG_PMAX * MVG_PMAX];
} mvg_theta_p;

/* Eq. (1) for the p-variate model:
 *   l(theta) = -(p n_loc / 2) log(2 pi) - 1/2 log|Sigma| - 1/2 Z^T Sigma^-1 Z,
 * d_z: p * n_loc FP64 (interleaved as above).  Precision MVG_FP64 or MVG_DST
 * (p = 2 also takes every precision of loglik, through loglik itself, with
 * identical results).  Outputs as for loglik.  Returns 0, -1..-8 for bad
 * arguments (-5: an invalid theta; -7: bad or unsupported options for this
 * p), MVG_ERR_*. */
int loglik_p(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
             const mvg_theta_p *th, int n_theta, const mvg_opts *o, double *h_loglik,
             double *h_logdet, double *h_quad, int64_t *h_status, void *hip_stream);

/* Generate Sigma(theta) of the p-variate model into a new library-owned
 * matrix (as cov_generate; precision MVG_FP64 or MVG_DST; p = 2 takes
 * cov_generate's path).  Returns 0, -1..-7, MVG_ERR_*. */
int cov_generate_p(const double *d_x, const double *d_y, int64_t n_loc,
                   const mvg_theta_p *th, const mvg_opts *o, mvg_mat **out,
                   void *hip_stream);

/* Profile likelihood of Section 5.2: the marginal variances are replaced by
 *   sigma_ii^2 = n^-1 Z_i^T R_ii^-1 Z_i,
 * R_ii the n x n correlation matrix of variable i alone (nu_ii, a, unit
 * variance; one univariate factorisation each), then Eq. (1) is evaluated at
 * theta with those variances (th->sigma_sq is not read).  h_sigma_sq
 * receives the p estimates; the other outputs as for loglik_p (one theta).
 * A failing univariate factorisation gives *h_status = -(1 + i) for
 * variable i.  Returns 0, -1..-9, MVG_ERR_*. */
int profile_loglik_p(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
                     const mvg_theta_p *th, const mvg_opts *o, double *h_sigma_sq,
                     double *h_loglik, double *h_logdet, double *h_quad, int64_t *h_status,
                     void *hip_stream);

/* ------------------------------------------------------- maximum likelihood
 *
 * The optimiser around Eq. (1) (Section 5.1 uses NLopt for this step without
 * naming a method): derivative-free Nelder-Mead simplex search (Nelder and
 * Mead 1965; reflection 1, expansion 2, contraction 1/2, shrink 1/2).  The
 * objective is called in batches: the starting simplex (dim + 1 points) and
 * every shrink (dim points) in one call, single points otherwise. */

/* Host objective for mvg_nelder_mead: f[i] = objective at row i of V
 * (m x dim, row-major); returns 0, or a non-zero code that stops the search
 * and is returned.  NaN values count as +infinity. */
typedef int (*mvg_batch_objective)(int m, const double *V, double *f, void *ctx);

/* Minimise f from x0 (starting simplex x0 and x0 + step e_i).  Stops when
 * max f - min f <= ftol over the simplex and every vertex is within xtol of
 * the best in every coordinate (*converged = 1), or after max_evals
 * evaluations (checked between steps, so a step may finish past it).  Host
 * only: no device work.  Returns 0, -1..-9 for bad arguments (dim in 1..64,
 * max_evals >= dim + 1), or the objective's code. */
int mvg_nelder_mead(int dim, const double *x0, double step, mvg_batch_objective f, void *ctx,
                    int max_evals, double ftol, double xtol, double *x_best, double *f_best,
                    int *n_evals, int *n_iters, int *converged);

typedef struct {
    int max_evals;  /* likelihood evaluations (0 = 1000)                        */
    double ftol;    /* simplex spread of -loglik (0 = 1e-6)                      */
    double xtol;    /* simplex size in the search coordinates (0 = 1e-5)        */
    double step;    /* starting simplex step in the search coordinates (0 = 0.1) */
} mvg_mle_opts;

/* Maximum-likelihood estimate of the bivariate theta from th0 by
 * mvg_nelder_mead on -loglik (any precision of loglik), searched in
 * unconstrained coordinates: log sigma11^2, log sigma22^2, log a,
 * logit(nu_ii / 5) (so 0 < nu_ii < 5), atanh beta.  A theta whose matrix
 * is not positive definite counts as -infinity.  th_hat, h_loglik: the best
 * point found; h_evals, h_iters, h_converged (nullable).  Returns 0, -1..-8
 * for bad arguments (-5: th0 invalid or nu_ii = 5), or loglik's error
 * codes. */
int mle_fit(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
            const mvg_theta *th0, const mvg_opts *o, const mvg_mle_opts *mo,
            mvg_theta *th_hat, double *h_loglik, int *h_evals, int *h_iters,
            int *h_converged, void *hip_stream);

/* One task of loglik_many: a dataset (device pointers, caller-owned) and a
 * theta. */
typedef struct {
    const double *x, *y, *z;  /* n_loc locations, 2 n_loc values (Representation I) */
    int64_t n_loc;
    mvg_theta theta;
} mvg_task;

/* Largest 2 n_loc of a loglik_many task. */
#define MVG_SMALL_MAX_ROWS 1024

/* Eq. (1) for many small problems (2 n_loc <= MVG_SMALL_MAX_ROWS each,
 * datasets and theta may all differ) in one persistent launch: a fixed grid
 * of workgroups takes tasks from a device queue, one workgroup per task
 * (generation, FP64 Cholesky, solve, log-determinant).  A task's result does
 * not depend on the other tasks of the batch (bitwise).  loglik with
 * n_theta > 1, FP64 and 2 n_loc <= MVG_SMALL_MAX_ROWS (and no keep) takes
 * this path.  Outputs as for loglik (host, n_tasks each; h_logdet, h_quad,
 * h_status nullable).  Returns 0, -1..-3 for bad arguments, -(100 + i) for
 * task i with an invalid theta or size, MVG_ERR_*. */
int loglik_many(const mvg_task *h_tasks, int n_tasks, double *h_loglik, double *h_logdet,
                double *h_quad, int64_t *h_status, void *hip_stream);

/* Scratch of loglik_many_noalloc: a fixed device array of this many bytes,
 * held by every device the library runs on until the process ends. */
#define MVG_NOALLOC_SCRATCH_BYTES (256ull << 20)
/* Largest n_tasks of one loglik_many_noalloc call. */
#define MVG_NOALLOC_MAX_TASKS 4096

/* loglik_many without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same tasks, outputs and results
 * (bitwise) as loglik_many; the task list, per-task outputs, queue counter
 * and per-workgroup workspaces live in the library's fixed scratch array of
 * MVG_NOALLOC_SCRATCH_BYTES on the current device instead of an allocation
 * (when it holds fewer N x N workspaces than loglik_many would allocate,
 * fewer workgroups take the same tasks).  The call stages through static
 * host buffers and synchronises hip_stream before it returns.  Calls from
 * one process are serialised; calls from several processes that overlap on
 * one GPU would share its array and race (there is no cross-process lock).
 * Returns as loglik_many, and MVG_ERR_LIMIT when n_tasks exceeds
 * MVG_NOALLOC_MAX_TASKS or one workspace does not fit the scratch. */
int loglik_many_noalloc(const mvg_task *h_tasks, int n_tasks, double *h_loglik,
                        double *h_logdet, double *h_quad, int64_t *h_status,
                        void *hip_stream);

/* TLR compression (Section 5.3) of the off-diagonal tiles of Sigma(theta) by
 * randomized SVD with absolute truncation s_i > tlr_acc; tiles needing a rank
 * above tlr_max_rank stay dense.  h_ranks (nullable, T*T int32, row-major,
 * -1 = dense) receives the ranks.  Returns 0, -1..-8, MVG_ERR_*. */
int tlr_compress(const double *d_x, const double *d_y, int64_t n_loc,
                 const mvg_theta *th, const mvg_opts *o, mvg_mat **out,
                 int32_t *h_ranks, void *hip_stream);

/* Cokriging predictor Eq. (3)-(4) on a resident factor:
 *   Zhat(s0) = c0^T Sigma^-1 Z,  c0[2r+i, j] = C_ij(||s0 - s_r||).
 * d_x0, d_y0: m targets (device).  d_zhat: 2m FP64, (Zhat_1, Zhat_2) per
 * target.  d_mse (nullable): m FP64 predictor MSE tr{C(0) - c0^T Sigma^-1 c0}
 * (Eq. 5).  Returns 0, -1..-7, MVG_ERR_*. */
int cokrige_predict(const mvg_factor *F, const double *d_x0, const double *d_y0,
                    int64_t m, double *d_zhat, double *d_mse, void *hip_stream);

/* d_z <- L d_eps for a factored dense matrix (lower factor L of Sigma):
 * draws Z ~ N(0, Sigma) from a standard-normal d_eps (2n FP64, device), the
 * data generator of the paper's synthetic experiments (Section 6.4).
 * Returns 0, -1..-3, MVG_ERR_*. */
int mvg_trmv(const mvg_mat *L, const double *d_eps, double *d_z, void *hip_stream);

/* Eq. (1) from a factored FP64 matrix (potrf_tiled): log|Sigma| = 2 sum
 * log L_jj and Z^T Sigma^-1 Z = ||L^-1 Z||^2 with the same kernels as
 * loglik, for a Z (device, p n_loc values) given after the factorisation
 * (for instance Z = L eps from mvg_trmv on the same factor).  h_logdet and
 * h_quad nullable.  Returns 0, -1 (not a factored FP64 matrix), -2, -3,
 * MVG_ERR_*. */
int mvg_mat_loglik(const mvg_mat *L, const double *d_z, double *h_loglik, double *h_logdet,
                   double *h_quad, void *hip_stream);

/* HBM bytes the library allocates for one likelihood evaluation of n_loc
 * locations with these options (matrix + workspaces), for admission control. */
size_t mvg_footprint(int64_t n_loc, const mvg_opts *o);

/* Number of variables p of a matrix (its order is p n_loc), or -1. */
int mvg_mat_nvar(const mvg_mat *A);

/* Shape of a matrix: n_loc, tile size, tile count per side, precision,
 * factored flag.  Any output pointer may be NULL. */
int mvg_mat_shape(const mvg_mat *A, int64_t *n_loc, int *nb, int *ntiles,
                  int *precision, int *factored);

/* Gather m entries (row[t], col[t]), 0-based, row >= col, of the stored lower
 * triangle (Sigma before potrf_tiled, L after) into d_out.  Dense and mixed
 * matrices only.  Returns 0, -1..-5, MVG_ERR_*. */
int mvg_mat_gather(const mvg_mat *A, const int64_t *d_rows, const int64_t *d_cols,
                   int64_t m, double *d_out, void *hip_stream);

/* Expand the lower triangle into a dense column-major 2n x 2n buffer d_out
 * (leading dimension ld >= 2n); the strict upper triangle is set to 0.
 * TLR tiles are expanded as U V^T.  Returns 0, -1..-3, MVG_ERR_*. */
int mvg_mat_to_dense(const mvg_mat *A, double *d_out, int64_t ld, void *hip_stream);

/* Resident factor accessors: the underlying matrix (factored), n_loc, and
 * w = Sigma^-1 Z (device pointer owned by the factor). */
const mvg_mat *mvg_factor_mat(const mvg_factor *F);
const double *mvg_factor_w(const mvg_factor *F);

void mvg_mat_destroy(mvg_mat *A);
void mvg_factor_destroy(mvg_factor *F);

/* ------------------------------------------------------------------ serving
 *
 * A request server over registered datasets (not in the paper): likelihood
 * and cokriging requests of uneven size are admitted by HBM footprint
 * (mvg_footprint) against a byte budget and run concurrently on n_workers
 * streams; small FP64 likelihoods waiting together are evaluated in one
 * persistent launch (loglik_many); factors stay resident in an LRU cache
 * keyed by (dataset, theta) and serve later cokriging requests (a miss
 * factors first).  Results (mvg_result) carry the server-clock arrival,
 * start and end times.  Datasets and cokriging buffers are caller-owned
 * device memory that must outlive the requests using them.  Calls are
 * thread-safe. */
enum { MVG_REQ_LOGLIK = 0, MVG_REQ_COKRIGE = 1 };

typedef struct {
    int64_t id;
    int kind;            /* MVG_REQ_* */
    int status;          /* 0, the pivot index, or an MVG_ERR_* / argument code */
    int64_t n_loc;
    double loglik, logdet, quad;   /* likelihood requests and cokriging misses */
    double t_arrive, t_start, t_end;  /* seconds on the server clock */
    int batch;           /* requests evaluated in the same launch */
    int cache_hit;       /* cokriging: 1 if the factor was resident */
    int precision;
} mvg_result;

typedef struct mvg_server mvg_server;

/* NULL on bad arguments (budget 0, n_workers outside 1..32). */
mvg_server *mvg_server_create(size_t hbm_budget, int n_workers, const mvg_opts *o);
/* Returns the dataset id (>= 0) or -1..-3. */
int mvg_server_add_dataset(mvg_server *S, const double *d_x, const double *d_y,
                           const double *d_z, int64_t n_loc);
/* Queues a request; t_arrive < 0 means now.  cokriging: m targets d_x0,
 * d_y0, predictions into d_zhat (2m).  Returns the request id or -1..-4. */
int64_t mvg_server_submit(mvg_server *S, int kind, int dataset, const mvg_theta *th,
                          const double *d_x0, const double *d_y0, int64_t m, double *d_zhat,
                          double t_arrive);
/* Moves up to max finished results into out, waiting up to wait_ms for the
 * first one; returns their number. */
int mvg_server_poll(mvg_server *S, mvg_result *out, int max, int wait_ms);
double mvg_server_clock(const mvg_server *S);
int mvg_server_stats(mvg_server *S, int64_t *hits, int64_t *misses, int64_t *batches,
                     size_t *cached_bytes);
/* Finishes the queued requests, then frees the server and its cache. */
void mvg_server_destroy(mvg_server *S);

/* Diagnostics: timing of kernel launches with HIP events recorded on the
 * stream each launch is enqueued on.  mvg_prof_enable(1) clears the records
 * and starts recording, mvg_prof_enable(0) stops.  mvg_prof_read sums the
 * records of one kind: MVG_PROF_TRAILING (the trailing-update GEMM kernel,
 * the FLOP sink of the factorisation; in the TLR factorisation its update
 * GEMM), MVG_PROF_SYRK (the look-ahead SYRK of the next diagonal tile), MVG_PROF_GEN (covariance
 * generation), MVG_PROF_POTRF (whole factorisation), MVG_PROF_SOLVE (solve and
 * reductions), MVG_PROF_COKRIGE, MVG_PROF_LOWP (the FP32/BF16 off-band
 * update of the mixed-precision factorisation), MVG_PROF_IR (iterative
 * refinement of the mixed-precision solve), MVG_PROF_TLRGEMM (every
 * batched-GEMM launch of the TLR compression and factorisation, flops
 * 2 M N K summed over its products), MVG_PROF_QR (the Householder QR launch
 * groups of the TLR compression: the sketch QR, and the truncating pivoted
 * QR; flops 4 m n^2 - 4 n^3 / 3 per unpivoted QR with its Q).  *flops and
 * *bytes are algorithmic counts (useful work, no padding).  Synchronises the
 * device. */
enum { MVG_PROF_TRAILING = 0, MVG_PROF_GEN = 1, MVG_PROF_POTRF = 2, MVG_PROF_SOLVE = 3,
       MVG_PROF_COKRIGE = 4, MVG_PROF_LOWP = 5, MVG_PROF_IR = 6, MVG_PROF_SYRK = 7,
       MVG_PROF_TLRGEMM = 8, MVG_PROF_QR = 9, MVG_PROF_NKINDS = 10 };
int mvg_prof_enable(int on);
int mvg_prof_read(int kind, int64_t *launches, double *total_ms, double *flops, double *bytes);

/* Iterative refinement of the last mixed-precision loglik call on the
 * calling thread, theta index i: *iters = correction sweeps applied,
 * *relres = final ||Z - Sigma x|| / ||Z||, *converged = 1 if a stopping
 * criterion (residual or quadratic form) was met, -1 if the refinement
 * stopped without meeting one (sweep budget or stagnation) or the mixed
 * factor met a non-positive pivot (then *iters = 0 and *relres is NaN):
 * loglik then evaluated that theta again in FP64 and returned the FP64
 * values and status (and, with keep, the FP64 factor).
 * Returns 0, or -1 if there is no such record. */
int mvg_ir_stats(int i, int *iters, double *relres, int *converged);

/* Message of the last failure on the calling thread ("" if none). */
const char *mvg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MVGEO_H */
