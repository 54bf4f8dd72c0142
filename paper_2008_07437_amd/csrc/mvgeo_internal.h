// Internal declarations of the gfx950 library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "mvgeo.h"

namespace mvg {

// Inner block: GEMM workgroup tile and the panel factorisation's block width.
constexpr int IB = 128;

// ------------------------------------------------------------------ Matern
//
// Quadrature table for K_nu(x) = e^-x * int_0^inf exp(-x (cosh t - 1)) cosh(nu t) dt
// (DLMF 10.32.9), trapezoidal rule on nodes t_k = k h_j.  Level j uses step
// h_j = 0.2 / 2^j for x in (X_{j-1}, X_j], X_j = 6 * 4^j; beyond X_4 the
// covariance underflows to 0.  The three orders (nu11, nu22, nu12) share the
// exponentials.
constexpr int QLEV = 5;
constexpr int QN = 400;  // table entries (sum of the level counts, padded)
__host__ __device__ constexpr int qlev_off(int j) {
  return j == 0 ? 0 : j == 1 ? 201 : j == 2 ? 241 : j == 3 ? 289 : 341;
}
__host__ __device__ constexpr int qlev_cnt(int j) {
  return j == 0 ? 201 : j == 1 ? 40 : j == 2 ? 48 : j == 3 ? 52 : 56;
}
__host__ __device__ constexpr double qlev_h(int j) {
  return j == 0 ? 0.2 : j == 1 ? 0.1 : j == 2 ? 0.05 : j == 3 ? 0.025 : 0.0125;
}
__host__ __device__ constexpr double qlev_xmax(int j) {
  return j == 0 ? 6.0 : j == 1 ? 24.0 : j == 2 ? 96.0 : j == 3 ? 384.0 : 1536.0;
}

// Per-theta constants of Eq. (2) for the orders o = 0 (1,1), 1 (2,2), 2 (1,2).
struct MaternArgs {
  double a;
  double coef[3];   // sigma11^2, sigma22^2, rho12 sigma1 sigma2
  double nu[3];     // nu11, nu22, nu12
  double lnorm[3];  // -log(2^(nu-1) Gamma(nu))
  int closed[3];    // 0: quadrature; 1: nu = 1/2; 2: nu = 3/2; 3: nu = 5/2
  int any_quad;
};

// Validates theta and fills the constants; returns 0 or -(index of the bad entry).
int matern_setup(const mvg_theta *th, MaternArgs *out);

// The p-variate model: orders o(i, j), i <= j, packed row by row
// (o = i p - i (i - 1) / 2 + j - i); the quadrature table holds
// cosh t_k - 1 and then cosh(nu_o t_k) for every order ((1 + no) x QN).
constexpr int PMAX = MVG_PMAX;
constexpr int PORD = PMAX * (PMAX + 1) / 2;
__host__ __device__ constexpr int pord(int i, int j, int p) {
  return i * p - i * (i - 1) / 2 + (j - i);
}
struct MaternArgsP {
  int p, no;
  double a;
  double coef[PORD];   // rho_ij sigma_i sigma_j
  double nu[PORD];
  double lnorm[PORD];  // -log(2^(nu-1) Gamma(nu))
  int closed[PORD];    // as MaternArgs::closed
  int any_quad;
};
int matern_setup_p(const mvg_theta_p *th, MaternArgsP *out);
int launch_quad_table_p(const MaternArgsP &P, double *d_qtab, hipStream_t st);

// ------------------------------------------------------------------- tiles

// Packed lower tile index, tiles of a column contiguous.
__host__ __device__ inline int64_t tidx(int I, int J, int T) {
  return (int64_t)J * T - ((int64_t)J * (J - 1)) / 2 + (I - J);
}

// TK_ZERO: an annihilated DST tile; every such tile maps to one shared,
// zero-filled FP64 tile that nothing writes.
enum TileKind : int { TK_F64 = 0, TK_F32 = 1, TK_ZERO = 2 };

// Tile storage: base + off[tidx] bytes, column-major inside the tile, ld = nb.
struct TileMap {
  char *base;
  const int64_t *off;  // device array, T(T+1)/2 byte offsets
  const int *kind;     // device array, TileKind per tile (nullptr: all F64)
  int T, nb;
  int iend;            // trailing updates touch tile rows < iend (T, or the DST band end)
};

struct TlrState;

}  // namespace mvg

struct mvg_mat {
  int64_t n_loc = 0, N = 0, Np = 0;
  int nb = 0, T = 0, precision = 0, factored = 0, band = 0;
  char *arena = nullptr;          // tile storage
  size_t arena_bytes = 0;
  int64_t *d_off = nullptr;       // per-tile byte offsets
  int *d_kind = nullptr;          // per-tile kind
  int64_t *h_off = nullptr;
  int *h_kind = nullptr;
  double *d_x = nullptr, *d_y = nullptr;  // library copies of the locations
  double *d_qtab = nullptr;               // quadrature table of theta
  double *d_winv = nullptr;               // W_k = L_kk^-1 per diagonal tile (nb x nb)
  mvg_theta theta{};
  mvg_opts opts{};
  mvg::MaternArgs margs{};
  int p = 2;                      // variables; p != 2 uses theta_p / margs_p
  mvg_theta_p theta_p{};
  mvg::MaternArgsP margs_p{};
  mvg::TlrState *tlr = nullptr;   // TLR storage (precision == MVG_TLR)
  mutable hipEvent_t done = nullptr;  // after the library's last asynchronous work on it
  mvg::TileMap map() const { return mvg::TileMap{arena, d_off, d_kind, T, nb, T}; }
};

struct mvg_factor {
  mvg_mat *A = nullptr;
  double *d_w = nullptr;   // Sigma^-1 Z (padded length Np)
  double *d_y = nullptr;   // L^-1 Z
};

namespace mvg {

// Thread-local error reporting.
void set_error(const char *fmt, ...);
int check_launch(const char *what);

// ------------------------------------------------------------ launchers
// All launchers enqueue on `st` and return 0 or an MVG_ERR_* code.

int launch_quad_table(const MaternArgs &P, double *d_qtab, hipStream_t st);
int launch_cov_tiles(const MaternArgs &P, const double *d_qtab, const double *d_x,
                     const double *d_y, int64_t n_loc, TileMap M, int tile_first, int tile_count,
                     hipStream_t st);
// p-variate Sigma (p != 2 or on request) over all tiles of M
int launch_cov_tiles_p(const MaternArgsP &P, const double *d_qtab, const double *d_x,
                       const double *d_y, int64_t n_loc, TileMap M, hipStream_t st);
// c0^T w and optionally ||L^-1 c0||^2 pieces for cokriging
int launch_cokrige_dot(const MaternArgs &P, const double *d_qtab, const double *d_x,
                       const double *d_y, int64_t n_loc, const double *d_x0, const double *d_y0,
                       int64_t m, const double *d_w, double *d_part, int nchunk, hipStream_t st);
int launch_cokrige_c0(const MaternArgs &P, const double *d_qtab, const double *d_x,
                      const double *d_y, int64_t n_loc, int64_t Np, const double *d_x0,
                      const double *d_y0, int64_t m, double *d_c0, hipStream_t st);

// dense FP64 Cholesky pieces
// Pivot rule: a pivot at or below 2^-40 of the variable's variance (tol[g % p]
// for global row g) is a failure.  gbase: global row of the tile's row 0
// (-1: k nb); lreal: rows of the tile that are not padding (0: nb).
struct PivotTol {
  double tol[PMAX];
  int p;
  int64_t N;
  int64_t gbase = -1;
  int lreal = 0;
};
PivotTol pivot_tol(const mvg_mat *A);
enum { TRAIL_UPDATE = 0, TRAIL_TRSM = 1, TRAIL_BAND = 2 };
template <int MODE>
int launch_trail(const TileMap &M, int k, int jlo, int64_t lid0, int64_t nwg, const double *P,
                 const double *W, hipStream_t st);
int diag_factor(const TileMap &M, int k, double *winv, int64_t *d_info, const PivotTol &pt,
                hipStream_t st);
int launch_syrk_next(const mvg_mat *A, int k, hipStream_t st);
int dense_potrf(mvg_mat *A, int64_t *d_info, hipStream_t st);
int mixed_potrf(mvg_mat *A, int64_t *d_info, hipStream_t st);
int launch_symv(const mvg_mat *A, const double *d_x, double *d_y, double *d_part, hipStream_t st);
// r = z - sx and out = ||r||^2; d_part holds reduce_chunks(n) doubles
int launch_axpy_norm(const double *d_z, const double *d_sx, double *d_r, int64_t n, double *d_part,
                     double *d_out, hipStream_t st);
int launch_dot(const double *d_a, const double *d_b, int64_t n, double *d_part, double *d_out,
               hipStream_t st);
int launch_axpy(double *d_x, const double *d_d, int64_t n, hipStream_t st);  // x += d
int reduce_chunks(int64_t n);
// FP64 matrix -> mixed-layout matrix of the same shape
int launch_mat_convert(const mvg_mat *S, mvg_mat *D, hipStream_t st);
int launch_fill_i64(int64_t *d, int64_t v, int64_t n, hipStream_t st);
int launch_fill_f64(double *d, double v, int64_t n, hipStream_t st);
int trsv_forward(const mvg_mat *A, double *d_v, hipStream_t st);     // v <- L^-1 v
int trsv_backward(const mvg_mat *A, double *d_v, hipStream_t st);    // v <- L^-T v
int trsm_backward_multi(const mvg_mat *A, double *d_V, int nrhs, hipStream_t st);  // V <- L^-T V
int launch_trmm_t(const mvg_mat *A, const double *d_X, double *d_Y, int nrhs, hipStream_t st);  // Y = L^T X
int launch_dot_cols(const double *d_A, const double *d_B, int64_t Np, int ncols, double *d_out,
                    hipStream_t st);
int trsm_forward_multi(const mvg_mat *A, double *d_V, int nrhs, hipStream_t st);  // V <- L^-1 V (col-major, ld Np)
int logdet_quad(const mvg_mat *A, const double *d_y, double *d_part, double *d_out2,
                hipStream_t st);  // d_out2 = {2 sum log L_jj, y^T y}
int launch_gather(const mvg_mat *A, const int64_t *rows, const int64_t *cols, int64_t m,
                  double *out, hipStream_t st);
int launch_to_dense(const mvg_mat *A, double *out, int64_t ld, hipStream_t st);
int launch_sum_sq_cols(const double *d_V, int64_t Np, int ncols, double *d_out, hipStream_t st);

// morton
int morton_sort(const double *d_x, const double *d_y, int64_t n, int64_t *d_perm, double *d_xs,
                double *d_ys, hipStream_t st);
int launch_trmv(const mvg_mat *L, const double *d_eps, double *d_z, hipStream_t st);

// many small likelihoods in one persistent launch (one workgroup per task)
constexpr int SMALL_MAX = 1024;  // 2n bound of a task
struct SmallTask {
  const double *x, *y, *z;  // device, n locations, 2n values
  int64_t n;
  MaternArgs P;
  double t0, t1;            // pivot tolerances (2^-40 sigma_ii^2)
};
// out: 4 per task; d_ws holds one small_workspace_doubles(nmax) slot per
// workgroup, min(small_batch_workgroups(ntask), max_wg if > 0) workgroups
int launch_small_loglik(const SmallTask *d_tasks, int ntask, int64_t nmax, int *d_counter,
                        double *d_ws, double *d_out, hipStream_t st, int max_wg = 0);
// a task of the batched kernel from a dataset and theta (theta validated by the caller)
SmallTask small_task(const double *x, const double *y, const double *z, int64_t n,
                     const mvg_theta &th);
size_t small_workspace_doubles(int64_t nmax);
int small_batch_workgroups(int ntask);

// second stream of the calling thread for look-ahead (default priority)
hipStream_t side_stream();

// Library memory that outlives a call: stream-ordered allocation that is
// usable on any stream when it returns (nullptr on failure), and a
// stream-ordered free of idle memory (no device-wide wait, unlike hipFree).
// Memory from hipMallocAsync on any stream may also be released with
// dev_free once idle.
void *dev_alloc(size_t bytes);
void dev_free(void *p);
// hipMallocAsync on st; when the device is out of memory, first returns the
// memory the library keeps cached (pooled tile arenas, freed stream-ordered
// memory kept mapped) and tries once more
hipError_t malloc_async(void **p, size_t bytes, hipStream_t st);

// event timing of launches (diagnostics); handles < 0 mean "not recording"
int prof_begin(int kind, hipStream_t st, double flops, double bytes);
void prof_end(int handle, hipStream_t st);

}  // namespace mvg
