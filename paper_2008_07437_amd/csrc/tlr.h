// Tile-low-rank (TLR) storage, the batched kernels it is built from, and the
// TLR compression / Cholesky / solve drivers (internal to the library).
#pragma once

#include <vector>

#include "mvgeo_internal.h"

namespace mvg {

// ------------------------------------------------------------ task lists

struct GemmTask {  // C = alpha op(A) op(B) + beta C, column-major
  const double *A, *B;
  double *C;
  int M, N, K, lda, ldb, ldc;
  int ta, tb;  // 1: transposed operand
  double alpha, beta;
  int tri;     // 1: A as stored is lower triangular (entries above its diagonal read as 0)
};

constexpr int QR_MAXM = 2048;  // rows of a QR task (tile size bound)
constexpr int QR_MAXN = 512;   // columns of a QR task (sketch width bound)
struct QrTask {
  double *A;    // m x n, overwritten by R (upper) and the reflectors (below)
  int m, n, lda;
  double *tau;  // n (nullable)
  double *Q;    // m x n (or m x rank) explicit Q (nullable)
  int ldq;
  int *piv;     // nullable: column pivoting, column order out (n)
  double tol;   // pivoting: stop when the remaining Frobenius norm <= tol
  int *rank;    // pivoting: reflectors applied (out)
  double *work; // randomized pivoting (launch_qrcp_panels): m x QRS_ROWS Gaussian,
                // then QRS_ROWS x n sample (nullable otherwise)
};


struct SketchTask {
  double *out;
  int rows, cols, ld;
  uint64_t seed, stream;
};

enum { COPY_PLAIN = 0, COPY_UPPER_TRI = 1, COPY_IDENTITY = 2, COPY_LOWER_TRI = 3, COPY_ZERO = 4 };
struct CopyTask {
  const double *src;
  double *dst;
  int rows, cols, lds, ldd;
  const int *idx;  // source column per destination column (nullable)
  int mode;
};

// d_start[t]: first block of task t (ascending); d_map (nullable): the task
// of every block, from launch_gemm_task_map, for lists longer than
// GEMM_TASKS_LDS (shorter lists are searched in LDS)
constexpr int GEMM_TASKS_LDS = 256;
// bs: output blocks of 64 x 64, 32 x 32 (tasks with M, N <= 32) or 128 x 64 (bs = 128)
int launch_gemm_batched(const GemmTask *d_tasks, const int64_t *d_start, int ntask, int64_t nblocks,
                        hipStream_t st, const int *d_map = nullptr, int bs = 64);
int launch_gemm_task_map(const int64_t *d_start, int ntask, int64_t nblocks, int *d_map,
                         hipStream_t st);
int64_t gemm_blocks(const GemmTask &t, int bs = 64);
// C (M x N) -= A (M x K) B^T (B: N x K), column-major, one large product;
// max_wg > 0 caps the workgroups (each then walks several blocks)
int launch_gemm_nt_sub(const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                       int M, int N, int K, hipStream_t st, int max_wg = 0);
int launch_qr(const QrTask *d_tasks, int ntask, int mmax, hipStream_t st);  // mmax: largest m
// unpivoted QR in panels (compact WY); tk.tau must hold (n + 8) x 8 doubles (T factors)
int launch_qr_blocked(const QrTask *d_tasks, int ntask, int mmax, hipStream_t st);
// unpivoted QR in panels of 16 over several launches (panel factor, then a
// multi-workgroup block-reflector update per panel; Q formed the same way);
// tk.tau must hold (n + 16) x 16 doubles; usable when qr_panels_ok
bool qr_panels_ok(int mmin, int mmax, int nmax);
int launch_qr_panels(const QrTask *d_tasks, int ntask, int mmax, int nmax, bool with_q,
                     hipStream_t st);
constexpr int QR_TAU_WIDTH = 16;  // T factors: (n + 16) x 16 doubles per task
// Column-pivoted QR of tall matrices stopped at a Frobenius tail (the
// k_qr pivoted form's contract: tk.piv, tk.rank, tk.tol, Q's first columns),
// with pivots chosen per panel of 16 from a Gaussian sample of the trailing
// matrix (randomized QRCP) and the factorisation done by the panel kernels.
// tk.work: m x QRS_ROWS doubles holding a standard-normal matrix (filled by
// the caller) followed by QRS_ROWS x n doubles of sample.
constexpr int QRS_ROWS = 32;
bool qrcp_panels_ok(int mmin, int mmax, int nmax);
int launch_qrcp_panels(const QrTask *d_tasks, int ntask, int mmax, int nmax, hipStream_t st);
int launch_gaussian(const SketchTask *d_tasks, int ntask, hipStream_t st);
int launch_copy_cols(const CopyTask *d_tasks, int ntask, hipStream_t st);

// ------------------------------------------------------------ TLR storage
//
// Dense diagonal tiles (nb x nb each, leading dimension nbp = nb rounded up
// to a multiple of 64 so that the dense diagonal kernels apply; the padding
// is an identity block) and, for every off-diagonal lower tile (I > J),
// either a low-rank pair (U, V), nb x r each, tile = U V^T, or a dense tile
// stored as U = tile, V = I (r = nb, reported as rank -1).
struct TlrStore {
  int T = 0, nb = 0, nbp = 0;
  int64_t N = 0;
  double *diag = nullptr;          // T * nbp * nbp
  std::vector<int> rank;           // per packed tile; diagonal entries unused
  std::vector<char> dense;         // 1: stored dense (U = tile, V = I)
  std::vector<int64_t> uoff;       // element offset of U in buf (V follows U)
  double *buf = nullptr;
  size_t cap = 0, used = 0;        // doubles
  hipStream_t reader = nullptr;    // a stream that may still read buf (drained before a growth)
  int reff(int64_t t) const { return dense[t] ? nb : rank[t]; }
  const double *U(int64_t t) const { return buf + uoff[t]; }
  const double *V(int64_t t) const { return buf + uoff[t] + (int64_t)nb * reff(t); }
};

// TLR state of a matrix: the compressed Sigma, its factor once factored, and
// device copies of the factor's offsets and effective ranks for the solves.
struct TlrState {
  TlrStore S, L;
  int64_t *d_uoff = nullptr;
  int *d_reff = nullptr;
};

int tlr_build(mvg_mat *A, const mvg_opts &o, hipStream_t st);          // Sigma -> TLR Sigma
int tlr_potrf(mvg_mat *A, const mvg_opts &o, int64_t *d_info, hipStream_t st);
int tlr_upload_meta(mvg_mat *A, hipStream_t st);
int tlr_trsm_forward(const mvg_mat *A, double *d_V, int nrhs, int64_t ldv, hipStream_t st);
int tlr_trsv_backward(const mvg_mat *A, double *d_v, hipStream_t st);
int tlr_logdet_quad(const mvg_mat *A, const double *d_y, double *d_part, double *d_out2,
                    hipStream_t st);
int tlr_to_dense(const mvg_mat *A, double *out, int64_t ld, hipStream_t st);
void tlr_state_free(TlrState *S);
void store_free(TlrStore &S);

// One pass of a TLR driver stages its host task lists to the device.  The
// lists are copied into pinned host memory (a per-thread pool of
// hipHostMalloc blocks), so the copies are asynchronous and the host can
// build the next lists while the device works (a copy from pageable memory
// would wait for the stream); release() synchronises the stream, frees the
// device copies and returns the pinned memory to the pool.
struct HostLists {
  std::vector<void *> dev;  // device buffers to free at the end
  void *stage(const void *p, size_t bytes, hipStream_t st, int *rc);
  void *scratch(size_t bytes, hipStream_t st, int *rc);  // device only, freed with the lists
  void release(hipStream_t st);
};

}  // namespace mvg
