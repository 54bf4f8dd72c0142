// Dense FP64 tiled Cholesky factorisation, triangular solves and reductions
// on gfx950 (Section 5.1-5.2: the tile Cholesky as POTRF / TRSM / SYRK /
// GEMM tasks; log|Sigma| = 2 sum log L_jj and Z^T Sigma^-1 Z = ||L^-1 Z||^2).
//
// Storage: lower tiles of nb x nb, column-major inside a tile (ld = nb).
// Right-looking factorisation with a look-ahead of one tile column: the
// panel of column k+1 (update of that column, then its factorisation) runs on
// a second stream while the trailing update of step k runs on the caller's
// stream.  The panel itself is factored in 128-wide inner blocks: a
// single-workgroup LDS Cholesky + triangular inverse of the 128 x 128
// diagonal block, then the rows below are solved as an in-place GEMM with
// the inverse, and the rest of the panel gets a rank-128 update.  Every
// GEMM-shaped step runs on v_mfma_f64_16x16x4_f64.
#include <algorithm>

#include "mvgeo_internal.h"

namespace mvg {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ fills

__global__ void k_fill_i64(int64_t *d, int64_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = v;
}
__global__ void k_fill_f64(double *d, double v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = v;
}
int launch_fill_i64(int64_t *d, int64_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, v, n);
  return check_launch("fill_i64");
}
int launch_fill_f64(double *d, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, v, n);
  return check_launch("fill_f64");
}

__device__ __forceinline__ double *tile_ptr(TileMap M, int I, int J) {
  return reinterpret_cast<double *>(M.base + M.off[tidx(I, J, M.T)]);
}

// --------------------------------------------------------- 128x128 GEMM block
//
// C (128x128) = or -= A (128xK) * B (128xK)^T, all column-major.  C may alias
// A (in-place TRSM): every global read of A completes before the epilogue
// writes C, so neither pointer is declared restrict.  256 threads,
// 4 waves in a 2x2 grid, each wave 64x64 = 4x4 MFMA 16x16 tiles.  K is staged
// through LDS 16 at a time, double buffered.  The MFMA takes the B fragment as
// its first operand so that each lane's accumulator holds 16 consecutive rows
// of one column: lane l, element e <-> C[l%16][l/16 + 4e] of the 16x16 tile.
constexpr int KB = 16;
constexpr int GEMM_LDS = 2 * 2 * IB * KB;  // doubles

template <bool SUB>
__device__ __forceinline__ void gemm_block(double *C, int ldc, const double *A, int lda,
                                           const double *__restrict__ B, int ldb, int K,
                                           double *__restrict__ smem) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  // LDS: buffer b holds the A slice at smem + b*2*IB*KB and the B slice after it

  dbl4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  // global -> register staging: thread loads column kk = tid/16, rows (tid%16)*8 .. +8
  const int kk = tid >> 4, r8 = (tid & 15) * 8;
  const double *ga = A + (int64_t)kk * lda + r8;
  const double *gb = B + (int64_t)kk * ldb + r8;
  double *la = smem + kk * IB + r8;
  double *lb = smem + IB * KB + kk * IB + r8;
  const int64_t stepa = (int64_t)KB * lda, stepb = (int64_t)KB * ldb;
  double2 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define MVG_GLOAD(pa, pb)                                               \
  do {                                                                  \
    const double2 *qa_ = reinterpret_cast<const double2 *>(pa);         \
    const double2 *qb_ = reinterpret_cast<const double2 *>(pb);         \
    ra0 = qa_[0]; ra1 = qa_[1]; ra2 = qa_[2]; ra3 = qa_[3];             \
    rb0 = qb_[0]; rb1 = qb_[1]; rb2 = qb_[2]; rb3 = qb_[3];             \
  } while (0)
#define MVG_SSTORE(off)                                                 \
  do {                                                                  \
    double2 *sa_ = reinterpret_cast<double2 *>(la + (off));             \
    double2 *sb_ = reinterpret_cast<double2 *>(lb + (off));             \
    sa_[0] = ra0; sa_[1] = ra1; sa_[2] = ra2; sa_[3] = ra3;             \
    sb_[0] = rb0; sb_[1] = rb1; sb_[2] = rb2; sb_[3] = rb3;             \
  } while (0)

  const int nk = K / KB;
  MVG_GLOAD(ga, gb);
  MVG_SSTORE(0);
  __syncthreads();
  const int l16 = lane & 15, lk = lane >> 4;
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = kb & 1;
    const bool more = kb + 1 < nk;
    if (more) MVG_GLOAD(ga + (kb + 1) * stepa, gb + (kb + 1) * stepb);
    const double *a = smem + buf * 2 * IB * KB + wr * 64 + l16;
    const double *b = smem + buf * 2 * IB * KB + IB * KB + wc * 64 + l16;
#pragma unroll
    for (int ks = 0; ks < KB; ks += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        af[t] = a[(ks + lk) * IB + t * 16];
        bf[t] = b[(ks + lk) * IB + t * 16];
      }
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[tj], af[ti], acc[ti][tj], 0, 0, 0);
    }
    if (more) MVG_SSTORE((buf ^ 1) * 2 * IB * KB);
    __syncthreads();
  }
#undef MVG_GLOAD
#undef MVG_SSTORE
  // epilogue
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wr * 64 + ti * 16 + l16;
        const int col = wc * 64 + tj * 16 + lk + 4 * e;
        double *p = C + (int64_t)col * ldc + row;
        if (SUB) *p -= acc[ti][tj][e];
        else *p = acc[ti][tj][e];
      }
}

// XCD-aware remap: blocks are dealt round-robin to the 8 XCDs; give each XCD
// a contiguous range of logical blocks so neighbouring tiles share its L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nwg_padded) {
  const int64_t per = nwg_padded >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// Trailing update of step k for tile columns j in [jlo, jhi], rows i in [j, T):
// A_ij -= L_ik L_jk^T (GEMM; SYRK on the diagonal tile, lower sub-blocks only).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_update_trailing(TileMap M, int k, int jlo, int jhi,
                                                         int64_t nwg, int64_t nwg_pad) {
  extern __shared__ double smem[];
  const int64_t lid = xcd_remap(blockIdx.x, nwg_pad);
  if (lid >= nwg) return;
  const int s = M.nb / IB, ss = s * s;
  int64_t t = lid / ss;
  const int sub = (int)(lid % ss);
  int j = jlo;
  while (t >= M.T - j) {
    t -= M.T - j;
    ++j;
  }
  const int i = j + (int)t;
  const int sr = sub % s, sc = sub / s;
  if (i == j && sr < sc) return;
  const int nb = M.nb;
  double *C = tile_ptr(M, i, j) + (int64_t)sc * IB * nb + sr * IB;
  const double *A = tile_ptr(M, i, k) + sr * IB;
  const double *B = tile_ptr(M, j, k) + sc * IB;
  gemm_block<true>(C, nb, A, nb, B, nb, nb, smem);
  (void)jhi;
}

// ------------------------------------------------------------ panel kernels
//
// The panel of tile column k (rows k nb .. Np, width nb) is factored in
// 64-wide inner blocks.  Every panel kernel is small (<= 32 KB LDS, about 100
// VGPRs per lane) so that it can be resident on a CU next to two
// trailing-update workgroups: the look-ahead panel never waits for the
// trailing GEMM to drain.
constexpr int PB = 64;
constexpr int SMALL_LDS = 2 * 2 * PB * KB;  // doubles (32 KB)

// C (64x64) = or -= A (64xK) B (64xK)^T, column-major, K % 16 == 0.  256
// threads, 4 waves in a 2x2 grid, each 32x32 = 2x2 MFMA 16x16 tiles.  C may
// alias A (in-place TRSM): all reads of A happen before the epilogue.
template <bool SUB>
__device__ __forceinline__ void gemm_block64(double *C, int ldc, const double *A, int lda,
                                             const double *__restrict__ B, int ldb, int K,
                                             double *__restrict__ smem) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int kk = tid >> 4, r4 = (tid & 15) * 4;
  const double *ga = A + (int64_t)kk * lda + r4;
  const double *gb = B + (int64_t)kk * ldb + r4;
  double *la = smem + kk * PB + r4;
  double *lb = smem + PB * KB + kk * PB + r4;
  const int64_t stepa = (int64_t)KB * lda, stepb = (int64_t)KB * ldb;
  double2 ra0, ra1, rb0, rb1;
#define MVG_GLOAD64(pa, pb)                                        \
  do {                                                             \
    const double2 *qa_ = reinterpret_cast<const double2 *>(pa);    \
    const double2 *qb_ = reinterpret_cast<const double2 *>(pb);    \
    ra0 = qa_[0]; ra1 = qa_[1]; rb0 = qb_[0]; rb1 = qb_[1];        \
  } while (0)
#define MVG_SSTORE64(off)                                          \
  do {                                                             \
    double2 *sa_ = reinterpret_cast<double2 *>(la + (off));        \
    double2 *sb_ = reinterpret_cast<double2 *>(lb + (off));        \
    sa_[0] = ra0; sa_[1] = ra1; sb_[0] = rb0; sb_[1] = rb1;        \
  } while (0)
  const int nk = K / KB;
  MVG_GLOAD64(ga, gb);
  MVG_SSTORE64(0);
  __syncthreads();
  const int l16 = lane & 15, lk = lane >> 4;
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = kb & 1;
    const bool more = kb + 1 < nk;
    if (more) MVG_GLOAD64(ga + (kb + 1) * stepa, gb + (kb + 1) * stepb);
    const double *a = smem + buf * 2 * PB * KB + wr * 32 + l16;
    const double *b = smem + buf * 2 * PB * KB + PB * KB + wc * 32 + l16;
#pragma unroll
    for (int ks = 0; ks < KB; ks += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        af[t] = a[(ks + lk) * PB + t * 16];
        bf[t] = b[(ks + lk) * PB + t * 16];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[tj], af[ti], acc[ti][tj], 0, 0, 0);
    }
    if (more) MVG_SSTORE64((buf ^ 1) * 2 * PB * KB);
    __syncthreads();
  }
#undef MVG_GLOAD64
#undef MVG_SSTORE64
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wr * 32 + ti * 16 + l16;
        const int col = wc * 32 + tj * 16 + lk + 4 * e;
        double *p = C + (int64_t)col * ldc + row;
        if (SUB) *p -= acc[ti][tj][e];
        else *p = acc[ti][tj][e];
      }
}

// Cholesky of the 64 x 64 diagonal block b of tile (k, k) and, in the same
// sweep, its inverse W = L^-1 by forward elimination on the identity.  The
// block lives in registers: thread (ty, tx) = (tid % 16, tid / 16) holds rows
// ty + 16 i and columns tx + 16 jj (i, jj < 4), of the factor and of W.  Each
// step broadcasts column j of the factor and row j of W through LDS (double
// buffered, one barrier per step).  A pivot at or below 2^-40 of its original
// diagonal entry (sigma11^2 or sigma22^2 by row parity, 1 in the padding) is a
// failure: the matrix is singular to working precision, and the sign of
// rounding noise must not decide; the first such global row (1-based) goes to
// *d_info.
__global__ __launch_bounds__(256) void k_potrf64(TileMap M, int k, int b, double *__restrict__ winv,
                                                 int64_t *__restrict__ d_info, double tol0,
                                                 double tol1, int64_t N) {
  __shared__ double scol[2][PB];
  __shared__ double srow[2][PB];
  const int tid = threadIdx.x;
  const int ty = tid & 15, tx = tid >> 4;
  const int nb = M.nb;
  double *G = tile_ptr(M, k, k) + (int64_t)b * PB * nb + b * PB;
  double a[4][4], x[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = ty + 16 * i, c = tx + 16 * jj;
      a[i][jj] = (r >= c) ? G[(int64_t)c * nb + r] : 0.0;
      x[i][jj] = (r == c) ? 1.0 : 0.0;
    }
  bool failed = false;
  const int64_t g0 = (int64_t)k * nb + (int64_t)b * PB;
  for (int j = 0; j < PB; ++j) {
    const int buf = j & 1, jq = j >> 4, jr = j & 15;
    if (tx == jr) {
#pragma unroll
      for (int i = 0; i < 4; ++i) scol[buf][ty + 16 * i] = a[i][jq];
    }
    if (ty == jr) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) srow[buf][tx + 16 * jj] = x[jq][jj];
    }
    __syncthreads();
    const double d = scol[buf][j];
    if (tid == 0 && !failed) {
      const int64_t g = g0 + j;
      const double tol = g >= N ? 0x1p-40 : ((g & 1) ? tol1 : tol0);
      if (!(d > tol) || !(d > 0.0)) {
        failed = true;
        atomicMin((unsigned long long *)d_info, (unsigned long long)(g + 1));
      }
    }
    const double ljj = sqrt(d);
    const double rinv = 1.0 / ljj;
    double lr[4], lc[4], xr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = ty + 16 * i;
      lr[i] = (r > j) ? scol[buf][r] * rinv : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int c = tx + 16 * jj;
      lc[jj] = (c > j) ? scol[buf][c] * rinv : 0.0;
      xr[jj] = srow[buf][c] * rinv;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        a[i][jj] -= lr[i] * lc[jj];
        x[i][jj] -= lr[i] * xr[jj];
      }
    if (tx == jr) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = ty + 16 * i;
        if (r == j) a[i][jq] = ljj;
        else if (r > j) a[i][jq] = lr[i];
      }
    }
    if (ty == jr) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) x[jq][jj] = xr[jj];
    }
  }
  double *W = winv + (int64_t)(g0 / PB) * PB * PB;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = ty + 16 * i, c = tx + 16 * jj;
      if (r >= c) G[(int64_t)c * nb + r] = a[i][jj];
      W[c * PB + r] = (r >= c) ? x[i][jj] : 0.0;
    }
}

// Panel TRSM for inner block b: 64-row blocks R in (b, nrb) of panel k:
// P[R, b] <- P[R, b] W_b^T, in place (each workgroup owns its 64 x 64 block).
__global__ __launch_bounds__(256) void k_trsm64(TileMap M, int k, int b,
                                                const double *__restrict__ W) {
  __shared__ double smem[SMALL_LDS];
  const int s = M.nb / PB;
  const int R = b + 1 + blockIdx.x;
  const int nb = M.nb;
  const int i = k + R / s, rl = R % s;
  double *C = tile_ptr(M, i, k) + (int64_t)b * PB * nb + rl * PB;
  gemm_block64<false>(C, nb, C, nb, W, PB, PB, smem);
}

// Panel update after inner block b: inner column blocks cb in (b, s), row
// blocks R >= cb: P[R, cb] -= P[R, b] P[cb, b]^T (rank-64).
__global__ __launch_bounds__(256) void k_panel_update64(TileMap M, int k, int b, int nrb) {
  __shared__ double smem[SMALL_LDS];
  const int s = M.nb / PB;
  const int ncb = s - (b + 1);
  const int R = b + 1 + blockIdx.x / ncb;
  const int cb = b + 1 + blockIdx.x % ncb;
  if (R >= nrb || R < cb) return;
  const int nb = M.nb;
  const int i = k + R / s, rl = R % s;
  double *P = tile_ptr(M, i, k);
  const double *D = tile_ptr(M, k, k);
  gemm_block64<true>(P + (int64_t)cb * PB * nb + rl * PB, nb, P + (int64_t)b * PB * nb + rl * PB, nb,
                     D + (int64_t)b * PB * nb + cb * PB, nb, PB, smem);
}

struct PivotTol {
  double t0, t1;
  int64_t N;
};

static int panel_factor(const TileMap &M, int k, double *winv, int64_t *d_info, const PivotTol &pt,
                        hipStream_t st) {
  const int s = M.nb / PB;
  const int nrb = (M.T - k) * s;  // 64-row blocks of panel k
  for (int b = 0; b < s; ++b) {
    hipLaunchKernelGGL(k_potrf64, dim3(1), dim3(256), 0, st, M, k, b, winv, d_info, pt.t0, pt.t1,
                       pt.N);
    if (int rc = check_launch("potrf64")) return rc;
    const int nbelow = nrb - (b + 1);
    if (nbelow > 0) {
      const double *W = winv + ((int64_t)k * s + b) * PB * PB;
      hipLaunchKernelGGL(k_trsm64, dim3(nbelow), dim3(256), 0, st, M, k, b, W);
      if (int rc = check_launch("trsm64")) return rc;
    }
    if (b + 1 < s) {
      const int ncb = s - (b + 1);
      hipLaunchKernelGGL(k_panel_update64, dim3(nbelow * ncb), dim3(256), 0, st, M, k, b, nrb);
      if (int rc = check_launch("panel_update64")) return rc;
    }
  }
  return 0;
}

// Useful flops of a trailing-update launch (rows past N are padding).
static double trailing_flops(int64_t N, int nb, int T, int k, int jlo, int jhi) {
  auto len = [&](int t) { return (double)std::min<int64_t>(nb, N - (int64_t)t * nb); };
  const double K = len(k);
  double f = 0.0;
  for (int j = jlo; j <= jhi; ++j) {
    const double cj = len(j);
    f += cj * (cj + 1.0) * K;  // SYRK on the diagonal tile
    for (int i = j + 1; i < T; ++i) f += 2.0 * len(i) * cj * K;
  }
  return f;
}

static int trailing(const TileMap &M, int64_t N, int k, int jlo, int jhi, hipStream_t st) {
  if (jlo > jhi || jlo >= M.T) return 0;
  const int s = M.nb / IB;
  int64_t ntile = 0;
  for (int j = jlo; j <= jhi; ++j) ntile += M.T - j;
  const int64_t nwg = ntile * s * s;
  const int64_t pad = (nwg + 7) / 8 * 8;
  // bytes: C read + written, the two panel operands read once per output tile
  const double bytes = 8.0 * (double)ntile * M.nb * M.nb * 4.0;
  int h = prof_begin(MVG_PROF_TRAILING, st, trailing_flops(N, M.nb, M.T, k, jlo, jhi), bytes);
  hipLaunchKernelGGL(k_update_trailing, dim3((unsigned)pad), dim3(256), GEMM_LDS * sizeof(double),
                     st, M, k, jlo, jhi, nwg, pad);
  prof_end(h, st);
  return check_launch("update_trailing");
}

// The trailing-update kernel uses exactly 64 KB of dynamic LDS; opt in once.
static int lds_optin() {
  static int done = 0;
  if (done) return 0;
  hipError_t e = hipFuncSetAttribute((const void *)k_update_trailing,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(GEMM_LDS * sizeof(double)));
  if (e != hipSuccess) {
    set_error("hipFuncSetAttribute (dynamic LDS) failed: %s", hipGetErrorString(e));
    return MVG_ERR_LAUNCH;
  }
  done = 1;
  return 0;
}

int dense_potrf(mvg_mat *A, int64_t *d_info, hipStream_t st) {
  if (int rc = lds_optin()) return rc;
  const TileMap M = A->map();
  const int T = M.T;
  if (!A->d_winv) {
    set_error("dense_potrf: matrix has no inverse-block store");
    return MVG_ERR_STATE;
  }
  hipStream_t side = side_stream();
  hipEvent_t evP, evR, ev0;
  hipEventCreateWithFlags(&evP, hipEventDisableTiming);
  hipEventCreateWithFlags(&evR, hipEventDisableTiming);
  hipEventCreateWithFlags(&ev0, hipEventDisableTiming);
  int rc = 0;
  const PivotTol pt{0x1p-40 * A->theta.sigma11_sq, 0x1p-40 * A->theta.sigma22_sq, A->N};
  hipEventRecord(ev0, st);
  hipStreamWaitEvent(side, ev0, 0);
  rc = panel_factor(M, 0, A->d_winv, d_info, pt, side);
  hipEventRecord(evP, side);
  for (int k = 0; k < T && !rc; ++k) {
    hipStreamWaitEvent(st, evP, 0);
    if (k + 2 < T) rc = trailing(M, A->N, k, k + 2, T - 1, st);
    hipEventRecord(evR, st);
    if (rc) break;
    if (k + 1 < T) {
      rc = trailing(M, A->N, k, k + 1, k + 1, side);
      if (!rc) rc = panel_factor(M, k + 1, A->d_winv, d_info, pt, side);
      hipEventRecord(evP, side);
      hipStreamWaitEvent(side, evR, 0);
    }
  }
  hipEventRecord(evP, side);
  hipStreamWaitEvent(st, evP, 0);
  hipEventDestroy(evP);
  hipEventDestroy(evR);
  hipEventDestroy(ev0);
  return rc;
}

// ------------------------------------------------------- triangular solves
//
// Vectors are padded to Np = T nb; nrhs right-hand sides are stored column
// after column with leading dimension ldv, blockIdx.z selects the column.
// The diagonal tiles are solved with the 64 x 64 inverses kept by the
// factorisation, so each step is a pair of small matrix-vector products.

// v_k <- L_kk^-1 v_k: for inner blocks b = 0..s-1: y_b = W_b v_b, then the
// rows of the tile below block b lose L[rows, b] y_b.  One workgroup.
__global__ __launch_bounds__(256) void k_trsv_tile_fwd(TileMap M, int k,
                                                       const double *__restrict__ winv,
                                                       double *__restrict__ V, int64_t ldv) {
  __shared__ double v[1024];
  __shared__ double part[4][PB];
  const int nb = M.nb, tid = threadIdx.x, s = nb / PB;
  const int row = tid & 63, wave = tid >> 6;
  double *vk = V + (int64_t)blockIdx.z * ldv + (int64_t)k * nb;
  const double *Lk = tile_ptr(M, k, k);
  for (int r = tid; r < nb; r += 256) v[r] = vk[r];
  __syncthreads();
  for (int b = 0; b < s; ++b) {
    const double *W = winv + ((int64_t)k * s + b) * PB * PB;
    double acc = 0.0;
#pragma unroll 4
    for (int c = wave * 16; c < wave * 16 + 16; ++c) acc += W[c * PB + row] * v[b * PB + c];
    part[wave][row] = acc;
    __syncthreads();
    if (tid < PB) v[b * PB + tid] = (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
    __syncthreads();
    for (int r = (b + 1) * PB + tid; r < nb; r += 256) {
      double t = 0.0;
      const double *col = Lk + (int64_t)(b * PB) * nb + r;
#pragma unroll 8
      for (int c = 0; c < PB; ++c) t += col[(int64_t)c * nb] * v[b * PB + c];
      v[r] -= t;
    }
    __syncthreads();
  }
  for (int r = tid; r < nb; r += 256) vk[r] = v[r];
}

// v_i -= L_ik y_k for tiles i in (k, T): 64 rows per workgroup, the four waves
// take a quarter of the columns each and are added in a fixed order.
__global__ __launch_bounds__(256) void k_gemv_fwd(TileMap M, int k, double *__restrict__ V,
                                                 int64_t ldv) {
  __shared__ double y[1024];
  __shared__ double part[4][64];
  const int nb = M.nb, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *Vc = V + (int64_t)blockIdx.z * ldv;
  const int chunks = nb / 64;
  const int i = k + 1 + blockIdx.x / chunks;
  const int r = (blockIdx.x % chunks) * 64 + lane;
  for (int c = tid; c < nb; c += 256) y[c] = Vc[(int64_t)k * nb + c];
  __syncthreads();
  const double *L = tile_ptr(M, i, k) + r;
  const int q = nb / 4;
  double s0 = 0.0, s1 = 0.0;
  for (int c = wave * q; c < wave * q + q; c += 2) {
    s0 += L[(int64_t)c * nb] * y[c];
    s1 += L[(int64_t)(c + 1) * nb] * y[c + 1];
  }
  part[wave][lane] = s0 + s1;
  __syncthreads();
  if (tid < 64)
    Vc[(int64_t)i * nb + r] -= (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
}

// v_k <- L_kk^-T v_k: inner blocks from the bottom: v_b -= L[rows below b, b]^T
// y_below, then y_b = W_b^T v_b.
__global__ __launch_bounds__(256) void k_trsv_tile_bwd(TileMap M, int k,
                                                       const double *__restrict__ winv,
                                                       double *__restrict__ V, int64_t ldv) {
  __shared__ double v[1024];
  __shared__ double part[4][PB];
  const int nb = M.nb, tid = threadIdx.x, s = nb / PB;
  const int lane = tid & 63, wave = tid >> 6;
  double *vk = V + (int64_t)blockIdx.z * ldv + (int64_t)k * nb;
  const double *Lk = tile_ptr(M, k, k);
  for (int r = tid; r < nb; r += 256) v[r] = vk[r];
  __syncthreads();
  for (int b = s - 1; b >= 0; --b) {
    // v_b[c] -= sum_{r >= (b+1)64} L[r][b64 + c] v[r]: one wave per column
    for (int c = wave; c < PB; c += 4) {
      const double *col = Lk + (int64_t)(b * PB + c) * nb;
      double t = 0.0;
      for (int r = (b + 1) * PB + lane; r < nb; r += 64) t += col[r] * v[r];
      for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
      if (lane == 0) part[0][c] = t;
    }
    __syncthreads();
    if (tid < PB) v[b * PB + tid] -= part[0][tid];
    __syncthreads();
    // y_b = W_b^T v_b: y[c] = sum_r W[r][c] v[r] (column c of W is contiguous)
    const double *W = winv + ((int64_t)k * s + b) * PB * PB;
    {
      const int c = lane;
      double acc = 0.0;
#pragma unroll 4
      for (int r = wave * 16; r < wave * 16 + 16; ++r) acc += W[c * PB + r] * v[b * PB + r];
      part[wave][c] = acc;
    }
    __syncthreads();
    if (tid < PB) v[b * PB + tid] = (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
    __syncthreads();
  }
  for (int r = tid; r < nb; r += 256) vk[r] = v[r];
}

// v_j -= L_kj^T w_k for tiles j in [0, k): 64 columns per workgroup, one wave
// per column at a time, lanes over rows.
__global__ __launch_bounds__(256) void k_gemv_bwd(TileMap M, int k, double *__restrict__ V,
                                                 int64_t ldv) {
  __shared__ double w[1024];
  const int nb = M.nb, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *Vc = V + (int64_t)blockIdx.z * ldv;
  const int cb = nb / 64;
  const int j = blockIdx.x / cb;
  const int c0 = (blockIdx.x % cb) * 64;
  for (int r = tid; r < nb; r += 256) w[r] = Vc[(int64_t)k * nb + r];
  __syncthreads();
  const double *L = tile_ptr(M, k, j);
  for (int c = c0 + wave; c < c0 + 64; c += 4) {
    const double *col = L + (int64_t)c * nb;
    double s = 0.0;
    for (int r = lane; r < nb; r += 64) s += col[r] * w[r];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) Vc[(int64_t)j * nb + c] -= s;
  }
}

static int solve_args_ok(const mvg_mat *A) {
  if (A->nb > 1024 || A->nb % PB || !A->d_winv) {
    set_error("triangular solve needs nb <= 1024, nb %% 64 == 0 and a factored matrix");
    return MVG_ERR_STATE;
  }
  return 0;
}

int trsm_forward_multi(const mvg_mat *A, double *d_V, int nrhs, hipStream_t st) {
  if (int rc = solve_args_ok(A)) return rc;
  const TileMap M = A->map();
  const int chunks = M.nb / 64;
  for (int k = 0; k < M.T; ++k) {
    hipLaunchKernelGGL(k_trsv_tile_fwd, dim3(1, 1, nrhs), dim3(256), 0, st, M, k,
                       (const double *)A->d_winv, d_V, A->Np);
    if (int rc = check_launch("trsv_tile_fwd")) return rc;
    if (k + 1 < M.T) {
      hipLaunchKernelGGL(k_gemv_fwd, dim3((M.T - k - 1) * chunks, 1, nrhs), dim3(256), 0, st, M, k,
                         d_V, A->Np);
      if (int rc = check_launch("gemv_fwd")) return rc;
    }
  }
  return 0;
}

int trsv_forward(const mvg_mat *A, double *d_v, hipStream_t st) {
  return trsm_forward_multi(A, d_v, 1, st);
}

int trsv_backward(const mvg_mat *A, double *d_v, hipStream_t st) {
  if (int rc = solve_args_ok(A)) return rc;
  const TileMap M = A->map();
  const int nb = M.nb;
  for (int k = M.T - 1; k >= 0; --k) {
    hipLaunchKernelGGL(k_trsv_tile_bwd, dim3(1), dim3(256), 0, st, M, k, (const double *)A->d_winv,
                       d_v, A->Np);
    if (int rc = check_launch("trsv_tile_bwd")) return rc;
    if (k > 0) {
      hipLaunchKernelGGL(k_gemv_bwd, dim3(k * (nb / 64)), dim3(256), 0, st, M, k, d_v, A->Np);
      if (int rc = check_launch("gemv_bwd")) return rc;
    }
  }
  return 0;
}

// ----------------------------------------------------------- reductions
//
// Deterministic two-stage sums: fixed-size chunks per workgroup, tree inside
// the workgroup, then one workgroup adds the partials in index order.
constexpr int RED_CHUNK = 4096;

__global__ __launch_bounds__(256) void k_logdet_quad_part(TileMap M, int64_t N,
                                                          const double *__restrict__ y,
                                                          double *__restrict__ part) {
  __shared__ double r0[256], r1[256];
  const int nb = M.nb;
  const int64_t base = (int64_t)blockIdx.x * RED_CHUNK;
  double a = 0.0, q = 0.0;
  for (int t = threadIdx.x; t < RED_CHUNK; t += 256) {
    const int64_t g = base + t;
    if (g >= N) break;
    const int kt = (int)(g / nb), r = (int)(g % nb);
    a += log(tile_ptr(M, kt, kt)[(int64_t)r * nb + r]);
    q += y[g] * y[g];
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = q;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r0[0];
    part[2 * blockIdx.x + 1] = r1[0];
  }
}

__global__ void k_reduce_pairs(const double *__restrict__ part, int n, double *__restrict__ out,
                               double scale0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double a = 0.0, q = 0.0;
    for (int i = 0; i < n; ++i) {
      a += part[2 * i];
      q += part[2 * i + 1];
    }
    out[0] = scale0 * a;
    out[1] = q;
  }
}

int logdet_quad(const mvg_mat *A, const double *d_y, double *d_part, double *d_out2,
                hipStream_t st) {
  const int nblk = (int)((A->N + RED_CHUNK - 1) / RED_CHUNK);
  hipLaunchKernelGGL(k_logdet_quad_part, dim3(nblk), dim3(256), 0, st, A->map(), A->N, d_y, d_part);
  if (int rc = check_launch("logdet_quad_part")) return rc;
  hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(64), 0, st, (const double *)d_part, nblk, d_out2,
                     2.0);
  return check_launch("reduce_pairs");
}

// sum of squares of each of ncols columns (length Np): out[c]
__global__ __launch_bounds__(256) void k_sum_sq_cols(const double *__restrict__ V, int64_t Np,
                                                     double *__restrict__ out) {
  __shared__ double r[256];
  const double *v = V + (int64_t)blockIdx.x * Np;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < Np; i += 256) s += v[i] * v[i];
  r[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) r[threadIdx.x] += r[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = r[0];
}

int launch_sum_sq_cols(const double *d_V, int64_t Np, int ncols, double *d_out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_sq_cols, dim3(ncols), dim3(256), 0, st, d_V, Np, d_out);
  return check_launch("sum_sq_cols");
}

// z = L eps: one thread per row r of tile row I, z_r = sum_{J<I} L_IJ[r,:] eps_J
// + sum_{c<=r} L_II[r,c] eps_I[c] (the diagonal tile's upper part is not read).
__global__ __launch_bounds__(256) void k_trmv(TileMap M, const double *__restrict__ eps,
                                              double *__restrict__ z, int64_t N) {
  const int nb = M.nb;
  const int chunks = (nb + 255) / 256;
  const int I = blockIdx.x / chunks;
  const int r = (blockIdx.x % chunks) * 256 + threadIdx.x;
  if (r >= nb) return;
  double s = 0.0;
  for (int J = 0; J < I; ++J) {
    const double *L = tile_ptr(M, I, J);
    const double *e = eps + (int64_t)J * nb;
    for (int c = 0; c < nb; ++c) s += L[(int64_t)c * nb + r] * e[c];
  }
  const double *L = tile_ptr(M, I, I);
  const double *e = eps + (int64_t)I * nb;
  for (int c = 0; c <= r; ++c) s += L[(int64_t)c * nb + r] * e[c];
  const int64_t g = (int64_t)I * nb + r;
  if (g < N) z[g] = s;
}

int launch_trmv(const mvg_mat *A, const double *d_eps, double *d_z, hipStream_t st) {
  // eps is read up to the padded length: stage a zero-padded copy
  double *ep = nullptr;
  if (hipMallocAsync((void **)&ep, sizeof(double) * A->Np, st) != hipSuccess) {
    hipGetLastError();
    set_error("trmv workspace allocation failed");
    return MVG_ERR_ALLOC;
  }
  int rc = launch_fill_f64(ep, 0.0, A->Np, st);
  if (!rc) {
    hipMemcpyAsync(ep, d_eps, sizeof(double) * A->N, hipMemcpyDeviceToDevice, st);
    const int chunks = (A->nb + 255) / 256;
    hipLaunchKernelGGL(k_trmv, dim3(A->T * chunks), dim3(256), 0, st, A->map(), (const double *)ep,
                       d_z, A->N);
    rc = check_launch("trmv");
  }
  hipFreeAsync(ep, st);
  return rc;
}

// ----------------------------------------------------------- inspection

__device__ __forceinline__ double load_entry(const TileMap &M, int64_t r, int64_t c) {
  const int I = (int)(r / M.nb), J = (int)(c / M.nb);
  const int64_t t = tidx(I, J, M.T);
  const int64_t e = (c % M.nb) * M.nb + (r % M.nb);
  if (M.kind && M.kind[t] == TK_F32)
    return (double)reinterpret_cast<const float *>(M.base + M.off[t])[e];
  return reinterpret_cast<const double *>(M.base + M.off[t])[e];
}

__global__ void k_gather(TileMap M, int64_t N, const int64_t *__restrict__ rows,
                         const int64_t *__restrict__ cols, int64_t m, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int64_t r = rows[i], c = cols[i];
  // only the stored lower triangle; anything else reads as NaN
  out[i] = (r >= 0 && c >= 0 && r < N && c <= r) ? load_entry(M, r, c) : __builtin_nan("");
}

int launch_gather(const mvg_mat *A, const int64_t *rows, const int64_t *cols, int64_t m,
                  double *out, hipStream_t st) {
  if (m <= 0) return 0;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, A->map(), A->N,
                     rows, cols, m, out);
  return check_launch("gather");
}

__global__ void k_to_dense(TileMap M, int64_t N, double *__restrict__ out, int64_t ld) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= N) return;
  out[c * ld + r] = (r >= c) ? load_entry(M, r, c) : 0.0;
}

int launch_to_dense(const mvg_mat *A, double *out, int64_t ld, hipStream_t st) {
  hipLaunchKernelGGL(k_to_dense, dim3((unsigned)((A->N + 255) / 256), (unsigned)A->N), dim3(256), 0,
                     st, A->map(), A->N, out, ld);
  return check_launch("to_dense");
}

}  // namespace mvg
