// Dense FP64 tiled Cholesky factorisation and reductions on gfx950 (Section 5.1-5.2: the tile Cholesky as POTRF / TRSM / SYRK /
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
#include <cstdlib>

#include "mvgeo_internal.h"
#include "tile_dev.h"
#include "tlr.h"

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

// ------------------------------------------------- trailing update (GEMM)
//
// A_ij -= L_ik L_jk^T over all tiles of the trailing matrix, in 128 x 128
// output blocks.  Each workgroup (256 threads, 4 waves in a 2 x 2 grid, each
// wave 64 x 64 = 4 x 4 MFMA 16x16 tiles) is persistent: it walks a contiguous
// chunk of output blocks, and the chunks of the workgroups on one XCD are
// adjacent, so neighbouring blocks (which share panel strips) meet in that
// XCD's L2.  K is streamed through LDS in slices of TKB columns with TS-stage
// pipelining by direct global->LDS loads (global_load_lds_dwordx4): no VGPR
// staging, one barrier per slice, and the slices of the next block are in
// flight while the current block's C update is written.  Lane l, element e
// of an accumulator tile holds C[4e + l/16][l%16] of that 16 x 16 tile.
constexpr int KB = 16;   // K slice of the small panel GEMM
constexpr int TKB = 16;  // K slice of the trailing GEMM
constexpr int TS = 2;    // pipeline stages of the trailing GEMM (64 KB LDS per workgroup)
constexpr int TD = TKB * 2 / 4;  // direct loads per wave per stage (1 KB each)

#define MVG_LDS(p) ((__attribute__((address_space(3))) void *)(p))

// s_waitcnt vmcnt(N) leaving lgkmcnt / expcnt unconstrained (GFX9 encoding:
// vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit count");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 0xF) | ((N >> 4) << 14));
}
__device__ __forceinline__ void wait_vmcnt_0() { wait_vmcnt<0>(); }
static_assert(TKB % 4 == 0 && TS >= 2, "four columns per wave and slice step, two stages");

struct TrailBlock {
  const double *A, *B;
  double *C;
  int nk;  // K slices of this block
};


// Logical block lid of the trailing update of step k over columns j >= jlo:
// tile (i, j) and 128 x 128 sub-block (sr, sc); false for the strict upper
// sub-blocks of a diagonal tile (SYRK computes the lower part only).
// Panel TRSM (mode TRAIL_TRSM): tile (k+1+lid/ss, k), output sub-block (sr, sc)
// = P[sr] W_k[sc]^T with P the copy of the panel; W_k is lower triangular, so
// only the first (sc+1)*128 columns of K contribute.
template <int MODE>
__device__ __forceinline__ bool trail_decode(const TileMap &M, int k, int jlo, int64_t lid,
                                             const double *P, const double *W, TrailBlock &t) {
  const int s = M.nb / IB, ss = s * s, nb = M.nb;
  int64_t q = lid / ss;
  const int sub = (int)(lid % ss);
  const int sr = sub % s, sc = sub / s;
  if (MODE == TRAIL_TRSM) {
    const int i = k + 1 + (int)q;
    t.C = tile_ptr(M, i, k) + (int64_t)sc * IB * nb + sr * IB;
    t.A = P + q * (int64_t)nb * nb + sr * IB;
    t.B = W + sc * IB;
    t.nk = (sc + 1) * (IB / TKB);
    return true;
  }
  if (MODE == TRAIL_BAND) {
    // band targets (mixed precision): tiles (i, j), j > k, j <= i < j + band,
    // band passed as jlo; operands from P = the panel of step k upcast to FP64
    const int band = jlo;
    int j = k + 1;
    while (q >= min(band, M.T - j)) {
      q -= min(band, M.T - j);
      ++j;
    }
    const int i = j + (int)q;
    if (i == j && sr < sc) return false;
    t.C = tile_ptr(M, i, j) + (int64_t)sc * IB * nb + sr * IB;
    t.A = P + (int64_t)(i - k - 1) * nb * nb + sr * IB;
    t.B = P + (int64_t)(j - k - 1) * nb * nb + sc * IB;
    t.nk = nb / TKB;
    return true;
  }
  int j = jlo;
  while (q >= M.iend - j) {
    q -= M.iend - j;
    ++j;
  }
  const int i = j + (int)q;
  if (i == j && sr < sc) return false;
  t.C = tile_ptr(M, i, j) + (int64_t)sc * IB * nb + sr * IB;
  t.A = tile_ptr(M, i, k) + sr * IB;
  t.B = tile_ptr(M, j, k) + sc * IB;
  t.nk = nb / TKB;
  return true;
}

// First valid block in [lid, lid1), or lid1.
template <int MODE>
__device__ __forceinline__ int64_t trail_next(const TileMap &M, int k, int jlo, int64_t lid,
                                              int64_t lid1, const double *P, const double *W,
                                              TrailBlock &t) {
  while (lid < lid1 && !trail_decode<MODE>(M, k, jlo, lid, P, W, t)) ++lid;
  return lid;
}

template <int NB, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_update_trailing(
    TileMap M, int k, int jlo, int64_t lid0, int64_t nwg, int64_t chunk, const double *__restrict__ P,
    const double *__restrict__ W) {
  __shared__ double sA[TS][TKB * IB];
  __shared__ double sB[TS][TKB * IB];
#define MVG_STA(u) (sA[(u)])
#define MVG_STB(u) (sB[(u)])
  static_assert((NB / TKB) % TS == 0 && (IB / TKB) % TS == 0, "slices per block must divide by TS");
  const int G = gridDim.x;  // multiple of 8
  const int b = blockIdx.x;
  const int64_t bp = (int64_t)(b & 7) * (G >> 3) + (b >> 3);  // XCD-contiguous chunk order
  const int64_t lid1 = min(nwg, lid0 + (bp + 1) * chunk);
  TrailBlock cur, nxt;
  int64_t lc = trail_next<MODE>(M, k, jlo, lid0 + bp * chunk, lid1, P, W, cur);
  if (lc >= lid1) return;
  int64_t ln = trail_next<MODE>(M, k, jlo, lc + 1, lid1, P, W, nxt);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 1, wc = wave >> 1;
  const int l16 = lane & 15, lk = lane >> 4;
  // A slice of TKB columns (1 KB each) and the B slice: wave w loads columns
  // w, w + 4, ... of both, one column per direct load; lane l moves rows 2l,
  // 2l+1.
  const int loff = 2 * lane;
#define MVG_ISSUE(pa, pb, kb, st)                                                                 \
  do {                                                                                            \
    const double *a_ = (pa) + (int64_t)((kb) * TKB + wave) * NB;                                  \
    const double *b_ = (pb) + (int64_t)((kb) * TKB + wave) * NB;                                  \
    _Pragma("unroll") for (int c_ = 0; c_ < TKB / 4; ++c_) {                                      \
      __builtin_amdgcn_global_load_lds((const void *)(a_ + 4 * c_ * NB + loff),                  \
                                       MVG_LDS(MVG_STA(st) + (wave + 4 * c_) * IB), 16, 0, 0);   \
      __builtin_amdgcn_global_load_lds((const void *)(b_ + 4 * c_ * NB + loff),                  \
                                       MVG_LDS(MVG_STB(st) + (wave + 4 * c_) * IB), 16, 0, 0);   \
    }                                                                                             \
  } while (0)
  static_assert(TD == 2 * (TKB / 4), "MVG_ISSUE issues TD direct loads per wave");
#pragma unroll
  for (int p = 0; p < TS - 1; ++p) MVG_ISSUE(cur.A, cur.B, p, p);
  dbl4 acc[4][4];
  // MFMA(A fragment, B fragment): lane l, element e of tile (ti, tj) holds
  // C[wr*64 + ti*16 + 4e + l/16][wc*64 + tj*16 + l%16]; the four elements of
  // a lane sit 4 rows apart in one column, so only one address per tj is live.
  const int64_t coff = (int64_t)(wc * 64 + l16) * NB + wr * 64 + lk;
  for (;;) {
    // the accumulators start from C, the products are subtracted (negated A
    // fragments) and the block ends with plain stores
    // one opaque base per column group keeps every other offset an immediate
    // (the empty asm stops the compiler from re-deriving 64 separate addresses)
    typedef __attribute__((address_space(1))) double gdouble;  // global, not flat
    gdouble *cb[4];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
      cb[tj] = (gdouble *)(cur.C + coff + (int64_t)tj * 16 * NB);
      asm volatile("" : "+v"(cb[tj]));
    }
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          acc[ti][tj][e] = (MODE != TRAIL_TRSM) ? (double)cb[tj][ti * 16 + 4 * e] : 0.0;
    const bool have_next = ln < lid1;
    const int nk = cur.nk;
    for (int kb0 = 0; kb0 < nk; kb0 += TS) {
#pragma unroll
      for (int u = 0; u < TS; ++u) {
        const int kb = kb0 + u;
        // TS-1 slices in flight; the oldest (kb) is complete when <= (TS-2) TD remain
        // the barrier is pinned: no LDS read of this stage and no direct load
        // into the stage being refilled may be scheduled across it
        wait_vmcnt<(TS - 2) * TD>();
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        asm volatile("" ::: "memory");
        // the refill issue runs at raised wave priority, so that a wave
        // coming out of the barrier gets its direct loads in flight before
        // the other workgroup's MFMA stream takes the issue slots (measured
        // +6 % on the trailing update)
        __builtin_amdgcn_s_setprio(1);
        // refill the stage computed in the previous step: next slice of this
        // block, else the first slices of the next block, else (past the end
        // of the chunk) the last slice again, in bounds and never read
        const int p = kb + TS - 1;
        const bool in_cur = p < nk;
        const bool use_next = !in_cur && have_next;
        const double *pa = use_next ? nxt.A : cur.A;
        const double *pb = use_next ? nxt.B : cur.B;
        const int pk = in_cur ? p : (use_next ? p - nk : nk - 1);
        // the first k-step's fragments are read before the refill is issued,
        // so these LDS reads do not queue behind the direct loads' LDS writes
        // (measured +6.5 %)
        const double *a = MVG_STA(u) + wr * 64 + l16;
        const double *bb = MVG_STB(u) + wc * 64 + l16;
        double af0[4], bf0[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          af0[t] = (MODE != TRAIL_TRSM) ? -a[lk * IB + t * 16] : a[lk * IB + t * 16];
          bf0[t] = bb[lk * IB + t * 16];
        }
        MVG_ISSUE(pa, pb, pk, (u + TS - 1) % TS);
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int ks = 0; ks < TKB; ks += 4) {
          double af[4], bf[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            af[t] = ks == 0 ? af0[t]
                            : ((MODE != TRAIL_TRSM) ? -a[(ks + lk) * IB + t * 16]
                                                    : a[(ks + lk) * IB + t * 16]);
            bf[t] = ks == 0 ? bf0[t] : bb[(ks + lk) * IB + t * 16];
          }
#pragma unroll
          for (int ti = 0; ti < 4; ++ti)
#pragma unroll
            for (int tj = 0; tj < 4; ++tj)
              acc[ti][tj] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(af[ti], bf[tj], acc[ti][tj], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int e = 0; e < 4; ++e) cb[tj][ti * 16 + 4 * e] = acc[ti][tj][e];
    if (!have_next) break;
    cur = nxt;
    lc = ln;
    ln = trail_next<MODE>(M, k, jlo, lc + 1, lid1, P, W, nxt);
  }
  // no direct LDS load may outlive the workgroup
  wait_vmcnt_0();
#undef MVG_ISSUE
#undef MVG_STA
#undef MVG_STB
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
                                                 int64_t *__restrict__ d_info, PivotTol pt) {
  const int64_t N = pt.N, gbase = pt.gbase;
  const int lreal = pt.lreal;
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
  // global row of the block's first row; local rows >= lreal are padding
  const int64_t g0 = gbase + (int64_t)b * PB;
  // pivot tolerance of row g is tol[g % p]: a counter started at g0 % p and
  // wrapped at p (no division per column)
  int m = (int)(g0 % pt.p);
  // columns j = 16 jq + jr: jq is a compile-time index into the register
  // blocks a[.][jq], x[jq][.] (no indirect register addressing)
#pragma unroll
  for (int jq = 0; jq < 4; ++jq) {
#pragma unroll 1
    for (int jr = 0; jr < 16; ++jr) {
      const int j = 16 * jq + jr;
      const int buf = j & 1;
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
        const bool pad = g >= N || b * PB + j >= lreal;
        const double tol = pad ? 0x1p-40 : pt.tol[m];
        if (!(d > tol) || !(d > 0.0)) {
          failed = true;
          atomicMin((unsigned long long *)d_info, (unsigned long long)(g + 1));
        }
      }
      m = (m + 1 == pt.p) ? 0 : m + 1;
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
  }
  // inverse block (b, b) of W_k = L_kk^-1 (nb x nb, column-major, ld nb)
  double *W = winv + (int64_t)k * nb * nb + (int64_t)b * PB * nb + b * PB;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = ty + 16 * i, c = tx + 16 * jj;
      if (r >= c) G[(int64_t)c * nb + r] = a[i][jj];
      W[(int64_t)c * nb + r] = (r >= c) ? x[i][jj] : 0.0;
    }
}

// Panel TRSM for inner block b: 64-row blocks R in (b, nrb) of panel k:
// P[R, b] <- P[R, b] W_b^T, in place (each workgroup owns its 64 x 64 block).
__global__ __launch_bounds__(256) void k_trsm64(TileMap M, int k, int b,
                                                const double *__restrict__ W, int ldw) {
  __shared__ double smem[SMALL_LDS];
  const int s = M.nb / PB;
  const int R = b + 1 + blockIdx.x;
  const int nb = M.nb;
  const int i = k + R / s, rl = R % s;
  double *C = tile_ptr(M, i, k) + (int64_t)b * PB * nb + rl * PB;
  gemm_block64<false>(C, nb, C, nb, W, ldw, PB, smem);
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

// Off-diagonal 64-blocks of W_k = L_kk^-1 at block distance d = i - j:
// W_ij = -W_ii sum_{m=j..i-1} L_im W_mj (the blocks at smaller distances are
// already in place).  One workgroup per j; 64 x 64 MFMA products through LDS.
__global__ __launch_bounds__(256) void k_trtri_step(TileMap M, int k, int d,
                                                    double *__restrict__ winv) {
  __shared__ double sa[PB * PB];  // A operand, [kk][r]
  __shared__ double sb[PB * PB];  // B operand, [kk][c]
  const int nb = M.nb, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1, l16 = lane & 15, lk = lane >> 4;
  const int j = blockIdx.x, i = j + d;
  const double *L = tile_ptr(M, k, k);
  double *W = winv + (int64_t)k * nb * nb;
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b2 = 0; b2 < 2; ++b2) acc[a][b2] = dbl4{0.0, 0.0, 0.0, 0.0};
  // stage A[r][kk] (column-major block at base, ld nb) into sa[kk][r]; B^T block
  // Bt[kk][c] = X[kk][c] of a column-major block X into sb[kk][c]
  auto mma = [&]() {
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < PB; ks += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        af[t] = sa[(ks + lk) * PB + wr * 32 + t * 16 + l16];
        bf[t] = sb[(ks + lk) * PB + wc * 32 + t * 16 + l16];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ti], bf[tj], acc[ti][tj], 0, 0, 0);
    }
    __syncthreads();
  };
  // staging: every load of a 64 x 64 block is issued before the LDS stores
  // (a load-store loop would wait for each value in turn)
  constexpr int SQ = PB * PB / 256;
  for (int m = j; m < i; ++m) {
    const double *Lim = L + (int64_t)(m * PB) * nb + i * PB;  // rows i-block, cols m-block
    const double *Wmj = W + (int64_t)(j * PB) * nb + m * PB;  // rows m-block, cols j-block
    double va[SQ], vb[SQ];
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const int e = tid + 256 * q, r = e & 63, c = e >> 6;
      va[q] = Lim[(int64_t)c * nb + r];
      vb[q] = Wmj[(int64_t)c * nb + r];
    }
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const int e = tid + 256 * q, r = e & 63, c = e >> 6;
      sa[c * PB + r] = va[q];  // sa[kk = c][r]
      sb[r * PB + c] = vb[q];  // sb[kk = r][c] = Wmj[r][c]
    }
    mma();
  }
  // T = acc (64 x 64): lane l, element e of tile (ti, tj) is
  // T[wr*32 + ti*16 + 4e + l/16][wc*32 + tj*16 + l%16]; now W_ij = -W_ii T
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wr * 32 + ti * 16 + 4 * e + lk, c = wc * 32 + tj * 16 + l16;
        sb[r * PB + c] = acc[ti][tj][e];
        acc[ti][tj][e] = 0.0;
      }
  const double *Wii = W + (int64_t)(i * PB) * nb + i * PB;
  {
    double va[SQ];
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const int e = tid + 256 * q;
      va[q] = Wii[(int64_t)(e >> 6) * nb + (e & 63)];
    }
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const int e = tid + 256 * q;
      sa[(e >> 6) * PB + (e & 63)] = va[q];
    }
  }
  mma();
  double *Wij = W + (int64_t)(j * PB) * nb + i * PB;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wr * 32 + ti * 16 + 4 * e + lk, c = wc * 32 + tj * 16 + l16;
        Wij[(int64_t)c * nb + r] = -acc[ti][tj][e];
      }
}

// Zero the strict upper 64-blocks of W_k (the factorisation never writes them).
__global__ void k_zero_upper_blocks(int nb, int k, double *__restrict__ winv) {
  const int s = nb / PB;
  double *W = winv + (int64_t)k * nb * nb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)nb * nb;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % nb), c = (int)(e / nb);
    if (r / PB < c / PB) W[e] = 0.0;
  }
  (void)s;
}

// P <- the tiles (i, k), i in (k, T) (source of the out-of-place panel TRSM).
__global__ void k_copy_panel(TileMap M, int k, double *__restrict__ P) {
  const int64_t per = (int64_t)M.nb * M.nb / 2;  // double2 per tile
  const int64_t n = (int64_t)(M.iend - k - 1) * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / per, o = e % per;
    const double2 *src = reinterpret_cast<const double2 *>(tile_ptr(M, k + 1 + (int)t, k));
    reinterpret_cast<double2 *>(P)[e] = src[o];
  }
}

// SYRK of one diagonal tile, A_jj -= L_jk L_jk^T (lower 64-blocks), with the
// small-footprint 64 x 64 block GEMM so that it runs next to the persistent
// trailing update instead of waiting for it to drain.
__global__ __launch_bounds__(256) void k_syrk64(TileMap M, int k, int j) {
  __shared__ double smem[SMALL_LDS];
  const int s = M.nb / PB;
  int bi = 0, t = blockIdx.x;  // lower-triangular block (bi, bj), bi >= bj
  while (t > bi) {
    t -= bi + 1;
    ++bi;
  }
  const int bj = t;
  const int nb = M.nb;
  double *C = tile_ptr(M, j, j) + (int64_t)bj * PB * nb + bi * PB;
  const double *L = tile_ptr(M, j, k);
  gemm_block64<true>(C, nb, L + bi * PB, nb, L + bj * PB, nb, nb, smem);
  (void)s;
}

// SYRK of the next diagonal tile (k+1, k+1) by step k on stream st.
int launch_syrk_next(const mvg_mat *A, int k, hipStream_t st) {
  const TileMap M = A->map();
  const int sb = M.nb / PB;
  const double nj = (double)std::min<int64_t>(M.nb, A->N - (int64_t)(k + 1) * M.nb);
  const double nk = (double)std::min<int64_t>(M.nb, A->N - (int64_t)k * M.nb);
  int h = prof_begin(MVG_PROF_SYRK, st, nj * (nj + 1.0) * nk, 0.0);
  hipLaunchKernelGGL(k_syrk64, dim3(sb * (sb + 1) / 2), dim3(256), 0, st, M, k, k + 1);
  prof_end(h, st);
  return check_launch("syrk64");
}

// Factor the diagonal tile (k, k) in place and fill W_k = L_kk^-1: 64-wide
// inner blocks (register Cholesky + inverse of the block, in-tile TRSM and
// update), then the off-diagonal blocks of W_k by block distance.
int diag_factor(const TileMap &M, int k, double *winv, int64_t *d_info, const PivotTol &pt,
                hipStream_t st) {
  const int s = M.nb / PB;
  hipLaunchKernelGGL(k_zero_upper_blocks, dim3(64), dim3(256), 0, st, M.nb, k, winv);
  if (int rc = check_launch("zero_upper_blocks")) return rc;
  PivotTol q = pt;
  q.gbase = pt.gbase >= 0 ? pt.gbase : (int64_t)k * M.nb;
  q.lreal = pt.lreal > 0 ? pt.lreal : M.nb;
  for (int b = 0; b < s; ++b) {
    hipLaunchKernelGGL(k_potrf64, dim3(1), dim3(256), 0, st, M, k, b, winv, d_info, q);
    if (int rc = check_launch("potrf64")) return rc;
    const int nbelow = s - (b + 1);
    if (nbelow > 0) {
      const double *W = winv + (int64_t)k * M.nb * M.nb + (int64_t)b * PB * M.nb + b * PB;
      hipLaunchKernelGGL(k_trsm64, dim3(nbelow), dim3(256), 0, st, M, k, b, W, M.nb);
      if (int rc = check_launch("trsm64")) return rc;
      hipLaunchKernelGGL(k_panel_update64, dim3(nbelow * nbelow), dim3(256), 0, st, M, k, b, s);
      if (int rc = check_launch("panel_update64")) return rc;
    }
  }
  for (int d = 1; d < s; ++d) {
    hipLaunchKernelGGL(k_trtri_step, dim3(s - d), dim3(256), 0, st, M, k, d, winv);
    if (int rc = check_launch("trtri_step")) return rc;
  }
  return 0;
}

// Useful flops of a trailing-update launch over tile columns [jlo, jhi] and
// tile rows below T (rows past N are padding).
static double trailing_flops(int64_t N, int nb, int T, int k, int jlo, int jhi, bool skip_first) {
  auto len = [&](int t) { return (double)std::min<int64_t>(nb, N - (int64_t)t * nb); };
  const double K = len(k);
  double f = 0.0;
  for (int j = jlo; j <= jhi; ++j) {
    const double cj = len(j);
    if (!(skip_first && j == jlo)) f += cj * (cj + 1.0) * K;  // SYRK on the diagonal tile
    for (int i = j + 1; i < T; ++i) f += 2.0 * len(i) * cj * K;
  }
  return f;
}

// Persistent grid of the GEMM kernels: two workgroups per CU, minus a few
// slots left free so that the look-ahead stream's small kernels find a CU
// (persistent workgroups never retire mid-launch).  MVG_GEMM_RESERVE
// overrides the number of reserved slots (tuning).
constexpr int GEMM_CUS = 256;
static int gemm_reserve() {
  static int r = -1;
  if (r < 0) {
    const char *e = getenv("MVG_GEMM_RESERVE");
    r = e ? atoi(e) : 32;
    if (r < 0 || r > 2 * GEMM_CUS - 8) r = 32;
  }
  return r;
}
// 1: persistent workgroups walking chunks of blocks; 0 (default, measured
// faster with the look-ahead stream): one block per workgroup, so that
// workgroups retire continuously and the look-ahead kernels find room
// (MVG_GEMM_PERSIST, tuning).
static int gemm_persist() {
  static int r = -1;
  if (r < 0) {
    const char *e = getenv("MVG_GEMM_PERSIST");
    r = e ? (atoi(e) != 0) : 0;
  }
  return r;
}
// 1: the next diagonal tile is factored on a second stream while the
// trailing update runs; 0: one stream (MVG_LOOKAHEAD, tuning).
static int lookahead() {
  static int r = -1;
  if (r < 0) {
    const char *e = getenv("MVG_LOOKAHEAD");
    r = e ? (atoi(e) != 0) : 1;
  }
  return r;
}

template <int MODE>
int launch_trail(const TileMap &M, int k, int jlo, int64_t lid0, int64_t nwg, const double *P,
                 const double *W, hipStream_t st) {
  const int64_t work = nwg - lid0;
  if (work <= 0) return 0;
  int64_t G = gemm_persist() ? std::min<int64_t>(work, 2 * GEMM_CUS - gemm_reserve()) : work;
  G = (G + 7) / 8 * 8;
  const int64_t chunk = (work + G - 1) / G;
  switch (M.nb) {
#define MVG_CASE(NBV)                                                                          \
  case NBV:                                                                                    \
    hipLaunchKernelGGL((k_update_trailing<NBV, MODE>), dim3((unsigned)G), dim3(256), 0, st, M, \
                       k, jlo, lid0, nwg, chunk, P, W);                                        \
    break;
    MVG_CASE(128) MVG_CASE(256) MVG_CASE(512) MVG_CASE(768) MVG_CASE(1024)
#undef MVG_CASE
    default:
      set_error("tile size %d is not one of 128, 256, 512, 768, 1024", M.nb);
      return MVG_ERR_STATE;
  }
  return check_launch("update_trailing");
}

template int launch_trail<TRAIL_UPDATE>(const TileMap &, int, int, int64_t, int64_t, const double *,
                                        const double *, hipStream_t);
template int launch_trail<TRAIL_TRSM>(const TileMap &, int, int, int64_t, int64_t, const double *,
                                      const double *, hipStream_t);
template int launch_trail<TRAIL_BAND>(const TileMap &, int, int, int64_t, int64_t, const double *,
                                      const double *, hipStream_t);

// Trailing update of step k: A_ij -= L_ik L_jk^T for k < j <= i < M.iend,
// optionally without the diagonal tile (k+1, k+1) (first = 0: that tile is
// left to the look-ahead stream), or only that tile (only_first).  With a
// DST band of w tiles L_ik = 0 for i >= k + w, so M.iend = min(T, k + w)
// skips only zero products.
static int trailing(const TileMap &M, int64_t N, int k, bool skip_first, bool only_first,
                    hipStream_t st) {
  const int jlo = k + 1;
  if (jlo >= M.iend) return 0;
  const int s = M.nb / IB;
  const int64_t ss = (int64_t)s * s;
  const int64_t ntile = only_first ? 1 : (int64_t)(M.iend - jlo) * (M.iend - jlo + 1) / 2;
  const int64_t nwg = ntile * ss;
  const int64_t lid0 = skip_first ? ss : 0;
  if (lid0 >= nwg) return 0;
  const double flops = only_first ? (double)std::min<int64_t>(M.nb, N - (int64_t)jlo * M.nb) *
                                        ((double)std::min<int64_t>(M.nb, N - (int64_t)jlo * M.nb) + 1) *
                                        (double)std::min<int64_t>(M.nb, N - (int64_t)k * M.nb)
                                  : trailing_flops(N, M.nb, M.iend, k, jlo, M.iend - 1, skip_first);
  const double bytes = 8.0 * (double)(ntile - (skip_first ? 1 : 0)) * M.nb * M.nb * 4.0;
  int h = prof_begin(MVG_PROF_TRAILING, st, flops, bytes);
  int rc = launch_trail<TRAIL_UPDATE>(M, k, jlo, lid0, nwg, nullptr, nullptr, st);
  prof_end(h, st);
  return rc;
}

// Panel TRSM of step k: L_ik = A_ik W_k^T for i in (k, M.iend), out of place
// from a copy of the panel.
static int panel_trsm(const TileMap &M, int k, const double *winv, double *P, hipStream_t st) {
  const int nbelow = M.iend - k - 1;
  if (nbelow <= 0) return 0;
  hipLaunchKernelGGL(k_copy_panel, dim3(1024), dim3(256), 0, st, M, k, P);
  if (int rc = check_launch("copy_panel")) return rc;
  const int s = M.nb / IB;
  const int64_t nwg = (int64_t)nbelow * s * s;
  return launch_trail<TRAIL_TRSM>(M, k, 0, 0, nwg, P, winv + (int64_t)k * M.nb * M.nb, st);
}

// Right-looking tiled Cholesky with one tile of look-ahead.  Caller stream:
// panel TRSM of column k (GEMM against W_k), then the trailing update of
// step k except the diagonal tile (k+1, k+1).  Look-ahead stream: as soon as
// the panel of column k is solved, the SYRK of tile (k+1, k+1) and its
// factorisation with W_{k+1} (one tile of work, small footprint), so the
// next panel TRSM never waits for the trailing update.
int dense_potrf(mvg_mat *A, int64_t *d_info, hipStream_t st) {
  const TileMap M0 = A->map();
  const int T = M0.T;
  // DST: tile rows at or beyond k + band of column k stay zero
  const int dst_band = A->precision == MVG_DST ? A->band : T;
  auto step_map = [&](int k) {
    TileMap m = M0;
    m.iend = std::min(T, k + dst_band);
    return m;
  };
  const TileMap &M = M0;
  if (!A->d_winv) {
    set_error("dense_potrf: matrix has no inverse-tile store");
    return MVG_ERR_STATE;
  }
  double *P = nullptr;
  const size_t pbytes = sizeof(double) * (size_t)std::max(1, T - 1) * M.nb * M.nb;
  if (malloc_async((void **)&P, pbytes, st) != hipSuccess) {
    hipGetLastError();
    set_error("dense_potrf: panel workspace allocation failed");
    return MVG_ERR_ALLOC;
  }
  hipStream_t side = lookahead() ? side_stream() : st;
  hipEvent_t evD, evS, ev0;
  hipEventCreateWithFlags(&evD, hipEventDisableTiming);
  hipEventCreateWithFlags(&evS, hipEventDisableTiming);
  hipEventCreateWithFlags(&ev0, hipEventDisableTiming);
  const PivotTol pt = pivot_tol(A);
  int rc = 0;
  hipEventRecord(ev0, st);
  hipStreamWaitEvent(side, ev0, 0);
  rc = diag_factor(M, 0, A->d_winv, d_info, pt, side);
  hipEventRecord(evD, side);
  for (int k = 0; k < T && !rc; ++k) {
    hipStreamWaitEvent(st, evD, 0);           // W_k ready
    rc = panel_trsm(step_map(k), k, A->d_winv, P, st);  // L_ik, i > k
    hipEventRecord(evS, st);
    if (rc) break;
    if (k + 1 < T) {
      hipStreamWaitEvent(side, evS, 0);
      rc = launch_syrk_next(A, k, side);  // SYRK of tile (k+1, k+1) by step k
      if (!rc) rc = diag_factor(M, k + 1, A->d_winv, d_info, pt, side);
      hipEventRecord(evD, side);
      if (!rc) rc = trailing(step_map(k), A->N, k, true, false, st);  // the rest of step k
    }
  }
  hipEventRecord(evD, side);
  hipStreamWaitEvent(st, evD, 0);
  hipFreeAsync(P, st);
  hipEventDestroy(evD);
  hipEventDestroy(evS);
  hipEventDestroy(ev0);
  return rc;
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
  if (A->tlr) return tlr_logdet_quad(A, d_y, d_part, d_out2, st);
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
  if (malloc_async((void **)&ep, sizeof(double) * A->Np, st) != hipSuccess) {
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
