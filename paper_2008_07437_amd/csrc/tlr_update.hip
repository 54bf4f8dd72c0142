// The column update of the tile-low-rank (TLR) Cholesky on gfx950 MFMA:
// C -= A B^T for one large product per tile column (all earlier columns'
// low-rank contributions at once).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>

#include "tlr.h"

namespace mvg {

typedef double dbl4t __attribute__((ext_vector_type(4)));

// ------------------------------------------- C -= A B^T for one large product
//
// The column update of the TLR factorisation: C (M x N) -= A (M x K) B^T
// (B: N x K), column-major, M up to 2e5, N = the tile size, K = the summed
// ranks.  128 x 128 blocks (four waves of 64 x 64, 4 x 4 tiles of
// v_mfma_f64_16x16x4f64), K slices of 16 staged through LDS with the next
// slice's global loads in flight during the current slice's MFMAs (double
// buffer), accumulators started from C so that the epilogue is stores only.
// All loads are issued from clamped, always-valid addresses and zeroed
// outside the matrix after a scheduling barrier (a load under a branch waits
// for its value); blocks that lie inside C store without masks.
constexpr int BG = 128, BK = 16;

__global__ __launch_bounds__(256) void k_gemm_nt_sub(const double *__restrict__ A, int lda,
                                                     const double *__restrict__ B, int ldb,
                                                     double *__restrict__ C, int ldc, int M, int N,
                                                     int K, int mblocks) {
  __shared__ double As[2][BK][BG + 4];
  __shared__ double Bs[2][BK][BG + 4];
  // Workgroups are dealt to the 8 XCDs in turn (w % 8).  On each XCD the
  // consecutive workgroups take all column blocks of one row block before
  // the next row block, so the blocks that read the same rows of A run
  // together and share that XCD's L2 (A is read about once from HBM instead
  // of once per column block); row blocks beyond a multiple of 8 follow in
  // plain order.
  int blk_r, blk_c;
  {
    const int w = blockIdx.x, nbk = (N + BG - 1) / BG;
    const int full = (mblocks / 8) * 8 * nbk;
    if (w < full) {
      const int t = w >> 3;
      blk_c = t % nbk;
      blk_r = (t / nbk) * 8 + (w & 7);
    } else {
      const int t = w - full;
      blk_c = t % nbk;
      blk_r = (mblocks / 8) * 8 + t / nbk;
    }
  }
  const int m0 = blk_r * BG, n0 = blk_c * BG;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1, l16 = lane & 15, lk = lane >> 4;
  // loader: thread t takes rows 2 (t % 64) + {0, 1} of slice columns t / 64 + 4 i
  const int lr = 2 * (tid & 63), lc = tid >> 6;
  double ra[8], rb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = min(k0 + lc + 4 * i, K - 1);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        ra[2 * i + h] = A[(int64_t)k * lda + min(m0 + lr + h, M - 1)];
        rb[2 * i + h] = B[(int64_t)k * ldb + min(n0 + lr + h, N - 1)];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool kok = k0 + lc + 4 * i < K;
        if (!(kok && m0 + lr + h < M)) ra[2 * i + h] = 0.0;
        if (!(kok && n0 + lr + h < N)) rb[2 * i + h] = 0.0;
      }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        As[buf][lc + 4 * i][lr + h] = -ra[2 * i + h];  // C -= A B^T
        Bs[buf][lc + 4 * i][lr + h] = rb[2 * i + h];
      }
  };
  const bool inside = m0 + BG <= M && n0 + BG <= N;
  // accumulators from C: tile (ti, tj) element (4 e + lk, l16)
  dbl4t acc[4][4];
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wr * 64 + ti * 16 + 4 * e + lk;
        const int gn = n0 + wc * 64 + tj * 16 + l16;
        acc[ti][tj][e] = C[(int64_t)min(gn, N - 1) * ldc + min(gm, M - 1)];
      }
  int buf = 0;
  if (K > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += BK) {
    if (k0 + BK < K) load(k0 + BK);  // in flight during this slice's MFMAs
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[buf][ks + lk][wr * 64 + i * 16 + l16];
        b[i] = Bs[buf][ks + lk][wc * 64 + i * 16 + l16];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (k0 + BK < K) store(buf ^ 1);  // the other buffer: last read a slice ago
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wr * 64 + ti * 16 + 4 * e + lk;
        const int gn = n0 + wc * 64 + tj * 16 + l16;
        if (inside || (gm < M && gn < N)) C[(int64_t)gn * ldc + gm] = acc[ti][tj][e];
      }
}

// The same product with the K slices moved straight from global memory into
// LDS (global_load_lds_dwordx4: no register staging, no LDS store
// instructions), two stages, one barrier per slice, the refill of the other
// stage issued at raised wave priority right after the barrier, and the first
// k-step's fragments read before it.  Requirements (checked by the launcher):
// K a multiple of 32 (the caller zero-pads A's and B's columns), M and N even,
// lda and ldb even, A and B 16-byte aligned.  A loader lane moves rows 2l,
// 2l + 1 of one column, clamped inside the matrix (rows past M or N only feed
// outputs that are not stored).
constexpr int NSL_K = 16;  // K slice
#define MVG_LDSP(p) ((__attribute__((address_space(3))) void *)(p))

template <int N>
__device__ __forceinline__ void nsl_wait_vmcnt() {
  static_assert(N >= 0 && N < 16, "small counts only");
  __builtin_amdgcn_s_waitcnt(0x0F70 | N);  // vmcnt(N); lgkmcnt, expcnt unconstrained
}

// A grid smaller than the block count (a multiple of 8) walks the blocks
// in steps of the grid, so that the product can leave CUs to concurrent
// work on another stream.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_nt_sub_lds(
    const double *__restrict__ A, int lda, const double *__restrict__ B, int ldb,
    double *__restrict__ C, int ldc, int M, int N, int K, int mblocks) {
  __shared__ double sA[2][NSL_K * BG];
  __shared__ double sB[2][NSL_K * BG];
  const int nbk = (N + BG - 1) / BG;
  for (int w = blockIdx.x; w < mblocks * nbk; w += gridDim.x) {
    int blk_r, blk_c;  // XCD order, as in k_gemm_nt_sub
    {
      const int full = (mblocks / 8) * 8 * nbk;
      if (w < full) {
        const int t = w >> 3;
        blk_c = t % nbk;
        blk_r = (t / nbk) * 8 + (w & 7);
      } else {
        const int t = w - full;
        blk_c = t % nbk;
        blk_r = (mblocks / 8) * 8 + t / nbk;
      }
    }
    const int m0 = blk_r * BG, n0 = blk_c * BG;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave & 1, wc = wave >> 1, l16 = lane & 15, lk = lane >> 4;
    const double *a0 = A + min(m0 + 2 * lane, M - 2);
    const double *b0 = B + min(n0 + 2 * lane, N - 2);
    // slice kb into stage st: wave w moves columns w, w + 4, w + 8, w + 12 of
    // the A and B slices (1 KB each)
    auto issue = [&](int kb, int st) {
#pragma unroll
      for (int c = 0; c < NSL_K / 4; ++c) {
        const int64_t k = (int64_t)kb * NSL_K + wave + 4 * c;
        __builtin_amdgcn_global_load_lds((const void *)(a0 + k * lda),
                                         MVG_LDSP(&sA[st][(wave + 4 * c) * BG]), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void *)(b0 + k * ldb),
                                         MVG_LDSP(&sB[st][(wave + 4 * c) * BG]), 16, 0, 0);
      }
    };
    const int nk = K / NSL_K;
    if (nk > 0) issue(0, 0);
    // accumulators from C: tile (ti, tj) element (4 e + lk, l16)
    dbl4t acc[4][4];
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gm = m0 + wr * 64 + ti * 16 + 4 * e + lk;
          const int gn = n0 + wc * 64 + tj * 16 + l16;
          acc[ti][tj][e] = C[(int64_t)min(gn, N - 1) * ldc + min(gm, M - 1)];
        }
    for (int kb = 0; kb < nk; ++kb) {
      const int u = kb & 1;
      // slice kb has landed (this wave's loads; the barrier covers the others'),
      // and every wave is done with the stage that is refilled next
      nsl_wait_vmcnt<0>();
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_setprio(1);
      const double *a = &sA[u][wr * 64 + l16];
      const double *bb = &sB[u][wc * 64 + l16];
      double af0[4], bf0[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        af0[t] = -a[lk * BG + t * 16];  // C -= A B^T
        bf0[t] = bb[lk * BG + t * 16];
      }
      if (kb + 1 < nk) issue(kb + 1, u ^ 1);
      __builtin_amdgcn_s_setprio(0);
#pragma unroll
      for (int ks = 0; ks < NSL_K; ks += 4) {
        double af[4], bf[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          af[t] = ks == 0 ? af0[t] : -a[(ks + lk) * BG + t * 16];
          bf[t] = ks == 0 ? bf0[t] : bb[(ks + lk) * BG + t * 16];
        }
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
          for (int tj = 0; tj < 4; ++tj)
            acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ti], bf[tj], acc[ti][tj], 0, 0, 0);
      }
    }
    nsl_wait_vmcnt<0>();  // no direct LDS load outlives the workgroup
    const bool inside = m0 + BG <= M && n0 + BG <= N;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gm = m0 + wr * 64 + ti * 16 + 4 * e + lk;
          const int gn = n0 + wc * 64 + tj * 16 + l16;
          if (inside || (gm < M && gn < N)) C[(int64_t)gn * ldc + gm] = acc[ti][tj][e];
        }
    __syncthreads();  // every wave is done with both stages before the next block's loads
  }
}

int launch_gemm_nt_sub(const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                       int M, int N, int K, hipStream_t st, int max_wg) {
  if (M <= 0 || N <= 0) return 0;
  const int64_t mb = (M + BG - 1) / BG, nbk = (N + BG - 1) / BG;
  if (mb * nbk >= ((int64_t)1 << 31)) {
    set_error("GEMM: %lld blocks", (long long)(mb * nbk));
    return MVG_ERR_LIMIT;
  }
  static const bool lds_path = [] {  // MVG_GEMM_NT_LDS=0: the register-staged kernel (experiments)
    const char *e = getenv("MVG_GEMM_NT_LDS");
    return !(e && atoi(e) == 0);
  }();
  if (lds_path && K % (2 * NSL_K) == 0 && M % 2 == 0 && N % 2 == 0 && lda % 2 == 0 &&
      ldb % 2 == 0 && ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0) {
    int64_t grid = mb * nbk;
    if (max_wg > 0 && grid > max_wg) grid = std::max<int64_t>(8, max_wg / 8 * 8);
    hipLaunchKernelGGL(k_gemm_nt_sub_lds, dim3((unsigned)grid), dim3(256), 0, st, A, lda, B, ldb, C,
                       ldc, M, N, K, (int)mb);
    return check_launch("gemm_nt_sub_lds");
  }
  hipLaunchKernelGGL(k_gemm_nt_sub, dim3((unsigned)(mb * nbk)), dim3(256), 0, st, A, lda, B, ldb,
                     C, ldc, M, N, K, (int)mb);
  return check_launch("gemm_nt_sub");
}

}  // namespace mvg
