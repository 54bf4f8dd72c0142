// Batched FP64 GEMMs of the tile-low-rank (TLR) path on gfx950 MFMA: C =
// alpha op(A) op(B) + beta C over a list of variable-size products (tile
// expansion, the small V^T V products, triangular applications, sketches).
// The TLR driver builds the lists on the host; the one large column update of
// each factorisation step is in tlr_update.hip.
#include <cmath>
#include <cstdint>
#include <cstdlib>

#include "tlr.h"

namespace mvg {

typedef double dbl4t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ batched GEMM
//
// C = alpha op(A) op(B) + beta C, column-major, op(X) = X or X^T.  One
// workgroup per 64 x 64 (or 32 x 32) block of C, four waves on
// v_mfma_f64_16x16x4f64; K slices staged through LDS with the next
// slice's global loads in flight during the current slice's MFMAs (one LDS
// buffer: 19 KB, so that many workgroups share a CU; most products here
// have a short K).  A block finds its task by binary search over the tasks'
// first-block offsets staged in LDS when the list is short, else from a
// block -> task map written by k_gemm_task_map.  All
// operand loads are from clamped, always-valid addresses and masked after a
// scheduling barrier (ragged edges, the zero triangle of a triangular A); C
// is read for beta != 0 with all of a lane's loads issued together.

__global__ void k_gemm_task_map(const int64_t *__restrict__ start, int ntask, int64_t nblocks,
                                int *__restrict__ map) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntask) return;
  const int64_t e = t + 1 < ntask ? start[t + 1] : nblocks;
  for (int64_t b = start[t]; b < e; ++b) map[b] = t;
}

// BS x BS output blocks (64: four waves of 32 x 32, 2 x 2 MFMA tiles each,
// K slices of 16; 32: four waves of 16 x 16, one tile each, K slices of 32,
// for products whose M and N are at most 32, e.g. V^T V of low-rank tiles).
// A slice holds 1024 values of each operand: four loads per thread.
template <int BS>
__global__ __launch_bounds__(256) void k_gemm_batched(const GemmTask *__restrict__ tasks,
                                                      const int64_t *__restrict__ start, int ntask,
                                                      const int *__restrict__ map) {
  constexpr int KS = 1024 / BS;   // K slice
  constexpr int TW = BS / 32;     // MFMA tiles per wave and dimension
  constexpr int SU = 256 / BS;    // k rows per load step, untransposed loader
  constexpr int ST = 256 / KS;    // m (n) rows per load step, transposed loader
  __shared__ double As[KS][BS + 2];
  __shared__ double Bs[KS][BS + 2];
  __shared__ int64_t sstart[GEMM_TASKS_LDS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t bid = blockIdx.x;
  int t;
  if (map) {
    t = map[bid];
  } else if (ntask <= GEMM_TASKS_LDS) {
    for (int i = tid; i < ntask; i += 256) sstart[i] = start[i];
    __syncthreads();
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sstart[mid] <= bid) lo = mid; else hi = mid - 1;
    }
    t = lo;
  } else {
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (start[mid] <= bid) lo = mid; else hi = mid - 1;
    }
    t = lo;
  }
  const GemmTask tk = tasks[t];
  const int M = tk.M, N = tk.N, K = tk.K;
  const int mt = (M + BS - 1) / BS;
  const int64_t local = bid - start[t];
  const int m0 = (int)(local % mt) * BS, n0 = (int)(local / mt) * BS;
  const int wr = wave & 1, wc = wave >> 1, l16 = lane & 15, lk = lane >> 4;
  // loader coordinates: thread tid takes (m, k) = (tid % BS, tid / BS + SU i)
  // of an operand stored with m contiguous, (tid / KS + ST i, tid % KS) of
  // one stored with k contiguous
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = tk.ta ? (tid / KS) + ST * i : (tid % BS);
      const int k = tk.ta ? (tid % KS) : (tid / BS) + SU * i;
      const int gm = min(m0 + m, M - 1), gk = min(k0 + k, K - 1);
      ra[i] = tk.ta ? tk.A[(int64_t)gm * tk.lda + gk] : tk.A[(int64_t)gk * tk.lda + gm];
      const int n = tk.tb ? (tid % BS) : (tid / KS) + ST * i;
      const int kb = tk.tb ? (tid / BS) + SU * i : (tid % KS);
      const int gn = min(n0 + n, N - 1), gkb = min(k0 + kb, K - 1);
      rb[i] = tk.tb ? tk.B[(int64_t)gkb * tk.ldb + gn] : tk.B[(int64_t)gn * tk.ldb + gkb];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = tk.ta ? (tid / KS) + ST * i : (tid % BS);
      const int k = tk.ta ? (tid % KS) : (tid / BS) + SU * i;
      const int gm = m0 + m, gk = k0 + k;
      // stored element (row, col) = (gm, gk), or (gk, gm) when transposed
      const bool zero_tri = tk.tri && (tk.ta ? gm > gk : gk > gm);
      if (!(gm < M && gk < K) || zero_tri) ra[i] = 0.0;
      const int n = tk.tb ? (tid % BS) : (tid / KS) + ST * i;
      const int kb = tk.tb ? (tid / BS) + SU * i : (tid % KS);
      if (!(n0 + n < N && k0 + kb < K)) rb[i] = 0.0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!tk.ta) As[(tid / BS) + SU * i][tid % BS] = ra[i];
      else As[tid % KS][(tid / KS) + ST * i] = ra[i];
      if (tk.tb) Bs[(tid / BS) + SU * i][tid % BS] = rb[i];
      else Bs[tid % KS][(tid / KS) + ST * i] = rb[i];
    }
  };
  dbl4t acc[TW][TW];
#pragma unroll
  for (int i = 0; i < TW; ++i)
#pragma unroll
    for (int j = 0; j < TW; ++j) acc[i][j] = dbl4t{0.0, 0.0, 0.0, 0.0};
  if (K > 0) load(0);
  for (int k0 = 0; k0 < K; k0 += KS) {
    store();
    __syncthreads();
    if (k0 + KS < K) load(k0 + KS);  // in flight during this slice's MFMAs
#pragma unroll
    for (int ks = 0; ks < KS; ks += 4) {
      double a[TW], b[TW];
#pragma unroll
      for (int i = 0; i < TW; ++i) {
        a[i] = As[ks + lk][wr * (BS / 2) + i * 16 + l16];
        b[i] = Bs[ks + lk][wc * (BS / 2) + i * 16 + l16];
      }
#pragma unroll
      for (int i = 0; i < TW; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[i][j] of a 16 x 16 tile: lane j + 16 (i % 4), element i / 4
  const double alpha = tk.alpha, beta = tk.beta;
  double cv[TW][TW][4];
  if (beta != 0.0) {  // uniform
#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
      for (int j = 0; j < TW; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gm = min(m0 + wr * (BS / 2) + i * 16 + 4 * e + lk, M - 1);
          const int gn = min(n0 + wc * (BS / 2) + j * 16 + l16, N - 1);
          cv[i][j][e] = tk.C[(int64_t)gn * tk.ldc + gm];
        }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
      for (int j = 0; j < TW; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) cv[i][j][e] = alpha * acc[i][j][e] + beta * cv[i][j][e];
  } else {
#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
      for (int j = 0; j < TW; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) cv[i][j][e] = alpha * acc[i][j][e];
  }
#pragma unroll
  for (int i = 0; i < TW; ++i)
#pragma unroll
    for (int j = 0; j < TW; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wr * (BS / 2) + i * 16 + 4 * e + lk;
        const int gn = n0 + wc * (BS / 2) + j * 16 + l16;
        if (gm < M && gn < N) tk.C[(int64_t)gn * tk.ldc + gm] = cv[i][j][e];
      }
}

int launch_gemm_batched(const GemmTask *d_tasks, const int64_t *d_start, int ntask, int64_t nblocks,
                        hipStream_t st, const int *d_map, int bs) {
  if (ntask <= 0 || nblocks <= 0) return 0;
  if (nblocks >= ((int64_t)1 << 31)) {
    set_error("batched GEMM: %lld blocks", (long long)nblocks);
    return MVG_ERR_LIMIT;
  }
  if (bs == 32)
    hipLaunchKernelGGL(k_gemm_batched<32>, dim3((unsigned)nblocks), dim3(256), 0, st, d_tasks,
                       d_start, ntask, d_map);
  else
    hipLaunchKernelGGL(k_gemm_batched<64>, dim3((unsigned)nblocks), dim3(256), 0, st, d_tasks,
                       d_start, ntask, d_map);
  return check_launch("gemm_batched");
}

int launch_gemm_task_map(const int64_t *d_start, int ntask, int64_t nblocks, int *d_map,
                         hipStream_t st) {
  if (ntask <= 0 || nblocks <= 0) return 0;
  hipLaunchKernelGGL(k_gemm_task_map, dim3((ntask + 255) / 256), dim3(256), 0, st, d_start, ntask,
                     nblocks, d_map);
  return check_launch("gemm_task_map");
}

int64_t gemm_blocks(const GemmTask &t, int bs) {
  if (t.M <= 0 || t.N <= 0) return 0;
  return (int64_t)((t.M + bs - 1) / bs) * ((t.N + bs - 1) / bs);
}

}  // namespace mvg
