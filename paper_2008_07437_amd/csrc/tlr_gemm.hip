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

// BM x BN output blocks, four waves in a 2 x 2 grid, each wave BM/2 x BN/2
// (BM/32 x BN/32 MFMA tiles), K slices of KS:
//   64 x 64, KS 16: the general case;
//   32 x 32, KS 32: products whose M and N are at most 32 (V^T V of low-rank
//     tiles);
//   128 x 64, KS 16: tall products with a long K (the sketches C Omega and
//     C^T Q of 1200-row tiles, V <- W V): twice the MFMAs per LDS fragment.
// Loader: an operand stored with its row (m or n) index contiguous is read
// as (idx, k) = (tid % D, tid / D + (256 / D) i), one stored with k
// contiguous as (tid / KS + (256 / KS) i, tid % KS).
template <int BM, int BN, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BM == 128 ? 2 : 4))) void k_gemm_batched(const GemmTask *__restrict__ tasks,
                                                      const int64_t *__restrict__ start, int ntask,
                                                      const int *__restrict__ map) {
  constexpr int TM = BM / 32, TN = BN / 32;  // MFMA tiles per wave
  constexpr int LA = BM * KS / 256, LB = BN * KS / 256;  // loads per thread and slice
  static_assert(LA >= 1 && LB >= 1 && 256 % BM == 0 && 256 % BN == 0 && 256 % KS == 0, "shape");
  __shared__ double As[KS][BM + 2];
  __shared__ double Bs[KS][BN + 2];
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
  const int mt = (M + BM - 1) / BM;
  const int64_t local = bid - start[t];
  const int m0 = (int)(local % mt) * BM, n0 = (int)(local / mt) * BN;
  const int wr = wave & 1, wc = wave >> 1, l16 = lane & 15, lk = lane >> 4;
  auto a_m = [&](int i) { return tk.ta ? tid / KS + (256 / KS) * i : tid % BM; };
  auto a_k = [&](int i) { return tk.ta ? tid % KS : tid / BM + (256 / BM) * i; };
  auto b_n = [&](int i) { return tk.tb ? tid % BN : tid / KS + (256 / KS) * i; };
  auto b_k = [&](int i) { return tk.tb ? tid / BN + (256 / BN) * i : tid % KS; };
  double ra[LA], rb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int gm = min(m0 + a_m(i), M - 1), gk = min(k0 + a_k(i), K - 1);
      ra[i] = tk.ta ? tk.A[(int64_t)gm * tk.lda + gk] : tk.A[(int64_t)gk * tk.lda + gm];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int gn = min(n0 + b_n(i), N - 1), gk = min(k0 + b_k(i), K - 1);
      rb[i] = tk.tb ? tk.B[(int64_t)gk * tk.ldb + gn] : tk.B[(int64_t)gn * tk.ldb + gk];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int gm = m0 + a_m(i), gk = k0 + a_k(i);
      // stored element (row, col) = (gm, gk), or (gk, gm) when transposed
      const bool zero_tri = tk.tri && (tk.ta ? gm > gk : gk > gm);
      if (!(gm < M && gk < K) || zero_tri) ra[i] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i)
      if (!(n0 + b_n(i) < N && k0 + b_k(i) < K)) rb[i] = 0.0;
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < LA; ++i) As[a_k(i)][a_m(i)] = ra[i];
#pragma unroll
    for (int i = 0; i < LB; ++i) Bs[b_k(i)][b_n(i)] = rb[i];
  };
  dbl4t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = dbl4t{0.0, 0.0, 0.0, 0.0};
  if (K > 0) load(0);
  for (int k0 = 0; k0 < K; k0 += KS) {
    store();
    __syncthreads();
    if (k0 + KS < K) load(k0 + KS);  // in flight during this slice's MFMAs
#pragma unroll
    for (int ks = 0; ks < KS; ks += 4) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[ks + lk][wr * (BM / 2) + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[ks + lk][wc * (BN / 2) + j * 16 + l16];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[i][j] of a 16 x 16 tile: lane j + 16 (i % 4), element i / 4
  const double alpha = tk.alpha, beta = tk.beta;
  double cv[TM][TN][4];
  if (beta != 0.0) {  // uniform
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gm = min(m0 + wr * (BM / 2) + i * 16 + 4 * e + lk, M - 1);
          const int gn = min(n0 + wc * (BN / 2) + j * 16 + l16, N - 1);
          cv[i][j][e] = tk.C[(int64_t)gn * tk.ldc + gm];
        }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) cv[i][j][e] = alpha * acc[i][j][e] + beta * cv[i][j][e];
  } else {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) cv[i][j][e] = alpha * acc[i][j][e];
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wr * (BM / 2) + i * 16 + 4 * e + lk;
        const int gn = n0 + wc * (BN / 2) + j * 16 + l16;
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
    hipLaunchKernelGGL((k_gemm_batched<32, 32, 32>), dim3((unsigned)nblocks), dim3(256), 0, st,
                       d_tasks, d_start, ntask, d_map);
  else if (bs == 128)
    hipLaunchKernelGGL((k_gemm_batched<128, 64, 16>), dim3((unsigned)nblocks), dim3(256), 0, st,
                       d_tasks, d_start, ntask, d_map);
  else
    hipLaunchKernelGGL((k_gemm_batched<64, 64, 16>), dim3((unsigned)nblocks), dim3(256), 0, st,
                       d_tasks, d_start, ntask, d_map);
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
  const int bm = bs, bn = bs == 128 ? 64 : bs;  // 128: 128 x 64 blocks
  return (int64_t)((t.M + bm - 1) / bm) * ((t.N + bn - 1) / bn);
}

}  // namespace mvg
