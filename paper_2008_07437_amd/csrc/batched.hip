// Many small likelihoods in one persistent launch (Eq. 1 per task).
//
// Each task is one (dataset, theta) pair with 2n <= SMALL_MAX rows.  A fixed
// grid of workgroups pulls task indices from a device counter until the list
// is exhausted; a workgroup evaluates its task alone: the per-theta
// quadrature table in LDS, the lower triangle of Sigma in its private
// workspace, a right-looking Cholesky in column blocks of SB (diagonal block
// in LDS with its inverse, panel by the inverse, trailing update on FP64
// MFMA), the forward solve folded into the factorisation, and the
// log-determinant and quadratic form summed in a fixed order.  A task's
// arithmetic does not depend on which workgroup runs it or on the other
// tasks, so results are the same alone and in any batch.
#include <cmath>

#include "matern_dev.h"

namespace mvg {

constexpr int SB = 32;             // column block
constexpr int SW = 8;              // waves per workgroup
constexpr int TU = 2;              // trailing tiles per wave in flight together
constexpr int STHREADS = 64 * SW;

typedef double dbl4s __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(STHREADS) void k_small_loglik(const SmallTask *__restrict__ tasks,
                                                           int ntask, int *__restrict__ counter,
                                                           double *__restrict__ ws_all,
                                                           int64_t ws_stride,
                                                           double *__restrict__ out) {
  __shared__ double sq[4 * QN];
  __shared__ double sD[SB][SB + 1];   // diagonal block -> L_kk
  __shared__ double sW[SB][SB + 1];   // W = L_kk^-1
  __shared__ double sy[SB];
  __shared__ int s_task, s_fail;
  __shared__ double s_logdet, s_quad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *ws = ws_all + (int64_t)blockIdx.x * ws_stride;
  for (;;) {
    if (tid == 0) s_task = atomicAdd(counter, 1);
    __syncthreads();
    const int ti = s_task;
    __syncthreads();
    if (ti >= ntask) break;
    const SmallTask tk = tasks[ti];
    const int n = (int)tk.n, N = 2 * n;
    double *A = ws;          // N x N, column-major, ld N (lower triangle used)
    double *zv = ws + (int64_t)N * N;  // right-hand side being solved
    // quadrature table
    for (int k = tid; k < QN; k += STHREADS) quad_entry(k, tk.P, sq);
    for (int i = tid; i < N; i += STHREADS) zv[i] = tk.z[i];
    if (tid == 0) {
      s_fail = 0;
      s_logdet = 0.0;
      s_quad = 0.0;
    }
    __syncthreads();
    // Sigma: 2 x 2 blocks of the n (n + 1) / 2 location pairs l >= r, pair
    // p = r (2n - r + 1) / 2 + (l - r), spread evenly over the threads
    const int npair = n * (n + 1) / 2;
    for (int pq = tid; pq < npair; pq += STHREADS) {
      // r = the column whose pairs contain pq (exact integer fix-up after the root)
      const double nn = 2.0 * n + 1.0;
      int r = (int)((nn - sqrt(nn * nn - 8.0 * (double)pq)) * 0.5);
      r = max(0, min(r, n - 1));
      while (r > 0 && r * (2 * n - r + 1) / 2 > pq) --r;
      while (r + 1 < n && (r + 1) * (2 * n - r) / 2 <= pq) ++r;
      const int l = r + (pq - r * (2 * n - r + 1) / 2);
      double c[3];
      cross_cov_block(tk.x[l], tk.y[l], tk.x[r], tk.y[r], tk.P, sq, c);
      double *a = A + (int64_t)(2 * r) * N + 2 * l;
      a[0] = c[0];
      a[1] = c[2];
      a[N] = c[2];
      a[N + 1] = c[1];
    }
    __syncthreads();
    for (int k0 = 0; k0 < N; k0 += SB) {
      const int kb = min(SB, N - k0);
      // (a) diagonal block: Cholesky in LDS (all threads, one column at a time)
      for (int e = tid; e < kb * kb; e += STHREADS) {
        const int r = e % kb, c = e / kb;
        sD[r][c] = (r >= c) ? A[(int64_t)(k0 + c) * N + k0 + r] : 0.0;
      }
      __syncthreads();
      for (int c = 0; c < kb; ++c) {
        const double d = sD[c][c];
        const int g = k0 + c;
        const double tol = (g & 1) ? tk.t1 : tk.t0;
        if (!(d > tol) || !(d > 0.0)) {
          if (tid == 0) s_fail = g + 1;
          break;  // uniform: every thread reads the same d
        }
        const double ljj = sqrt(d);
        __syncthreads();
        if (tid == 0) {
          sD[c][c] = ljj;
          s_logdet += log(ljj);
        }
        for (int r = c + 1 + tid; r < kb; r += STHREADS) sD[r][c] /= ljj;
        __syncthreads();
        for (int e = tid; e < kb * kb; e += STHREADS) {
          const int r = e % kb, q = e / kb;
          if (q > c && r >= q) sD[r][q] -= sD[r][c] * sD[q][c];
        }
        __syncthreads();
      }
      __syncthreads();
      if (s_fail) break;
      // W = L_kk^-1 by columns (thread c), then y_k = W z_k; entries outside
      // the kb x kb block are zero
      for (int e = tid; e < SB * SB; e += STHREADS) sW[e % SB][e / SB] = 0.0;
      __syncthreads();
      if (tid < kb) {
        const int c = tid;
        for (int r = c; r < kb; ++r) {
          double s = (r == c) ? 1.0 : 0.0;
          for (int q = c; q < r; ++q) s -= sD[r][q] * sW[q][c];
          sW[r][c] = s / sD[r][r];
        }
      }
      __syncthreads();
      if (tid < SB) {
        double s = 0.0;
        for (int q = 0; q <= tid && q < kb; ++q) s += sW[tid][q] * zv[k0 + q];
        sy[tid] = tid < kb ? s : 0.0;
      }
      __syncthreads();
      if (tid == 0) {
        double q = s_quad;
        for (int c = 0; c < kb; ++c) q += sy[c] * sy[c];
        s_quad = q;
      }
      // L_kk back to A (the solve of later columns does not need it)
      for (int e = tid; e < kb * kb; e += STHREADS) {
        const int r = e % kb, c = e / kb;
        if (r >= c) A[(int64_t)(k0 + c) * N + k0 + r] = sD[r][c];
      }
      // (b) panel rows i >= k0 + kb: L_i = A_i W^T on MFMA, 16 rows per wave
      //     (a wave reads its rows' A values before it overwrites them)
      const int r0 = k0 + kb;
      const int l16 = lane & 15, lk = lane >> 4;
      for (int t = wave; t < (N - r0 + 15) / 16; t += SW) {
        const int row = r0 + t * 16 + l16;
        double av[SB / 4];
#pragma unroll
        for (int kk = 0; kk < SB / 4; ++kk) {
          const int q = 4 * kk + lk;
          av[kk] = (row < N && q < kb) ? A[(int64_t)(k0 + q) * N + row] : 0.0;
        }
#pragma unroll
        for (int half = 0; half < SB / 16; ++half) {
          dbl4s acc = dbl4s{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kk = 0; kk < SB / 4; ++kk)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], sW[half * 16 + l16][4 * kk + lk], acc,
                                                       0, 0, 0);
          const int c = half * 16 + l16;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int gi = r0 + t * 16 + 4 * e + lk;
            if (gi < N && c < kb) A[(int64_t)(k0 + c) * N + gi] = acc[e];
          }
        }
      }
      __syncthreads();
      for (int i = r0 + tid; i < N; i += STHREADS) {  // z_i -= L_i y_k
        double zi = 0.0;
        for (int c = 0; c < kb; ++c) zi += A[(int64_t)(k0 + c) * N + i] * sy[c];
        zv[i] -= zi;
      }
      // (c) trailing update A_ij -= L_i L_j^T for k0 + kb <= j <= i, 16 x 16
      //     tiles on MFMA (lane j + 16 (i % 4), element i / 4 of a tile); a
      //     wave takes TU tiles at a time so that their loads are in flight
      //     together (the workspace is in global memory: latency-bound)
      const int m = (N - r0 + 15) / 16;
      const int ntile = m * (m + 1) / 2;
      for (int t0 = wave; t0 < ntile; t0 += SW * TU) {
        int I[TU], J[TU];
#pragma unroll
        for (int u = 0; u < TU; ++u) {  // tile (I, J), J <= I, row-major over the lower triangle
          const int t = t0 + u * SW;
          int ii = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
          while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;  // exact after rounding
          while (ii * (ii + 1) / 2 > t) --ii;
          I[u] = t < ntile ? ii : m;  // past the end: a row of tiles beyond N (all masked)
          J[u] = t < ntile ? t - ii * (ii + 1) / 2 : 0;
        }
        dbl4s acc[TU];
        double av[TU][SB / 4], bv[TU][SB / 4];
#pragma unroll
        for (int u = 0; u < TU; ++u) {
          const int rowA = r0 + I[u] * 16 + l16, rowB = r0 + J[u] * 16 + l16;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int gi = r0 + I[u] * 16 + 4 * e + lk, gj = r0 + J[u] * 16 + l16;
            acc[u][e] = (gi < N && gj < N) ? A[(int64_t)gj * N + gi] : 0.0;
          }
#pragma unroll
          for (int kk = 0; kk < SB / 4; ++kk) {
            const int q = 4 * kk + lk;
            av[u][kk] = (rowA < N && q < kb) ? -A[(int64_t)(k0 + q) * N + rowA] : 0.0;
            bv[u][kk] = (rowB < N && q < kb) ? A[(int64_t)(k0 + q) * N + rowB] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < TU; ++u)
#pragma unroll
          for (int kk = 0; kk < SB / 4; ++kk)
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][kk], bv[u][kk], acc[u], 0, 0, 0);
#pragma unroll
        for (int u = 0; u < TU; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int gi = r0 + I[u] * 16 + 4 * e + lk, gj = r0 + J[u] * 16 + l16;
            if (gi < N && gj < N) A[(int64_t)gj * N + gi] = acc[u][e];
          }
      }
      __syncthreads();
    }
    if (tid == 0) {
      double *o = out + 4 * (int64_t)ti;
      if (s_fail) {
        o[0] = -INFINITY;
        o[1] = NAN;
        o[2] = NAN;
        o[3] = (double)s_fail;
      } else {
        const double logdet = 2.0 * s_logdet, quad = s_quad;
        o[0] = -(double)n * log(2.0 * M_PI) - 0.5 * logdet - 0.5 * quad;
        o[1] = logdet;
        o[2] = quad;
        o[3] = 0.0;
      }
    }
    __syncthreads();
  }
}

__global__ void k_zero_int(int *p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

int small_batch_workgroups(int ntask) { return ntask < 2 * 256 ? ntask : 2 * 256; }

size_t small_workspace_doubles(int64_t nmax) {
  const int64_t N = 2 * nmax;
  return (size_t)(N * N + N);
}

int launch_small_loglik(const SmallTask *d_tasks, int ntask, int64_t nmax, int *d_counter,
                        double *d_ws, double *d_out, hipStream_t st) {
  if (ntask <= 0) return 0;
  if (2 * nmax > SMALL_MAX) {
    set_error("batched small likelihood: 2n = %lld above %d", (long long)(2 * nmax), SMALL_MAX);
    return MVG_ERR_LIMIT;
  }
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, d_counter);
  if (int rc = check_launch("zero_int")) return rc;
  const int G = small_batch_workgroups(ntask);
  hipLaunchKernelGGL(k_small_loglik, dim3(G), dim3(STHREADS), 0, st, d_tasks, ntask, d_counter, d_ws,
                     (int64_t)small_workspace_doubles(nmax), d_out);
  return check_launch("small_loglik");
}

}  // namespace mvg
