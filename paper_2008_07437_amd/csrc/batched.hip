// Many small likelihoods in one persistent launch (Eq. 1 per task).
//
// Each task is one (dataset, theta) pair with 2n <= SMALL_MAX rows.  A fixed
// grid of workgroups pulls task indices from a device counter until the list
// is exhausted; a workgroup evaluates its task alone: the per-theta
// quadrature table in LDS, the lower triangle of Sigma in its private
// workspace, a left-looking Cholesky in column blocks of SB (each block
// column first receives all earlier columns' updates on FP64 MFMA, then its
// diagonal block is factored by one wave in registers with its inverse and
// the rows below are solved by that inverse on MFMA), the forward solve
// folded into the factorisation,
// and the log-determinant and quadratic form summed in a fixed order.  A task's
// arithmetic does not depend on which workgroup runs it or on the other
// tasks, so results are the same alone and in any batch.
#include <cmath>

#include "matern_dev.h"

namespace mvg {

constexpr int SB = 32;             // column block
constexpr int SW = 4;              // waves per workgroup (two workgroups per CU)
constexpr int STHREADS = 64 * SW;

typedef double dbl4s __attribute__((ext_vector_type(4)));

// A[col * N + row] from a clamped address inside the task's N x N workspace.
// Masked entries are loaded unconditionally and zeroed afterwards, behind a
// scheduling barrier: a load under a branch, or a select scheduled next to
// its load, waits for the value at once, and a wave's loads then go out one
// at a time instead of all in flight together.
// The offset is formed in 32 bits (the workspace of one task is below 4 GiB)
// so that the load takes the uniform base in scalar registers.
__device__ __forceinline__ double clamped_load(const double *A, int N, int col, int row) {
  const unsigned off = ((unsigned)min(col, N - 1) * (unsigned)N + (unsigned)min(row, N - 1)) * 8u;
  return *(const double *)((const char *)A + off);
}

__device__ __forceinline__ double load_at(const double *A, int N, int col, int row) {
  return *(const double *)((const char *)A + ((unsigned)col * (unsigned)N + (unsigned)row) * 8u);
}

__device__ __forceinline__ void store_at(double *A, int N, int col, int row, double v) {
  *(double *)((char *)A + ((unsigned)col * (unsigned)N + (unsigned)row) * 8u) = v;
}

// x of lane l (l uniform) as a uniform value
__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum of x over the 16 lanes of a DPP row (lanes 16 g .. 16 g + 15), in lane
// 16 g: pairs, quads, halves of the row (lane i with 7 - i), then the row
// mirrored (lane i with 15 - i).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double row16_sum(double x) {
  x += dpp_d<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_d<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_d<0x141>(x);  // row_half_mirror
  x += dpp_d<0x140>(x);  // row_mirror
  return x;
}

// Left-looking update of the columns k0 .. k0 + kb - 1 (kb <= 16 NT), rows
// k0 .. N - 1, by the columns q in [qlo, k0): A[r][c] -= sum_q L[r][q] L[c][q],
// on FP64 MFMA.  The rows are cut into 32-row output blocks, one per wave
// (2 x NT tiles of 16 x 16: lane j + 16 (i % 4), element i / 4 of a tile);
// when there are fewer blocks than waves, the q range of a block is split over
// several waves and their partial tiles are summed in a fixed order through
// the workgroup's scratch.  The block columns are updated two at a time
// (NT = 4: 64 columns by every earlier column, then the second block of the
// pair by the first one alone, NT = 2), so the panels L[., < k0] are read once
// per 64 columns: about a sixth of the bytes of a right-looking update, which
// reads and writes the trailing matrix at every step.  Every load is from a
// clamped address inside the task's N x N workspace, masked after the load;
// the next 16 columns' operands are in flight while the current ones feed
// the MFMAs.  Outputs above the diagonal (the first row block of the second
// block of a pair) are computed and stored like the others and never read.
template <int NT>
__device__ __forceinline__ void left_update(double *A, int N, int k0, int kb, int qlo,
                                            double *part, int wave, int lane, int tid) {
  constexpr int BW = 16 * NT;  // output columns of a block
  const int l16 = lane & 15, lk = lane >> 4;
  const int nout = (N - k0 + 31) / 32;
  const int splits = nout >= SW ? 1 : SW / nout;
  const int nitems = nout * splits;
  const int K = k0 - qlo;
  const int kc = (K / splits + 7) / 8 * 8;  // q per part (a multiple of 8)
  for (int it = wave; it < nitems; it += SW) {
    const int b = it / splits, pt = it % splits;
    const int iA = k0 + 32 * b;
    const int q0 = qlo + min(K, pt * kc), q1 = qlo + min(K, pt * kc + kc);
    dbl4s acc[2][NT];
#pragma unroll
    for (int hi = 0; hi < 2; ++hi)
#pragma unroll
      for (int hj = 0; hj < NT; ++hj)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          acc[hi][hj][e] = pt == 0 ? clamped_load(A, N, k0 + 16 * hj + l16, iA + 16 * hi + 4 * e + lk)
                                   : 0.0;
    double ca[2][2], cb[NT][2];  // [h][kk]: rows 16 h + l16, columns q + 4 kk + lk
    auto fetch = [&](int q, double (&fa)[2][2], double (&fb)[NT][2]) {
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
        for (int h = 0; h < 2; ++h) fa[h][kk] = clamped_load(A, N, q + 4 * kk + lk, iA + 16 * h + l16);
#pragma unroll
        for (int h = 0; h < NT; ++h) fb[h][kk] = clamped_load(A, N, q + 4 * kk + lk, k0 + 16 * h + l16);
      }
    };
    // two chunks of 8 columns in flight ahead of the one feeding the MFMAs
    // (addresses clamped to the last column; chunks past q1 are not used)
    double ma[2][2], mb[NT][2];
    if (q0 < q1) {
      fetch(q0, ca, cb);
      fetch(min(q0 + 8, q1 - 1), ma, mb);
    }
    for (int q = q0; q < q1; q += 8) {
      double na[2][2], nb2[NT][2];
      fetch(min(q + 16, q1 - 1), na, nb2);
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        const bool okq = q + 4 * kk + lk < q1;
#pragma unroll
        for (int h = 0; h < 2; ++h) ca[h][kk] = (okq && iA + 16 * h + l16 < N) ? -ca[h][kk] : 0.0;
#pragma unroll
        for (int h = 0; h < NT; ++h)
          if (!(okq && 16 * h + l16 < kb)) cb[h][kk] = 0.0;
      }
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int hi = 0; hi < 2; ++hi)
#pragma unroll
          for (int hj = 0; hj < NT; ++hj)
            acc[hi][hj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[hi][kk], cb[hj][kk], acc[hi][hj], 0, 0, 0);
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          ca[h][kk] = ma[h][kk];
          ma[h][kk] = na[h][kk];
        }
#pragma unroll
        for (int h = 0; h < NT; ++h) {
          cb[h][kk] = mb[h][kk];
          mb[h][kk] = nb2[h][kk];
        }
      }
    }
#pragma unroll
    for (int hi = 0; hi < 2; ++hi)
#pragma unroll
      for (int hj = 0; hj < NT; ++hj)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = 16 * hi + 4 * e + lk, c = 16 * hj + l16;
          if (splits == 1) {
            if (iA + r < N && c < kb) store_at(A, N, k0 + c, iA + r, acc[hi][hj][e]);
          } else {
            part[(int64_t)wave * (32 * BW) + c * 32 + r] = acc[hi][hj][e];
          }
        }
  }
  if (splits > 1) {  // item it ran on wave it (nitems <= SW)
    __syncthreads();
    for (int e = tid; e < nout * 32 * BW; e += STHREADS) {
      const int b = e / (32 * BW), idx = e % (32 * BW), r = idx % 32, c = idx / 32;
      double t = 0.0;
      for (int p = 0; p < splits; ++p) t += part[(int64_t)(b * splits + p) * (32 * BW) + idx];
      if (k0 + 32 * b + r < N && c < kb) store_at(A, N, k0 + c, k0 + 32 * b + r, t);
    }
  }
}

// Two workgroups per CU (at most 256 registers per lane): one task's
// generation (FP64 VALU) runs beside another's factorisation (MFMA, memory).
__global__ __launch_bounds__(STHREADS) __attribute__((amdgpu_waves_per_eu(2))) void k_small_loglik(
    const SmallTask *__restrict__ tasks, int ntask, int *__restrict__ counter,
    double *__restrict__ ws_all, int64_t ws_stride, double *__restrict__ out) {
  __shared__ double sq[4 * QN];
  __shared__ double sW[SB][SB + 1];   // W = L_kk^-1
  __shared__ double sy[SB];
  __shared__ double slg[SB];          // log L_jj of the block
  __shared__ double szk[SB];          // z of the block's rows
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
    double *part = zv + N;   // SW partial 32 x 64 tiles of the split updates
    // quadrature table
    for (int k = tid; k < QN; k += STHREADS) quad_entry(k, tk.P, sq);
    for (int i = tid; i < N; i += STHREADS) zv[i] = tk.z[i];
    if (tid == 0) {
      s_fail = 0;
      s_logdet = 0.0;
      s_quad = 0.0;
    }
    __syncthreads();
    // Sigma: 2 x 2 blocks of the n (n + 1) / 2 location pairs l >= r, spread
    // evenly over the threads.  Column r of the pairs (l = r .. n - 1) and
    // column n - 1 - r together hold n + 1 pairs, so pair p is entry p % (n + 1)
    // of folded row p / (n + 1) (for odd n the middle column is the last,
    // half-filled row); a thread steps its (row, entry) by STHREADS pairs.
    const int npair = n * (n + 1) / 2, wf = n + 1;
    int fi = tid / wf, fc = tid % wf;
    for (int pq = tid; pq < npair; pq += STHREADS) {
      const bool first = fc < n - fi;
      const int r = first ? fi : n - 1 - fi;
      const int l = first ? fi + fc : r + (fc - (n - fi));
      double c[3];
      cross_cov_block(tk.x[l], tk.y[l], tk.x[r], tk.y[r], tk.P, sq, c);
      double *a = A + (int64_t)(2 * r) * N + 2 * l;
      a[0] = c[0];
      a[1] = c[2];
      a[N] = c[2];
      a[N + 1] = c[1];
      fc += STHREADS;
      while (fc >= wf) {
        fc -= wf;
        ++fi;
      }
    }
    __syncthreads();
    for (int k0 = 0; k0 < N; k0 += SB) {
      const int kb = min(SB, N - k0);
      // (u) this block column receives all earlier columns' updates at once
      // (two at a time: the first block of a pair takes every earlier
      // column for both blocks, the second then only the first's columns)
      if (k0 > 0) {
        if ((k0 / SB) % 2 == 0)
          left_update<2 * SB / 16>(A, N, k0, min(2 * SB, N - k0), 0, part, wave, lane, tid);
        else
          left_update<SB / 16>(A, N, k0, kb, k0 - SB, part, wave, lane, tid);
        __syncthreads();
      }
      // (a) diagonal block by wave 0 in registers, without workgroup
      // barriers: lane r holds row r of the block (lanes 32..63 the same rows;
      // only lanes < 32 write).  Column c's pivot and entries come from their
      // lanes as uniform values (readlane); then W = L_kk^-1, column c by lane
      // c, and L_kk back to A.  The arithmetic per entry is that of a
      // column-by-column Cholesky and a forward substitution per column.
      if (wave == 0) {
        const int rr = lane & 31;
        const bool wl = lane < 32;
        double a[SB];
#pragma unroll
        for (int c = 0; c < SB; ++c) a[c] = clamped_load(A, N, k0 + c, k0 + rr);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < SB; ++c)
          if (!(c <= rr && rr < kb)) a[c] = 0.0;
        if (wl && lane < kb) szk[lane] = zv[k0 + lane];  // final: earlier blocks have updated it
        int fail = 0;
#pragma unroll
        for (int c = 0; c < SB; ++c) {
          if (fail || c >= kb) continue;  // uniform (no break: the loop stays unrolled)
          const double d = readlane_d(a[c], c);
          const int g = k0 + c;
          const double tol = (g & 1) ? tk.t1 : tk.t0;
          if (!(d > tol) || !(d > 0.0)) {  // uniform
            fail = g + 1;
            continue;
          }
          const double ljj = sqrt(d);
          a[c] = rr == c ? ljj : (rr > c ? a[c] / ljj : a[c]);
#pragma unroll
          for (int q = c + 1; q < SB; ++q) a[q] -= a[c] * readlane_d(a[c], q);  // rows q <= rr used
        }
        if (fail) {
          if (lane == 0) s_fail = fail;
        } else {
          double dg = 0.0;  // this lane's L_rr (static register indices)
#pragma unroll
          for (int q = 0; q < SB; ++q)
            if (q == rr) dg = a[q];
          if (wl && lane < kb) slg[lane] = log(dg);
          // column c of W by lane c (rows above c are zeros, so the sums over
          // q < c add exact zeros); entries outside the kb x kb block are zero
          const int c = rr;
          double w[SB];
#pragma unroll
          for (int r = 0; r < SB; ++r) {
            // (the right-hand side e_c enters as the 1 at r = c, where the sum
            // is over zeros: no per-lane constant held across the task loop)
            double sacc = 0.0;
#pragma unroll
            for (int q = 0; q < r; ++q) sacc -= readlane_d(a[q], r) * w[q];
            w[r] = (r >= c && r < kb) ? (r == c ? 1.0 : sacc) / readlane_d(a[r], r) : 0.0;
          }
          if (wl) {
#pragma unroll
            for (int r = 0; r < SB; ++r) sW[r][c] = w[r];
            // L_kk back to A (the solve of later columns does not need it)
            if (rr < kb)
#pragma unroll
              for (int q = 0; q < SB; ++q)
                if (q <= rr) A[(int64_t)(k0 + q) * N + k0 + rr] = a[q];
          }
        }
      }
      __syncthreads();
      if (s_fail) break;
      if (tid == 0) {
        double ld = s_logdet;
        for (int c = 0; c < kb; ++c) ld += slg[c];
        s_logdet = ld;
      }
      if (tid < SB) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < SB; ++q)
          if (q <= tid && q < kb) s += sW[tid][q] * szk[q];
        sy[tid] = tid < kb ? s : 0.0;
      }
      __syncthreads();
      if (tid == 0) {
        double q = s_quad;
        for (int c = 0; c < kb; ++c) q += sy[c] * sy[c];
        s_quad = q;
      }
      // (b) panel rows i >= k0 + kb: L_i = A_i W^T on MFMA, 16 rows per wave
      //     (a wave reads its rows' A values before it overwrites them), and
      //     the solve's z_i -= L_i y_k from the same accumulators (a row's 16
      //     columns of a half are in the 16 lanes of one DPP row)
      //     W's fragments are the same for every tile (registers); the next
      //     tile's A values are in flight while this one's feed the MFMAs
      const int r0 = k0 + kb;
      const int l16 = lane & 15, lk = lane >> 4;
      const int ntile = (N - r0 + 15) / 16;
      double wf[SB / 16][SB / 4];
#pragma unroll
      for (int half = 0; half < SB / 16; ++half)
#pragma unroll
        for (int kk = 0; kk < SB / 4; ++kk) wf[half][kk] = sW[half * 16 + l16][4 * kk + lk];
      double avn[SB / 4];
#pragma unroll
      for (int kk = 0; kk < SB / 4; ++kk)
        avn[kk] = clamped_load(A, N, k0 + 4 * kk + lk, r0 + wave * 16 + l16);
      for (int t = wave; t < ntile; t += SW) {
        const int row = r0 + t * 16 + l16;
        double av[SB / 4];
#pragma unroll
        for (int kk = 0; kk < SB / 4; ++kk) {
          av[kk] = avn[kk];
          avn[kk] = clamped_load(A, N, k0 + 4 * kk + lk, row + 16 * SW);  // next tile (clamped)
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kk = 0; kk < SB / 4; ++kk)
          if (!(row < N && 4 * kk + lk < kb)) av[kk] = 0.0;
        double zp[4] = {0.0, 0.0, 0.0, 0.0};  // rows 4 e + lk of the tile
#pragma unroll
        for (int half = 0; half < SB / 16; ++half) {
          dbl4s acc = dbl4s{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kk = 0; kk < SB / 4; ++kk)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], wf[half][kk], acc, 0, 0, 0);
          const int c = half * 16 + l16;
          const double yc = sy[c];  // zero for c >= kb
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int gi = r0 + t * 16 + 4 * e + lk;
            if (gi < N && c < kb) A[(int64_t)(k0 + c) * N + gi] = acc[e];
            zp[e] += acc[e] * yc;
          }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double zs = row16_sum(zp[e]);
          const int gi = r0 + t * 16 + 4 * e + lk;
          if (l16 == 0 && gi < N) zv[gi] -= zs;
        }
      }
      __syncthreads();
    }    if (tid == 0) {
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
  return (size_t)(N * N + N + SW * SB * 2 * SB);  // matrix, right-hand side, split partials
}

int launch_small_loglik(const SmallTask *d_tasks, int ntask, int64_t nmax, int *d_counter,
                        double *d_ws, double *d_out, hipStream_t st, int max_wg) {
  if (ntask <= 0) return 0;
  if (2 * nmax > SMALL_MAX) {
    set_error("batched small likelihood: 2n = %lld above %d", (long long)(2 * nmax), SMALL_MAX);
    return MVG_ERR_LIMIT;
  }
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, d_counter);
  if (int rc = check_launch("zero_int")) return rc;
  int G = small_batch_workgroups(ntask);
  if (max_wg > 0 && G > max_wg) G = max_wg;  // the workspace holds max_wg task slots
  hipLaunchKernelGGL(k_small_loglik, dim3(G), dim3(STHREADS), 0, st, d_tasks, ntask, d_counter, d_ws,
                     (int64_t)small_workspace_doubles(nmax), d_out);
  return check_launch("small_loglik");
}

}  // namespace mvg
