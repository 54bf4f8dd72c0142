// Batched small dense linear algebra for the tile-low-rank (TLR) path on
// gfx950 (the GEMMs are in tlr_gemm.hip): Householder QR of tall-skinny
// matrices (one workgroup per matrix, or panels over
// several launches; unpivoted, column-pivoted, or with randomized pivots and
// a Frobenius-tail stop), Gaussian sketch matrices.  One list entry per product / matrix; the TLR
// driver builds the lists on the host.
#include <cmath>

#include "tlr.h"

namespace mvg {

typedef double dbl4t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------- Householder QR
//
// A (m x n, m >= n, column-major, lda) = Q R by n Householder reflectors
// H_j = I - tau_j v_j v_j^T (v_j(j) = 1, stored below the diagonal of A; R
// above and on it).  If Q is given, the first n columns of H_0 ... H_{n-1}
// are written there (m x n, ldq).  One workgroup per matrix; column c of the
// trailing update belongs to wave c % QW throughout.
constexpr int QW = 8;  // waves per QR workgroup

// Columns c0, c0 + QW, ..., c0 + (NC-1) QW (those < n) of A, rows j..m-1, are
// replaced by (I - tau v v^T) times themselves by one wave: all their
// elements are loaded first (independent loads in flight), then the inner
// products, the wave reductions and the updates.  With nrm, the squared norm
// of each updated column's rows j+1..m-1 goes to nrm[c] (lane 0).  m <= 64 QE.
template <int QE, int NC>
__device__ __forceinline__ void reflect_cols(double *A, int lda, int c0, int n, const double *v,
                                             int j, int m, double tau, int lane, double *nrm) {
  // pass 1: inner products.  All loads of the NC columns are issued together
  // from clamped indices (inside the m x n matrix) and zeroed where masked
  // after a scheduling barrier (a load under a branch waits for its value
  // before the next); the values serve pass 2 as well.
  double w[NC];
  double x[NC][QE];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int c = min(c0 + k * QW, n - 1);
#pragma unroll
    for (int e = 0; e < QE; ++e) x[k][e] = A[(int64_t)c * lda + min(j + lane + 64 * e, m - 1)];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < NC; ++k)
#pragma unroll
    for (int e = 0; e < QE; ++e)
      if (!(c0 + k * QW < n && j + lane + 64 * e < m)) x[k][e] = 0.0;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    w[k] = 0.0;
#pragma unroll
    for (int e = 0; e < QE; ++e) {
      const int i = j + lane + 64 * e;
      if (i < m) w[k] += v[i] * x[k][e];
    }
  }
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < NC; ++k) w[k] += __shfl_xor(w[k], o);
  // pass 2: update from the values of pass 1 (only this wave writes the
  // columns c0 + k QW)
  double ss[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int c = c0 + k * QW;
    const double tw = tau * w[k];
    ss[k] = 0.0;
    if (c < n) {
      double *col = A + (int64_t)c * lda;
#pragma unroll
      for (int e = 0; e < QE; ++e) {
        const int i = j + lane + 64 * e;
        if (i < m) {
          const double y = x[k][e] - tw * v[i];
          col[i] = y;
          if (i > j) ss[k] += y * y;
        }
      }
    }
  }
  if (nrm) {
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int k = 0; k < NC; ++k) ss[k] += __shfl_xor(ss[k], o);
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < NC; ++k)
        if (c0 + k * QW < n) nrm[c0 + k * QW] = ss[k];
  }
}

// With tk.piv: column pivoting (largest remaining column norm first, ties to
// the lower index) and early stop once the Frobenius norm of the remaining
// block is <= tk.tol; *tk.rank receives the number of reflectors k, tk.piv
// the column order, and only the first k columns of Q are formed.
template <int QE, int NC>
__global__ __launch_bounds__(64 * QW) void k_qr(const QrTask *__restrict__ tasks) {
  __shared__ double v[QR_MAXM];
  __shared__ double s_tau[QR_MAXN];
  __shared__ double s_nrm[QR_MAXN];
  __shared__ int s_piv[QR_MAXN];
  __shared__ double red[QW];
  __shared__ int s_arg;
  __shared__ double s_tail;
  const QrTask tk = tasks[blockIdx.x];
  const int m = tk.m, n = tk.n, lda = tk.lda;
  double *A = tk.A;
  const bool pivot = tk.piv != nullptr;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (pivot) {
    for (int c = wave; c < n; c += QW) {
      const double *ac = A + (int64_t)c * lda;
      double ss = 0.0;
      for (int i = lane; i < m; i += 64) ss += ac[i] * ac[i];
      for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
      if (lane == 0) {
        s_nrm[c] = ss;
        s_piv[c] = c;
      }
    }
    __syncthreads();
  }
  int kmax = n;
  for (int j = 0; j < n; ++j) {
    if (pivot) {
      if (wave == 0) {
        double best = -1.0, tail = 0.0;
        int bi = n;
        for (int c = j + lane; c < n; c += 64) {
          const double t = s_nrm[c];
          tail += t;
          if (t > best) {
            best = t;
            bi = c;
          }
        }
        for (int o = 32; o > 0; o >>= 1) {
          tail += __shfl_xor(tail, o);
          const double ob = __shfl_xor(best, o);
          const int oi = __shfl_xor(bi, o);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (lane == 0) {
          s_arg = bi;
          s_tail = tail;
        }
      }
      __syncthreads();
      if (s_tail <= tk.tol * tk.tol) {  // uniform
        kmax = j;
        break;
      }
      const int p = s_arg;
      if (p != j) {
        double *aj = A + (int64_t)j * lda, *ap = A + (int64_t)p * lda;
        for (int i = tid; i < m; i += 64 * QW) {
          const double t = aj[i];
          aj[i] = ap[i];
          ap[i] = t;
        }
        if (tid == 0) {
          const double tn = s_nrm[j];
          s_nrm[j] = s_nrm[p];
          s_nrm[p] = tn;
          const int ti = s_piv[j];
          s_piv[j] = s_piv[p];
          s_piv[p] = ti;
        }
      }
      __syncthreads();
    }
    double *aj = A + (int64_t)j * lda;
    double ss = 0.0;
    for (int i = j + 1 + tid; i < m; i += 64 * QW) ss += aj[i] * aj[i];
    for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    double sigma2 = 0.0;
    for (int w = 0; w < QW; ++w) sigma2 += red[w];
    const double alpha = aj[j];
    double tau = 0.0, scale = 0.0, beta = alpha;
    if (sigma2 > 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    for (int i = j + 1 + tid; i < m; i += 64 * QW) {
      const double vi = aj[i] * scale;
      v[i] = vi;
    }
    if (tid == 0) {
      v[j] = 1.0;
      s_tau[j] = tau;
    }
    __syncthreads();
    // store the reflector below the diagonal and beta on it
    for (int i = j + 1 + tid; i < m; i += 64 * QW) aj[i] = v[i];
    if (tid == 0) aj[j] = beta;
    if (tau != 0.0 || pivot) {
      for (int c0 = j + 1 + (((wave - (j + 1)) % QW + QW) % QW); c0 < n; c0 += QW * NC)
        reflect_cols<QE, NC>(A, lda, c0, n, v, j, m, tau, lane, pivot ? s_nrm : nullptr);
    }
    __syncthreads();
  }
  if (tk.tau)
    for (int j = tid; j < kmax; j += 64 * QW) tk.tau[j] = s_tau[j];
  if (pivot) {
    for (int c = tid; c < n; c += 64 * QW) tk.piv[c] = s_piv[c];
    if (tid == 0) *tk.rank = kmax;
  }
  if (!tk.Q) return;
  double *Q = tk.Q;
  const int ldq = tk.ldq;
  for (int c = wave; c < kmax; c += QW)
    for (int i = lane; i < m; i += 64) Q[(int64_t)c * ldq + i] = (i == c) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = kmax - 1; j >= 0; --j) {
    const double tau = s_tau[j];
    const double *aj = A + (int64_t)j * lda;
    for (int i = j + 1 + tid; i < m; i += 64 * QW) v[i] = aj[i];
    if (tid == 0) v[j] = 1.0;
    __syncthreads();
    if (tau != 0.0) {
      for (int c0 = j + (((wave - j) % QW + QW) % QW); c0 < kmax; c0 += QW * NC)
        reflect_cols<QE, NC>(Q, ldq, c0, kmax, v, j, m, tau, lane, nullptr);
    }
    __syncthreads();
  }
}

// ----------------------------------------------------- blocked Householder
//
// A = Q R without pivoting, reflectors grouped in panels of QB columns
// (compact WY form H_p = I - V T V^T, Schreiber and Van Loan): a panel is
// factored column by column, then the rest of A is updated once per panel,
// A_c <- A_c - V T^T (V^T A_c), and Q = H_1 ... H_P [I; 0] is formed panel by
// panel from the last.  One workgroup per matrix; V of the current panel
// lives in LDS; the T factors go to tk.tau ((n + QB) x QB doubles, required).
constexpr int QB = 8;
constexpr int BWV = 8;  // waves per blocked-QR workgroup

template <int QE, int NC>
__device__ __forceinline__ void apply_block(double *A, int lda, int c0, int n, int p0, int m,
                                            int bw, const double (*V)[QR_MAXM], const double (*T)[QB],
                                            bool trans, int lane) {
  // columns c0, c0 + BWV, ... (< n): rows p0..m-1 <- (I - V op(T) V^T) rows
  double y[NC][QB];
#pragma unroll
  for (int k = 0; k < NC; ++k)
#pragma unroll
    for (int q = 0; q < QB; ++q) y[k][q] = 0.0;
  // the lane's rows of the columns, loaded from clamped indices (inside the
  // m x n matrix) all at once and zeroed where masked after a scheduling
  // barrier (a load under a branch waits for its value before the next);
  // kept for the final update, which therefore reads A only here
  double x[NC][QE];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int c = min(c0 + k * BWV, n - 1);
#pragma unroll
    for (int e = 0; e < QE; ++e) x[k][e] = A[(int64_t)c * lda + min(p0 + lane + 64 * e, m - 1)];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < NC; ++k)
#pragma unroll
    for (int e = 0; e < QE; ++e)
      if (!(c0 + k * BWV < n && p0 + lane + 64 * e < m)) x[k][e] = 0.0;
  {
#pragma unroll
    for (int e = 0; e < QE; ++e) {
      const int r = lane + 64 * e;
      if (p0 + r < m)
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const double vq = V[q][r];
#pragma unroll
          for (int k = 0; k < NC; ++k) y[k][q] += vq * x[k][e];
        }
      __builtin_amdgcn_sched_barrier(0);  // keep the LDS reads of V row by row
    }
  }
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int q = 0; q < QB; ++q) y[k][q] += __shfl_xor(y[k][q], o);
  // y <- op(T) y  (T upper triangular; T^T for the factorisation)
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double t[QB];
#pragma unroll
    for (int a = 0; a < QB; ++a) {
      double sacc = 0.0;
#pragma unroll
      for (int b = 0; b < QB; ++b) {
        const double tab = trans ? T[b][a] : T[a][b];
        if (a < bw && b < bw) sacc += tab * y[k][b];
      }
      t[a] = sacc;
    }
#pragma unroll
    for (int a = 0; a < QB; ++a) y[k][a] = t[a];
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int c = c0 + k * BWV;
    if (c >= n) continue;
    double *col = A + (int64_t)c * lda;
#pragma unroll
    for (int e = 0; e < QE; ++e) {
      const int r = lane + 64 * e, i = p0 + r;
      if (i < m) {
        double d = 0.0;
#pragma unroll
        for (int q = 0; q < QB; ++q) d += V[q][r] * y[k][q];
        col[i] = x[k][e] - d;  // x holds col[i]: only this wave writes column c
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int QE, int NC>
__global__ __launch_bounds__(64 * BWV) void k_qr_blocked(const QrTask *__restrict__ tasks) {
  __shared__ double V[QB][QR_MAXM];  // reflector q in V[q][.]: lane-contiguous reads
  __shared__ double T[QB][QB];
  __shared__ double G[QB][QB];
  __shared__ double s_tau[QB];
  __shared__ double red[BWV];
  const QrTask tk = tasks[blockIdx.x];
  const int m = tk.m, n = tk.n, lda = tk.lda;
  double *A = tk.A;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double *Tg = tk.tau;  // n x QB: T of panel p at rows p .. p + QB - 1
  for (int p0 = 0; p0 < n; p0 += QB) {
    const int bw = min(QB, n - p0);
    for (int e = tid; e < (m - p0) * QB; e += 64 * BWV) V[e % QB][e / QB] = 0.0;
    __syncthreads();
    // panel: reflectors of columns p0 .. p0 + bw - 1
    for (int jj = 0; jj < bw; ++jj) {
      const int j = p0 + jj;
      double *aj = A + (int64_t)j * lda;
      double ss = 0.0;
      for (int i = j + 1 + tid; i < m; i += 64 * BWV) ss += aj[i] * aj[i];
      for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
      if (lane == 0) red[wave] = ss;
      __syncthreads();
      double sigma2 = 0.0;
      for (int w = 0; w < BWV; ++w) sigma2 += red[w];
      const double alpha = aj[j];
      double tau = 0.0, scale = 0.0, beta = alpha;
      if (sigma2 > 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma2);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      for (int i = j + 1 + tid; i < m; i += 64 * BWV) V[jj][i - p0] = aj[i] * scale;
      if (tid == 0) {
        V[jj][j - p0] = 1.0;
        s_tau[jj] = tau;
      }
      __syncthreads();
      for (int i = j + 1 + tid; i < m; i += 64 * BWV) aj[i] = V[jj][i - p0];
      if (tid == 0) aj[j] = beta;
      // the remaining panel columns, one per wave
      const int c = j + 1 + wave;
      if (tau != 0.0 && c < p0 + bw) {
        double *ac = A + (int64_t)c * lda;
        // rows j + lane + 64 e (< m; 64 QE >= m): loaded at once from clamped
        // rows, used in the same order as a row-by-row loop
        double av[QE];
#pragma unroll
        for (int e = 0; e < QE; ++e) av[e] = ac[min(j + lane + 64 * e, m - 1)];
        __builtin_amdgcn_sched_barrier(0);
        double w = 0.0;
#pragma unroll
        for (int e = 0; e < QE; ++e) {
          const int i = j + lane + 64 * e;
          if (i < m) w += V[jj][i - p0] * av[e];
        }
        for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
        const double tw = tau * w;
#pragma unroll
        for (int e = 0; e < QE; ++e) {
          const int i = j + lane + 64 * e;
          if (i < m) ac[i] = av[e] - tw * V[jj][i - p0];  // only this wave writes column c
        }
      }
      __syncthreads();
    }
    // T of the panel: T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j)
    for (int q = wave; q < QB * QB; q += BWV) {
      const int a = q / QB, b = q % QB;
      double d = 0.0;
      if (a < b && b < bw)
        for (int r = lane; r < m - p0; r += 64) d += V[a][r] * V[b][r];
      for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
      if (lane == 0) G[a][b] = d;
    }
    __syncthreads();
    if (tid == 0) {
      for (int a = 0; a < QB; ++a)
        for (int b = 0; b < QB; ++b) T[a][b] = 0.0;
      for (int b = 0; b < bw; ++b) {
        T[b][b] = s_tau[b];
        for (int a = 0; a < b; ++a) {
          double sacc = 0.0;
          for (int c = a; c < b; ++c) sacc += T[a][c] * G[c][b];
          T[a][b] = -s_tau[b] * sacc;
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < QB * QB; e += 64 * BWV) Tg[(int64_t)(p0 + e / QB) * QB + e % QB] = T[e / QB][e % QB];
    // rest of A: A_c <- (I - V T^T V^T) A_c
    for (int c0 = p0 + bw + wave; c0 < n; c0 += BWV * NC)
      apply_block<QE, NC>(A, lda, c0, n, p0, m, bw, V, T, true, lane);
    __syncthreads();
  }
  if (!tk.Q) return;
  double *Q = tk.Q;
  const int ldq = tk.ldq;
  for (int c = wave; c < n; c += BWV)
    for (int i = lane; i < m; i += 64) Q[(int64_t)c * ldq + i] = (i == c) ? 1.0 : 0.0;
  for (int p0 = ((n - 1) / QB) * QB; p0 >= 0; p0 -= QB) {
    const int bw = min(QB, n - p0);
    __syncthreads();
    for (int e = tid; e < (m - p0) * QB; e += 64 * BWV) {
      const int r = e / QB, q = e % QB, i = p0 + r;
      double val = 0.0;
      if (q < bw) val = (r == q) ? 1.0 : (r > q ? A[(int64_t)(p0 + q) * lda + i] : 0.0);
      V[q][r] = val;
    }
    for (int e = tid; e < QB * QB; e += 64 * BWV) T[e / QB][e % QB] = Tg[(int64_t)(p0 + e / QB) * QB + e % QB];
    __syncthreads();
    for (int c0 = p0 + wave; c0 < n; c0 += BWV * NC)
      apply_block<QE, NC>(Q, ldq, c0, n, p0, m, bw, V, T, false, lane);
  }
}

int launch_qr_blocked(const QrTask *d_tasks, int ntask, int mmax, hipStream_t st) {
  if (ntask <= 0) return 0;
  if (mmax > QR_MAXM) {
    set_error("QR: %d rows above %d", mmax, QR_MAXM);
    return MVG_ERR_LIMIT;
  }
  const dim3 g(ntask), b(64 * BWV);
  if (mmax <= 64 * 4)
    hipLaunchKernelGGL((k_qr_blocked<4, 2>), g, b, 0, st, d_tasks);
  else if (mmax <= 64 * 8)
    hipLaunchKernelGGL((k_qr_blocked<8, 1>), g, b, 0, st, d_tasks);
  else if (mmax <= 64 * 16)
    hipLaunchKernelGGL((k_qr_blocked<16, 1>), g, b, 0, st, d_tasks);
  else if (mmax <= 64 * 20)
    hipLaunchKernelGGL((k_qr_blocked<20, 1>), g, b, 0, st, d_tasks);
  else
    hipLaunchKernelGGL((k_qr_blocked<32, 1>), g, b, 0, st, d_tasks);
  return check_launch("qr_blocked");
}

// ------------------------------------------ blocked QR over several launches
//
// The same factorisation as k_qr_blocked (compact WY panels, Schreiber and
// Van Loan), split so that one large matrix is not left to one workgroup:
// per panel of PQB columns one launch factors the panel of every task (one
// workgroup per task, the panel in registers) and one launch applies the
// panel's block reflector to the rest of A (several workgroups per task,
// PAP_CB columns each, on FP64 MFMA); Q = H_1 ... H_P [I; 0] is then formed
// panel by panel from the last by the same apply kernel.  A panel step costs
// two workgroup barriers and one wave-reduction of PQB values; the matrix
// itself stays in L2 / HBM (an nb x s sketch is up to 6 MB).
// Requirements (checked by the launcher): m % 4 == 0, n + PQB <= m <= PQ_MAXM;
// and (checked where the tasks are built) lda, ldq even and A, Q 16-byte
// aligned, for the 16-byte loads of the apply and sample kernels.
constexpr int PQB = 16;          // panel width
constexpr int PQ_MAXM = 1536;    // rows: 6 (3) per panel thread of 256 (512)
constexpr int PAP_CB = 32;       // columns per apply workgroup

// Cross-lane sums without LDS.  Inside a row of 16 lanes the exchanges are
// DPP moves: quad_perm [1,0,3,2] pairs lane i with i ^ 1, quad_perm
// [2,3,0,1] with i ^ 2, row_half_mirror with i ^ 7 and row_mirror with
// i ^ 15.  Across rows, gfx950's lane swaps exchange whole halves of two
// registers: v_permlane16_swap swaps the odd rows of its first operand with
// the even rows of its second, v_permlane32_swap lanes 32-63 of the first
// with lanes 0-31 of the second.  Each all-reduce step adds a value and its
// partner's, so a lane and its partner form the same sum in swapped order:
// every lane of a group ends with bitwise the same result.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_XOR7 = 0x141, DPP_XOR15 = 0x140;

__device__ __forceinline__ double join_d(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// x + y after swapping the odd rows of x with the even rows of y: rows 0, 2
// get x's rows 0 + 1 and 2 + 3, rows 1, 3 get y's
__device__ __forceinline__ double swap16_add(double x, double y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false,
                                                   false);
  return join_d(lo[0], hi[0]) + join_d(lo[1], hi[1]);
}

// x + y after swapping lanes 32-63 of x with lanes 0-31 of y: lanes 0-31
// get x's halves summed, lanes 32-63 y's
__device__ __forceinline__ double swap32_add(double x, double y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false,
                                                   false);
  return join_d(lo[0], hi[0]) + join_d(lo[1], hi[1]);
}

// sum over the 64 lanes, in every lane
__device__ __forceinline__ double wave_sum(double s) {
  s += dpp_d<DPP_XOR15>(s);
  s += dpp_d<DPP_XOR7>(s);
  s += dpp_d<DPP_XOR2>(s);
  s += dpp_d<DPP_XOR1>(s);
  s = swap16_add(s, s);
  return swap32_add(s, s);
}

// Sums over the 64 lanes of 16 values at once, halving the values a lane
// holds at each step (the lane keeps the half selected by one bit of its
// index and receives its partner's values of that half): lane i ends with
// the sum of value ((i >> 2) & 15), the same in the four lanes of a quad.
// The two cross-row halvings are lane swaps (no selects); the two in-row
// halvings are DPP moves with selects; the last two steps are all-reduces.
__device__ __forceinline__ double wave_sum16(const double (&d)[16], int lane) {
  double h8[8], h4[4], h2[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) h8[k] = swap32_add(d[k], d[k + 8]);   // value k + 8 (lane bit 5)
#pragma unroll
  for (int k = 0; k < 4; ++k) h4[k] = swap16_add(h8[k], h8[k + 4]); // + 4 (lane bit 4)
  const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int k = 0; k < 2; ++k) {  // + 2 (lane bit 3)
    const double keep = b3 ? h4[k + 2] : h4[k], send = b3 ? h4[k] : h4[k + 2];
    h2[k] = keep + dpp_d<DPP_XOR15>(send);
  }
  double s;
  {  // + 1 (lane bit 2)
    const double keep = b2 ? h2[1] : h2[0], send = b2 ? h2[0] : h2[1];
    s = keep + dpp_d<DPP_XOR7>(send);
  }
  s += dpp_d<DPP_XOR2>(s);
  s += dpp_d<DPP_XOR1>(s);
  return s;
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}

// (b, i) <- the larger of (b, i) and (ob, oi): larger value, ties to the
// lower index (a total order, so both partners of a step keep the same pair)
__device__ __forceinline__ void argmax_step(double &b, int &i, double ob, int oi) {
  if (ob > b || (ob == b && oi < i)) {
    b = ob;
    i = oi;
  }
}

// the pair with the largest value over the 64 lanes (ties to the lowest
// index), in every lane
__device__ __forceinline__ void wave_argmax(double &b, int &i) {
  argmax_step(b, i, dpp_d<DPP_XOR15>(b), dpp_i<DPP_XOR15>(i));
  argmax_step(b, i, dpp_d<DPP_XOR7>(b), dpp_i<DPP_XOR7>(i));
  argmax_step(b, i, dpp_d<DPP_XOR2>(b), dpp_i<DPP_XOR2>(i));
  argmax_step(b, i, dpp_d<DPP_XOR1>(b), dpp_i<DPP_XOR1>(i));
  {  // rows 2k and 2k + 1: each lane gets both rows' pairs (its own is one of them)
    const long long bb = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)bb, (unsigned)bb, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(bb >> 32), (unsigned)(bb >> 32), false,
                                                     false);
    const auto ii = __builtin_amdgcn_permlane16_swap((unsigned)i, (unsigned)i, false, false);
    b = join_d(lo[0], hi[0]);
    i = (int)ii[0];
    argmax_step(b, i, join_d(lo[1], hi[1]), (int)ii[1]);
  }
  {  // halves 0-31 and 32-63
    const long long bb = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bb, (unsigned)bb, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(bb >> 32), (unsigned)(bb >> 32), false,
                                                     false);
    const auto ii = __builtin_amdgcn_permlane32_swap((unsigned)i, (unsigned)i, false, false);
    b = join_d(lo[0], hi[0]);
    i = (int)ii[0];
    argmax_step(b, i, join_d(lo[1], hi[1]), (int)ii[1]);
  }
}

// T factors in tk.tau: panel p0 at rows p0 .. p0 + PQB - 1 of a PQB-wide
// row-major array ((n + PQB) x PQB doubles).
template <int RPT, int NT, bool UNR>
__global__ __launch_bounds__(NT) void k_qr_panel(const QrTask *__restrict__ tasks, int p0) {
  __shared__ double red_s[NT / 64];
  __shared__ double red_d[NT / 64][PQB];
  __shared__ double s_alpha;
  __shared__ double s_tau[PQB];
  __shared__ double sG[PQB][PQB + 1];  // sG[c][jj] = V[:, c]^T v_jj, c < jj
  const QrTask tk = tasks[blockIdx.x];
  const int m = tk.m, n = tk.n, lda = tk.lda;
  if (p0 >= n) return;  // uniform: this task has no panel here
  if (tk.rank && *tk.rank <= p0) return;  // pivoted form: truncated before this panel
  const int pb = min(PQB, n - p0);
  double *A = tk.A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // rows p0 + tid + NT e of the panel columns: loaded together from clamped
  // addresses, zeroed outside the matrix after a scheduling barrier
  double a[RPT][PQB];
#pragma unroll
  for (int e = 0; e < RPT; ++e) {
    const int r = min(p0 + tid + NT * e, m - 1);
#pragma unroll
    for (int c = 0; c < PQB; ++c) a[e][c] = A[(int64_t)min(p0 + c, n - 1) * lda + r];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int e = 0; e < RPT; ++e)
#pragma unroll
    for (int c = 0; c < PQB; ++c)
      if (p0 + tid + NT * e >= m || c >= pb) a[e][c] = 0.0;
  // one reflector step; with UNR the 16 steps are unrolled so that the column
  // index jj is a constant in each (no per-element selects on it)
  auto step = [&](const int jj) __attribute__((always_inline)) {
    const int j = p0 + jj;
    // squared norm of column jj below row j, and its entry on row j
    double ss = 0.0;
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
      const int r = p0 + tid + NT * e;
      double x = 0.0;
#pragma unroll
      for (int c = 0; c < PQB; ++c)
        if (c == jj) x = a[e][c];
      if (r > j) ss += x * x;
      if (r == j) s_alpha = x;
    }
    ss = wave_sum(ss);
    if (lane == 0) red_s[wave] = ss;
    __syncthreads();
    double sigma2 = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) sigma2 += red_s[w];
    const double alpha = s_alpha;
    double tau = 0.0, scale = 0.0, beta = alpha;
    if (sigma2 > 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // the reflector below row j (v_j = 1 implicit), beta on row j; then the
    // inner products of v with every other panel column: d_c for c > jj
    // (to update them), d_c = V[:, c]^T v for c < jj (for T)
    double v[RPT];
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
      const int r = p0 + tid + NT * e;
#pragma unroll
      for (int c = 0; c < PQB; ++c)
        if (c == jj) {
          if (r > j) a[e][c] *= scale;
          else if (r == j) a[e][c] = beta;
          v[e] = r > j ? a[e][c] : (r == j ? 1.0 : 0.0);
        }
    }
    double d[PQB];
#pragma unroll
    for (int c = 0; c < PQB; ++c) {
      d[c] = 0.0;
#pragma unroll
      for (int e = 0; e < RPT; ++e) d[c] += a[e][c] * v[e];
    }
    {
      const double dw = wave_sum16(d, lane);  // this wave's sum of column (lane >> 2) & 15
      if ((lane & 3) == 0) red_d[wave][lane >> 2] = dw;
    }
    __syncthreads();
    // lane c < PQB sums the waves' partials of column c in a fixed order;
    // every lane reads the 16 sums from those lanes (uniform values)
    double part = 0.0;
    if (lane < PQB)
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) part += red_d[w][lane];
    if (tid < jj) sG[tid][jj] = part;  // wave 0: column tid of V against v_jj
    if (tid == 0) s_tau[jj] = tau;
    const long long pbits = __double_as_longlong(part);
    // rows >= j of the columns right of jj: a -= tau (v^T a) v (a zero
    // multiplier leaves the other columns as they are)
#pragma unroll
    for (int c = 0; c < PQB; ++c) {
      const int lo = __builtin_amdgcn_readlane((int)pbits, c);
      const int hi = __builtin_amdgcn_readlane((int)(pbits >> 32), c);
      const double dc = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
      if (UNR && c <= jj) continue;  // constant when unrolled
      const double td = c > jj ? tau * dc : 0.0;
#pragma unroll
      for (int e = 0; e < RPT; ++e) a[e][c] -= td * v[e];
    }
  };
  if constexpr (UNR) {
#pragma unroll
    for (int jj = 0; jj < PQB; ++jj)
      if (jj < pb) step(jj);
  } else {
    for (int jj = 0; jj < pb; ++jj) step(jj);
  }
  // the panel back (R on and above the diagonal, reflectors below)
#pragma unroll
  for (int e = 0; e < RPT; ++e) {
    const int r = p0 + tid + NT * e;
    if (r < m)
#pragma unroll
      for (int c = 0; c < PQB; ++c)
        if (c < pb) A[(int64_t)(p0 + c) * lda + r] = a[e][c];
  }
  // T, row c by thread c: T_cc = tau_c, T[c][b] = -tau_b sum_{c <= l < b}
  // T[c][l] (V[:, l]^T v_b) for b > c; zero outside the pb x pb block
  __syncthreads();
  if (tid < PQB) {
    double t[PQB];
#pragma unroll
    for (int b = 0; b < PQB; ++b) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < b; ++l)
        if (l >= tid) acc += t[l] * sG[l][b];
      t[b] = (b < tid || tid >= pb || b >= pb) ? 0.0 : (b == tid ? s_tau[b] : -s_tau[b] * acc);
    }
    double *Tg = tk.tau + (int64_t)(p0 + tid) * PQB;
#pragma unroll
    for (int b = 0; b < PQB; ++b) Tg[b] = t[b];
  }
}

// X <- (I - V op(T) V^T) X on rows p0 .. m-1, for PAP_CB columns of X per
// workgroup.  V: the panel's reflectors (columns p0 .. p0 + pb - 1 of tk.A,
// unit on row p0 + q, zero above).  MODE 0 (factorisation): X = columns
// p0 + pb + PAP_CB b of tk.A, op(T) = T^T.  MODE 1 (forming Q): X = columns
// p0 + PAP_CB b of tk.Q, op(T) = T.
// W = V^T X runs on v_mfma_f64_16x16x4f64 with the contraction over rows:
// in K-step s lane l holds row r0 + 4 (l / 16) + s, so a lane's four rows
// are consecutive (one 32-byte load per column); then W' = op(T) W in LDS;
// then X -= V W' on the same MFMA with X tiles as accumulators.
template <int MODE, int NTH>
__device__ __forceinline__ void apply_panel(const QrTask &tk, const int p0, const int c0) {
  __shared__ double sW[NTH / 64][PQB][PAP_CB + 1];
  __shared__ double sN[PQB][PAP_CB + 1];  // -op(T) W
  __shared__ double sT[PQB][PQB + 1];
  __shared__ double sC[NTH / 64][PAP_CB];
  const int m = tk.m, n = tk.n, lda = tk.lda;
  const int pb = min(PQB, n - p0);
  double *X = MODE == 0 ? tk.A : tk.Q;
  const int ldx = MODE == 0 ? lda : tk.ldq;
  const int M = m - p0;  // rows of the block (a multiple of 4)
  const double *V = tk.A + (int64_t)p0 * lda + p0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int qv = min(l16, pb - 1);                      // clamped reflector column
  const int xc0 = min(c0 + l16, n - 1), xc1 = min(c0 + 16 + l16, n - 1);
  const bool xok0 = c0 + l16 < n, xok1 = c0 + 16 + l16 < n;
  const int nchunk = (M + 15) / 16;
  // ---- W = V^T X
  dbl4t acc[2] = {dbl4t{0.0, 0.0, 0.0, 0.0}, dbl4t{0.0, 0.0, 0.0, 0.0}};
  // two chunks per iteration (ch and ch + 4 waves), all their loads issued
  // together; a chunk past the end is read from clamped rows and masked
  constexpr int NW = NTH / 64;
  for (int ch = wave; ch < nchunk; ch += 2 * NW) {
    double vv[2][4], x0[2][4], x1[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      // the lane's 4 rows as two 16-byte loads per column (even offsets:
      // lda, ldx and p0 are even, rl a multiple of 4)
      const int rl = min(16 * (ch + u * NW) + 4 * lk, M - 4);  // in bounds (M % 4 == 0)
      const double2 *pv = (const double2 *)(V + (int64_t)qv * lda + rl);
      const double2 *pa = (const double2 *)(X + (int64_t)xc0 * ldx + p0 + rl);
      const double2 *pc = (const double2 *)(X + (int64_t)xc1 * ldx + p0 + rl);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double2 v2 = pv[h], a2 = pa[h], c2 = pc[h];
        vv[u][2 * h] = v2.x;
        vv[u][2 * h + 1] = v2.y;
        x0[u][2 * h] = a2.x;
        x0[u][2 * h + 1] = a2.y;
        x1[u][2 * h] = c2.x;
        x1[u][2 * h + 1] = c2.y;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int rr = 16 * (ch + u * NW) + 4 * lk;  // first of the lane's 4 rows
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int r = rr + s;
        const bool rok = r < M;
        double vq = vv[u][s];
        if (r < l16) vq = 0.0;            // above the unit diagonal of V
        else if (r == l16) vq = 1.0;
        if (!rok || l16 >= pb) vq = 0.0;
        const double xa = (rok && xok0) ? x0[u][s] : 0.0;
        const double xb = (rok && xok1) ? x1[u][s] : 0.0;
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(vq, xa, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(vq, xb, acc[1], 0, 0, 0);
      }
    }
  }
  // D[q][c] of a 16 x 16 tile: lane c + 16 (q % 4), element q / 4
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int e = 0; e < 4; ++e) sW[wave][4 * e + lk][16 * h + l16] = acc[h][e];
  if (tid < PQB * PQB) {
    const int i = tid / PQB, k = tid % PQB;
    sT[i][k] = tk.tau[(int64_t)(p0 + i) * PQB + k];
  }
  __syncthreads();
  // the four waves' partial sums, in a fixed order
  for (int o = tid; o < PQB * PAP_CB; o += NTH) {
    const int q = o / PAP_CB, c = o % PAP_CB;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NTH / 64; ++w) t += sW[w][q][c];
    sW[0][q][c] = t;
  }
  __syncthreads();
  for (int o = tid; o < PQB * PAP_CB; o += NTH) {
    const int q = o / PAP_CB, c = o % PAP_CB;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < PQB; ++k) t += (MODE == 0 ? sT[k][q] : sT[q][k]) * sW[0][k][c];
    sN[q][c] = -t;
  }
  __syncthreads();
  // ---- X -= V W', as X^T -= W'^T V^T so that a lane's accumulator holds
  // one row of 8 columns (16 lanes: 16 consecutive rows of a column per
  // load / store); accumulators start from X.  With tk.work (pivoted form,
  // MODE 0) also the squared norms of the updated columns below the panel's
  // rows (rows p0 + pb ..), for the truncation test.
  double css[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  double nq[4][2];  // -W'^T operands of this lane: q = 4 s + lk, column 16 h + l16
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int h = 0; h < 2; ++h) nq[s][h] = sN[4 * s + lk][16 * h + l16];
  int xcol[2][4];  // clamped columns of this lane's accumulator elements
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int e = 0; e < 4; ++e) xcol[h][e] = min(c0 + 16 * h + 4 * e + lk, n - 1);
  for (int ch = wave; ch < nchunk; ch += 2 * NW) {
    double va[2][4];
    dbl4t xt[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int rv = min(16 * (ch + u * NW) + l16, M - 1);  // this lane's row
#pragma unroll
      for (int s = 0; s < 4; ++s) va[u][s] = V[(int64_t)min(4 * s + lk, pb - 1) * lda + rv];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) xt[u][h][e] = X[(int64_t)xcol[h][e] * ldx + p0 + rv];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r = 16 * (ch + u * NW) + l16;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int q = 4 * s + lk;
        double vq = va[u][s];
        if (r < q) vq = 0.0;
        else if (r == q) vq = 1.0;
        if (r >= M || q >= pb) vq = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
          xt[u][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(nq[s][h], vq, xt[u][h], 0, 0, 0);
      }
      if (r < M) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (c0 + 16 * h + 4 * e + lk < n) X[(int64_t)xcol[h][e] * ldx + p0 + r] = xt[u][h][e];
        if (r >= pb)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) css[h][e] += xt[u][h][e] * xt[u][h][e];
      }
    }
  }
  if (MODE == 0 && tk.work) {
    // the 16 lanes (rows) of a column in a fixed order, then the waves in a
    // fixed order
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double c = css[h][e];
        c += dpp_d<DPP_XOR15>(c);
        c += dpp_d<DPP_XOR7>(c);
        c += dpp_d<DPP_XOR2>(c);
        c += dpp_d<DPP_XOR1>(c);
        if (l16 == 0) sC[wave][16 * h + 4 * e + lk] = c;
      }
    __syncthreads();
    if (tid < PAP_CB && c0 + tid < n) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NTH / 64; ++w) t += sC[w][tid];
      tk.work[(int64_t)QRS_ROWS * (m + n) + c0 + tid] = t;
    }
  }
}

template <int MODE, int NTH>
__global__ __launch_bounds__(NTH) void k_qr_apply(const QrTask *__restrict__ tasks, int p0,
                                                          int nblk) {
  const QrTask tk = tasks[blockIdx.x / nblk];
  const int n = tk.n;
  if (p0 >= n) return;
  if (MODE == 1 && !tk.Q) return;
  if (tk.rank && *tk.rank <= p0) return;  // pivoted form: truncated before this panel
  const int pb = min(PQB, n - p0);
  const int c0 = (MODE == 0 ? p0 + pb : p0) + PAP_CB * (blockIdx.x % nblk);
  if (c0 >= n) return;  // uniform per workgroup
  apply_panel<MODE, NTH>(tk, p0, c0);
}

// Q = H_1 ... H_P [I; 0] in one launch: a workgroup owns PAP_CB columns of Q
// (columns are transformed independently), sets them to [I; 0] and applies
// the panels' block reflectors from the last to the first.  A panel at p0
// leaves columns left of p0 unchanged (their rows from p0 down are zero), so
// the workgroup skips the panels right of its columns; the arithmetic per
// column is that of the apply kernel launched once per panel.
template <int NTH>
__global__ __launch_bounds__(NTH) void k_qr_formq(const QrTask *__restrict__ tasks, int nblk) {
  const QrTask tk = tasks[blockIdx.x / nblk];
  if (!tk.Q) return;
  const int n = tk.n, m = tk.m;
  const int c0 = PAP_CB * (blockIdx.x % nblk);
  if (c0 >= n) return;  // uniform per workgroup
  for (int c = c0; c < min(c0 + PAP_CB, n); ++c)
    for (int i = threadIdx.x; i < m; i += NTH) tk.Q[(int64_t)c * tk.ldq + i] = (i == c) ? 1.0 : 0.0;
  __syncthreads();
  const int last = min(n - 1, c0 + PAP_CB - 1);
  const int plim = tk.rank ? min(n, *tk.rank) : n;  // pivoted form: panels before the rank
  for (int p0 = ((n - 1) / PQB) * PQB; p0 >= 0; p0 -= PQB) {
    if (p0 > last || p0 >= plim) continue;  // uniform
    apply_panel<1, NTH>(tk, p0, c0);
    __syncthreads();
  }
}

// ------------------------------------------------ randomized pivoted QR
//
// Column-pivoted Householder QR stopped at the first k with a trailing
// Frobenius norm <= tk.tol (the contract of k_qr's pivoted form), for tall
// matrices, built from the panel kernels above.  Per panel of PQB columns:
// a Gaussian sample G = Omega^T A_trail (QRS_ROWS rows) of the trailing
// matrix; PQB pivots by column-pivoted QR of G (exact column norms of the
// small sample at every step); the pivots' columns swapped into place (all
// rows of A); the unpivoted panel factorisation and block-reflector update;
// then the truncation test.  Randomized pivot selection from a sample with
// oversampling: Martinsson, Quintana-Orti, Heavner and van de Geijn (2017);
// Duersch and Gu (2017).  The truncation test is exact whatever the pivots:
// after the panel, the tail after j reflectors (j inside the panel) is
//   ||A_trail||_F^2 + sum_{j < i < p0 + PQB} ||R(i, i:n)||^2,
// a sum of non-negative terms (orthogonal reflectors keep the norms of the
// rows they act on), so no cancellation.
// tk.work: Omega (m x QRS_ROWS, column-major, standard normal, filled by the
// caller) | G (QRS_ROWS x n) | squared column norms of the trailing block (n).

__global__ void k_qr_rinit(const QrTask *__restrict__ tasks) {
  const QrTask tk = tasks[blockIdx.x];
  for (int c = threadIdx.x; c < tk.n; c += blockDim.x) tk.piv[c] = c;
  if (threadIdx.x == 0) *tk.rank = tk.n;
}

// G[:, c] = Omega(0 : m - q0, :)^T A(q0 : m, c) for columns c >= q0, PAP_CB
// columns per workgroup (same MFMA layout as the first product of k_qr_apply).
template <int NTH>
__global__ __launch_bounds__(NTH) void k_qr_sample(const QrTask *__restrict__ tasks, int q0,
                                                           int nblk) {
  __shared__ double sW[NTH / 64][QRS_ROWS][PAP_CB + 1];
  const QrTask tk = tasks[blockIdx.x / nblk];
  const int b = blockIdx.x % nblk;
  const int m = tk.m, n = tk.n, lda = tk.lda;
  if (q0 >= n || *tk.rank <= q0) return;
  const int c0 = q0 + PAP_CB * b;
  if (c0 >= n) return;
  const int M = m - q0;
  const double *Om = tk.work;  // Omega[r][q] at Om[q m + r]
  double *G = tk.work + (int64_t)QRS_ROWS * m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int xc0 = min(c0 + l16, n - 1), xc1 = min(c0 + 16 + l16, n - 1);
  const bool xok0 = c0 + l16 < n, xok1 = c0 + 16 + l16 < n;
  const int nchunk = (M + 15) / 16;
  dbl4t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4t{0.0, 0.0, 0.0, 0.0};
  for (int ch = wave; ch < nchunk; ch += NTH / 64) {
    const int rr = 16 * ch + 4 * lk;
    const int rl = min(rr, M - 4);
    double o0[4], o1[4], x0[4], x1[4];
    {  // two 16-byte loads per column (m, lda and q0 even, rl a multiple of 4)
      const double2 *p0 = (const double2 *)(Om + (int64_t)l16 * m + rl);
      const double2 *p1 = (const double2 *)(Om + (int64_t)(16 + l16) * m + rl);
      const double2 *pa = (const double2 *)(tk.A + (int64_t)xc0 * lda + q0 + rl);
      const double2 *pc = (const double2 *)(tk.A + (int64_t)xc1 * lda + q0 + rl);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double2 a = p0[h], b = p1[h], c = pa[h], d = pc[h];
        o0[2 * h] = a.x;
        o0[2 * h + 1] = a.y;
        o1[2 * h] = b.x;
        o1[2 * h + 1] = b.y;
        x0[2 * h] = c.x;
        x0[2 * h + 1] = c.y;
        x1[2 * h] = d.x;
        x1[2 * h + 1] = d.y;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool rok = rr + s < M;
      const double a0 = rok ? o0[s] : 0.0, a1 = rok ? o1[s] : 0.0;
      const double xa = (rok && xok0) ? x0[s] : 0.0;
      const double xb = (rok && xok1) ? x1[s] : 0.0;
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, xa, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, xb, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, xa, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, xb, acc[1][1], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) sW[wave][16 * i + 4 * e + lk][16 * j + l16] = acc[i][j][e];
  __syncthreads();
  for (int o = tid; o < QRS_ROWS * PAP_CB; o += NTH) {
    const int q = o % QRS_ROWS, c = o / QRS_ROWS;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NTH / 64; ++w) t += sW[w][q][c];
    if (c0 + c < n) G[(int64_t)(c0 + c) * QRS_ROWS + q] = t;
  }
}

// PQB pivots for the panel at p0 from the sample G(:, p0:n): column-pivoted
// Householder QR of G (largest remaining column norm, ties to the lower
// index; exact norms every step), then the same column swaps on A (all m
// rows, in order) and on tk.piv.  One workgroup per task; each thread keeps
// the sample columns c = tid + 256 k in registers (QRS_ROWS values each).
constexpr int PICK_THREADS = 256;
constexpr int PICK_COLS = QR_MAXN / PICK_THREADS;  // columns per thread

__global__ __launch_bounds__(PICK_THREADS) void k_qr_pick(const QrTask *__restrict__ tasks, int p0) {
  __shared__ double s_best[PICK_THREADS / 64];
  __shared__ int s_bidx[PICK_THREADS / 64];
  __shared__ double scol[2][QRS_ROWS];  // the two columns of a swap
  __shared__ double sv[QRS_ROWS];
  __shared__ int sswap[PQB];
  __shared__ int smove[2][2 * PQB];  // positions moved to, and the start of their columns
  __shared__ double s_tau;
  const QrTask tk = tasks[blockIdx.x];
  const int m = tk.m, n = tk.n, lda = tk.lda;
  if (p0 >= n || *tk.rank <= p0) return;
  const int nrem = n - p0, steps = min(PQB, nrem);
  const double *G = tk.work + (int64_t)QRS_ROWS * m + (int64_t)p0 * QRS_ROWS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double g[PICK_COLS][QRS_ROWS];
#pragma unroll
  for (int k = 0; k < PICK_COLS; ++k) {
    const int c = min(tid + PICK_THREADS * k, nrem - 1);
#pragma unroll
    for (int i = 0; i < QRS_ROWS; ++i) g[k][i] = G[(int64_t)c * QRS_ROWS + i];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < PICK_COLS; ++k)
    if (tid + PICK_THREADS * k >= nrem)
#pragma unroll
      for (int i = 0; i < QRS_ROWS; ++i) g[k][i] = 0.0;
  for (int t = 0; t < steps; ++t) {
    // the thread's largest remaining norm (rows t ..), ties to the lower column
    double best = -1.0;
    int bi = nrem;
#pragma unroll
    for (int k = 0; k < PICK_COLS; ++k) {
      const int c = tid + PICK_THREADS * k;
      double ss = 0.0;
#pragma unroll
      for (int i = 0; i < QRS_ROWS; ++i)
        if (i >= t) ss += g[k][i] * g[k][i];
      if (c >= t && c < nrem && ss > best) {
        best = ss;
        bi = c;
      }
    }
    wave_argmax(best, bi);
    if (lane == 0) {
      s_best[wave] = best;
      s_bidx[wave] = bi;
    }
    __syncthreads();
    int pcol = s_bidx[0];
    double pb = s_best[0];
#pragma unroll
    for (int w = 1; w < PICK_THREADS / 64; ++w)
      if (s_best[w] > pb || (s_best[w] == pb && s_bidx[w] < pcol)) {
        pb = s_best[w];
        pcol = s_bidx[w];
      }
    if (tid == 0) sswap[t] = pcol;
    // swap columns t and pcol through LDS (t < PQB: thread t, slot 0)
    if (pcol != t) {
#pragma unroll
      for (int k = 0; k < PICK_COLS; ++k) {
        const int c = tid + PICK_THREADS * k;
        if (c == pcol)
#pragma unroll
          for (int i = 0; i < QRS_ROWS; ++i) scol[0][i] = g[k][i];
        if (c == t)
#pragma unroll
          for (int i = 0; i < QRS_ROWS; ++i) scol[1][i] = g[k][i];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < PICK_COLS; ++k) {
        const int c = tid + PICK_THREADS * k;
        if (c == pcol)
#pragma unroll
          for (int i = 0; i < QRS_ROWS; ++i) g[k][i] = scol[1][i];
        if (c == t)
#pragma unroll
          for (int i = 0; i < QRS_ROWS; ++i) g[k][i] = scol[0][i];
      }
    }
    // reflector of column t (rows t ..), by its owner: thread t, slot 0
    if (tid == t) {
      double ss = 0.0, alpha = 0.0;
#pragma unroll
      for (int i = 0; i < QRS_ROWS; ++i) {
        if (i > t) ss += g[0][i] * g[0][i];
        if (i == t) alpha = g[0][i];
      }
      double tau = 0.0, scale = 0.0;
      if (ss > 0.0) {
        const double nrm = sqrt(alpha * alpha + ss);
        const double beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int i = 0; i < QRS_ROWS; ++i) sv[i] = i > t ? g[0][i] * scale : (i == t ? 1.0 : 0.0);
      s_tau = tau;
    }
    __syncthreads();
    const double tau = s_tau;
    double v[QRS_ROWS];
#pragma unroll
    for (int i = 0; i < QRS_ROWS; ++i) v[i] = sv[i];
#pragma unroll
    for (int k = 0; k < PICK_COLS; ++k) {
      const int c = tid + PICK_THREADS * k;
      if (c > t && c < nrem) {
        double w = 0.0;
#pragma unroll
        for (int i = 0; i < QRS_ROWS; ++i) w += v[i] * g[k][i];
#pragma unroll
        for (int i = 0; i < QRS_ROWS; ++i) g[k][i] -= tau * w * v[i];
      }
    }
    __syncthreads();  // s_best, scol, sv and s_tau are rewritten next step
  }
  // The swaps (t, sswap[t]) in sequence, applied at once: every position a
  // swap touches (t, or sswap[t]) receives the column that started at
  // src(q), found by undoing the swaps from the last; a thread moves its rows
  // of all those columns (all loads before any store; repeated positions
  // move the same value twice), and the column order likewise.
  if (tid < 2 * steps) {
    const int q = tid < steps ? tid : sswap[tid - steps];
    int src = q;
    for (int t = steps - 1; t >= 0; --t) {
      const int pc = sswap[t];
      if (src == t) src = pc;
      else if (src == pc) src = t;
    }
    smove[0][tid] = q;
    smove[1][tid] = src;
  }
  __syncthreads();
  const int nmv = 2 * steps;
  int pv = 0;
  if (tid < nmv) pv = tk.piv[p0 + smove[1][tid]];
  for (int r0 = 0; r0 < m; r0 += PICK_THREADS) {
    const int r = min(r0 + tid, m - 1);
    double val[2 * PQB];
#pragma unroll
    for (int k = 0; k < 2 * PQB; ++k)
      val[k] = tk.A[(int64_t)(p0 + smove[1][min(k, nmv - 1)]) * lda + r];
    __builtin_amdgcn_sched_barrier(0);
    if (r0 + tid < m)
#pragma unroll
      for (int k = 0; k < 2 * PQB; ++k)
        if (k < nmv) tk.A[(int64_t)(p0 + smove[0][k]) * lda + r] = val[k];
  }
  __syncthreads();  // every piv read above precedes the writes
  if (tid < nmv) tk.piv[p0 + smove[0][tid]] = pv;
}

// Truncation test after the panel at p0 (one workgroup per task): squared
// norms r_i of the panel's rows of R (columns i .. n - 1) and of the
// trailing block (from the column norms k_qr_apply left in tk.work), then
// the first k (p0 <= k <= p0 + pb, k = 0 also tested on the first panel)
// whose tail is <= tol; *tk.rank = k when found.  Fixed summation orders.
__global__ __launch_bounds__(256) void k_qr_tail(const QrTask *__restrict__ tasks, int p0) {
  __shared__ double red[256];
  __shared__ double srow[PQB][17];
  const QrTask tk = tasks[blockIdx.x];
  const int m = tk.m, n = tk.n, lda = tk.lda;
  if (p0 >= n || *tk.rank <= p0) return;
  const int pb = min(PQB, n - p0), c1 = p0 + pb;
  const int tid = threadIdx.x;
  const double *cn = tk.work + (int64_t)QRS_ROWS * (m + n);
  double t = 0.0;
  for (int c = c1 + tid; c < n; c += 256) t += cn[c];
  red[tid] = t;
  // rows of R: thread (i, g) = (tid % 16, tid / 16) sums columns i + g, i + g + 16, ...
  {
    const int i = tid % PQB, g = tid / PQB;
    double r = 0.0;
    if (i < pb)
      for (int c = p0 + i + g; c < n; c += 16) {
        const double v = tk.A[(int64_t)c * lda + p0 + i];
        r += v * v;
      }
    srow[i][g] = r;
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    double ri[PQB];
    for (int i = 0; i < PQB; ++i) {
      double r = 0.0;
      for (int g = 0; g < 16; ++g) r += srow[i][g];
      ri[i] = r;
    }
    // tailsq[k - p0] = squared tail after k reflectors, k = p0 .. c1
    double tailsq[PQB + 1];
    double acc = red[0];
    tailsq[pb] = acc;
    for (int k = c1 - 1; k >= p0; --k) {
      acc += ri[k - p0];
      tailsq[k - p0] = acc;
    }
    const double tol2 = tk.tol * tk.tol;
    int found = -1;
    for (int k = (p0 == 0 ? p0 : p0 + 1); k <= c1 && found < 0; ++k)
      if (tailsq[k - p0] <= tol2) found = k;
    if (found >= 0) *tk.rank = found;
  }
}

__global__ void k_qr_qinit(const QrTask *__restrict__ tasks, int nblk) {
  // Q = [I; 0]: one workgroup per (task, 64 columns)
  const QrTask tk = tasks[blockIdx.x / nblk];
  if (!tk.Q) return;
  const int c0 = 64 * (blockIdx.x % nblk);
  for (int c = c0; c < min(c0 + 64, tk.n); ++c)
    for (int i = threadIdx.x; i < tk.m; i += blockDim.x)
      tk.Q[(int64_t)c * tk.ldq + i] = (i == c) ? 1.0 : 0.0;
}

// Panel workgroup size: 256 threads (rows per thread ceil(m / 256)) or 512
// (MVG_QR_PANEL_THREADS=512, experiments); reflector steps unrolled unless
// MVG_QR_PANEL_UNROLL=0 (experiments).
static int panel_threads() {
  static const int t = [] {
    const char *e = getenv("MVG_QR_PANEL_THREADS");
    return e && atoi(e) == 512 ? 512 : 256;
  }();
  return t;
}

static bool panel_unroll() {
  static const bool u = [] {
    const char *e = getenv("MVG_QR_PANEL_UNROLL");
    return !(e && atoi(e) == 0);
  }();
  return u;
}

template <bool UNR>
static void launch_panel_t(const QrTask *d_tasks, int ntask, int mmax, int p0, hipStream_t st) {
  const dim3 g(ntask);
  if (panel_threads() == 512) {
    const int rpt = (mmax + 511) / 512;
    if (rpt == 1)
      hipLaunchKernelGGL((k_qr_panel<1, 512, UNR>), g, dim3(512), 0, st, d_tasks, p0);
    else if (rpt == 2)
      hipLaunchKernelGGL((k_qr_panel<2, 512, UNR>), g, dim3(512), 0, st, d_tasks, p0);
    else
      hipLaunchKernelGGL((k_qr_panel<3, 512, UNR>), g, dim3(512), 0, st, d_tasks, p0);
    return;
  }
  const int rpt = (mmax + 255) / 256;
  switch (rpt) {
    case 1: hipLaunchKernelGGL((k_qr_panel<1, 256, UNR>), g, dim3(256), 0, st, d_tasks, p0); break;
    case 2: hipLaunchKernelGGL((k_qr_panel<2, 256, UNR>), g, dim3(256), 0, st, d_tasks, p0); break;
    case 3: hipLaunchKernelGGL((k_qr_panel<3, 256, UNR>), g, dim3(256), 0, st, d_tasks, p0); break;
    case 4: hipLaunchKernelGGL((k_qr_panel<4, 256, UNR>), g, dim3(256), 0, st, d_tasks, p0); break;
    case 5: hipLaunchKernelGGL((k_qr_panel<5, 256, UNR>), g, dim3(256), 0, st, d_tasks, p0); break;
    default: hipLaunchKernelGGL((k_qr_panel<6, 256, UNR>), g, dim3(256), 0, st, d_tasks, p0); break;
  }
}

static void launch_panel(const QrTask *d_tasks, int ntask, int mmax, int p0, hipStream_t st) {
  if (panel_unroll())
    launch_panel_t<true>(d_tasks, ntask, mmax, p0, st);
  else
    launch_panel_t<false>(d_tasks, ntask, mmax, p0, st);
}

// Apply / sample workgroup size: 512 threads (8 waves share a column
// block's rows), or 256 by MVG_QR_APPLY_THREADS=256 (experiments).  There is
// no 1024-thread form: at 128 registers per lane it spills, and a run of it
// took a GPU memory fault whose cause was not found.
static int apply_threads() {
  static const int t = [] {
    const char *e = getenv("MVG_QR_APPLY_THREADS");
    return e && atoi(e) == 256 ? 256 : 512;
  }();
  return t;
}

template <int MODE>
static void launch_apply(const QrTask *d_tasks, int ntask, int nblk, int p0, hipStream_t st) {
  const dim3 g(ntask * nblk);
  switch (apply_threads()) {
    case 256: hipLaunchKernelGGL((k_qr_apply<MODE, 256>), g, dim3(256), 0, st, d_tasks, p0, nblk); break;
    default: hipLaunchKernelGGL((k_qr_apply<MODE, 512>), g, dim3(512), 0, st, d_tasks, p0, nblk); break;
  }
}

// Q formation in one launch (k_qr_formq) unless MVG_QR_FORMQ_FUSED=0
// (experiments: one apply launch per panel).
static bool formq_fused() {
  static const bool f = [] {
    const char *e = getenv("MVG_QR_FORMQ_FUSED");
    return !(e && atoi(e) == 0);
  }();
  return f;
}

static void launch_formq(const QrTask *d_tasks, int ntask, int nmax, hipStream_t st) {
  const int nblk = (nmax + PAP_CB - 1) / PAP_CB;
  const dim3 g(ntask * nblk);
  switch (apply_threads()) {
    case 256: hipLaunchKernelGGL((k_qr_formq<256>), g, dim3(256), 0, st, d_tasks, nblk); break;
    default: hipLaunchKernelGGL((k_qr_formq<512>), g, dim3(512), 0, st, d_tasks, nblk); break;
  }
}

static void launch_sample(const QrTask *d_tasks, int ntask, int sblk, int p0, hipStream_t st) {
  const dim3 g(ntask * sblk);
  switch (apply_threads()) {
    case 256: hipLaunchKernelGGL((k_qr_sample<256>), g, dim3(256), 0, st, d_tasks, p0, sblk); break;
    default: hipLaunchKernelGGL((k_qr_sample<512>), g, dim3(512), 0, st, d_tasks, p0, sblk); break;
  }
}

bool qr_panels_ok(int mmin, int mmax, int nmax) {
  return mmax <= PQ_MAXM && (mmin % 4) == 0 && (mmax % 4) == 0 && nmax + PQB <= mmin;
}

int launch_qr_panels(const QrTask *d_tasks, int ntask, int mmax, int nmax, bool with_q,
                     hipStream_t st) {
  if (ntask <= 0 || nmax <= 0) return 0;
  if (mmax > PQ_MAXM) {
    set_error("QR: %d rows above %d", mmax, PQ_MAXM);
    return MVG_ERR_LIMIT;
  }
  for (int p0 = 0; p0 < nmax; p0 += PQB) {
    launch_panel(d_tasks, ntask, mmax, p0, st);
    if (int rc = check_launch("qr_panel")) return rc;
    const int rest = nmax - p0 - PQB;
    if (rest > 0) {
      const int nblk = (rest + PAP_CB - 1) / PAP_CB;
      launch_apply<0>(d_tasks, ntask, nblk, p0, st);
      if (int rc = check_launch("qr_apply")) return rc;
    }
  }
  if (!with_q) return 0;
  if (formq_fused()) {
    launch_formq(d_tasks, ntask, nmax, st);
    return check_launch("qr_formq");
  }
  const int qb = (nmax + 63) / 64;
  hipLaunchKernelGGL(k_qr_qinit, dim3(ntask * qb), dim3(256), 0, st, d_tasks, qb);
  if (int rc = check_launch("qr_qinit")) return rc;
  for (int p0 = ((nmax - 1) / PQB) * PQB; p0 >= 0; p0 -= PQB) {
    const int nblk = (nmax - p0 + PAP_CB - 1) / PAP_CB;
    launch_apply<1>(d_tasks, ntask, nblk, p0, st);
    if (int rc = check_launch("qr_apply")) return rc;
  }
  return 0;
}

bool qrcp_panels_ok(int mmin, int mmax, int nmax) {
  return qr_panels_ok(mmin, mmax, nmax) && nmax <= QR_MAXN;
}

int launch_qrcp_panels(const QrTask *d_tasks, int ntask, int mmax, int nmax, hipStream_t st) {
  if (ntask <= 0 || nmax <= 0) return 0;
  if (mmax > PQ_MAXM || nmax > QR_MAXN) {
    set_error("pivoted QR: %d x %d above %d x %d", mmax, nmax, PQ_MAXM, QR_MAXN);
    return MVG_ERR_LIMIT;
  }
  hipLaunchKernelGGL(k_qr_rinit, dim3(ntask), dim3(256), 0, st, d_tasks);
  if (int rc = check_launch("qr_rinit")) return rc;
  for (int p0 = 0; p0 < nmax; p0 += PQB) {
    const int sblk = (nmax - p0 + PAP_CB - 1) / PAP_CB;
    launch_sample(d_tasks, ntask, sblk, p0, st);
    if (int rc = check_launch("qr_sample")) return rc;
    hipLaunchKernelGGL(k_qr_pick, dim3(ntask), dim3(PICK_THREADS), 0, st, d_tasks, p0);
    if (int rc = check_launch("qr_pick")) return rc;
    launch_panel(d_tasks, ntask, mmax, p0, st);
    if (int rc = check_launch("qr_panel")) return rc;
    const int rest = nmax - p0 - PQB;
    if (rest > 0) {
      const int nblk = (rest + PAP_CB - 1) / PAP_CB;
      launch_apply<0>(d_tasks, ntask, nblk, p0, st);
      if (int rc = check_launch("qr_apply")) return rc;
    }
    hipLaunchKernelGGL(k_qr_tail, dim3(ntask), dim3(256), 0, st, d_tasks, p0);
    if (int rc = check_launch("qr_tail")) return rc;
  }
  if (formq_fused()) {
    launch_formq(d_tasks, ntask, nmax, st);
    return check_launch("qr_formq");
  }
  const int qb = (nmax + 63) / 64;
  hipLaunchKernelGGL(k_qr_qinit, dim3(ntask * qb), dim3(256), 0, st, d_tasks, qb);
  if (int rc = check_launch("qr_qinit")) return rc;
  for (int p0 = ((nmax - 1) / PQB) * PQB; p0 >= 0; p0 -= PQB) {
    const int nblk = (nmax - p0 + PAP_CB - 1) / PAP_CB;
    launch_apply<1>(d_tasks, ntask, nblk, p0, st);
    if (int rc = check_launch("qr_apply")) return rc;
  }
  return 0;
}

int launch_qr(const QrTask *d_tasks, int ntask, int mmax, hipStream_t st) {
  if (ntask <= 0) return 0;
  if (mmax > QR_MAXM) {
    set_error("QR: %d rows above %d", mmax, QR_MAXM);
    return MVG_ERR_LIMIT;
  }
  const dim3 g(ntask), b(64 * QW);
  if (mmax <= 64 * 4)
    hipLaunchKernelGGL((k_qr<4, 8>), g, b, 0, st, d_tasks);
  else if (mmax <= 64 * 8)
    hipLaunchKernelGGL((k_qr<8, 6>), g, b, 0, st, d_tasks);
  else if (mmax <= 64 * 16)
    hipLaunchKernelGGL((k_qr<16, 3>), g, b, 0, st, d_tasks);
  else if (mmax <= 64 * 20)
    hipLaunchKernelGGL((k_qr<20, 2>), g, b, 0, st, d_tasks);
  else
    hipLaunchKernelGGL((k_qr<32, 1>), g, b, 0, st, d_tasks);
  return check_launch("qr");
}


// -------------------------------------------------------- Gaussian sketch
//
// Philox4x32-10 (Salmon et al., SC'11) keyed by (seed, stream), counter =
// element index; Box-Muller turns two 32-bit words into a standard normal.
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__global__ void k_gaussian(const SketchTask *__restrict__ tasks) {
  const SketchTask tk = tasks[blockIdx.y];
  const int64_t total = (int64_t)tk.rows * tk.cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), (uint32_t)tk.stream,
                     (uint32_t)(tk.stream >> 32)};
    philox10(c, (uint32_t)tk.seed, (uint32_t)(tk.seed >> 32));
    const double u1 = ((double)c[0] + 1.0) * 0x1p-32;  // (0, 1]
    const double u2 = (double)c[1] * 0x1p-32;
    const double r = sqrt(-2.0 * log(u1));
    const int64_t row = e % tk.rows, col = e / tk.rows;
    tk.out[col * tk.ld + row] = r * cospi(2.0 * u2);
  }
}

int launch_gaussian(const SketchTask *d_tasks, int ntask, hipStream_t st) {
  if (ntask <= 0) return 0;
  hipLaunchKernelGGL(k_gaussian, dim3(64, ntask), dim3(256), 0, st, d_tasks);
  return check_launch("gaussian");
}

// ------------------------------------------------------------ data movement

// dst (rows x cols, ldd) = src (rows x cols, lds) with src columns picked by
// idx (nullable: identity) and optionally the lower triangle only (upper 0).
__global__ void k_copy_cols(const CopyTask *__restrict__ tasks) {
  const CopyTask tk = tasks[blockIdx.y];
  const int64_t total = (int64_t)tk.rows * tk.cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % tk.rows), c = (int)(e / tk.rows);
    const int sc = tk.idx ? tk.idx[c] : c;
    double v = tk.src[(int64_t)sc * tk.lds + r];
    if (tk.mode == COPY_UPPER_TRI && r > c) v = 0.0;
    if (tk.mode == COPY_LOWER_TRI && r < c) v = 0.0;
    if (tk.mode == COPY_ZERO) v = 0.0;
    if (tk.mode == COPY_IDENTITY) v = (r == c) ? 1.0 : 0.0;
    tk.dst[(int64_t)c * tk.ldd + r] = v;
  }
}

int launch_copy_cols(const CopyTask *d_tasks, int ntask, hipStream_t st) {
  if (ntask <= 0) return 0;
  hipLaunchKernelGGL(k_copy_cols, dim3(64, ntask), dim3(256), 0, st, d_tasks);
  return check_launch("copy_cols");
}

}  // namespace mvg
