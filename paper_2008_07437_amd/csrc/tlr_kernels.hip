// Batched small dense linear algebra for the tile-low-rank (TLR) path on
// gfx950: FP64 GEMM on MFMA over lists of variable-size products, Householder
// QR of tall-skinny matrices (one workgroup per matrix, or panels over
// several launches; unpivoted, column-pivoted, or with randomized pivots and
// a Frobenius-tail stop), Gaussian sketch matrices.  One list entry per product / matrix; the TLR
// driver builds the lists on the host.
#include <cmath>

#include "tlr.h"

namespace mvg {

typedef double dbl4t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ batched GEMM
//
// C = alpha op(A) op(B) + beta C, column-major, op(X) = X or X^T.  One
// workgroup per 64 x 64 block of C; four waves of 32 x 32 (2 x 2 tiles of
// v_mfma_f64_16x16x4f64); K slices of 16 staged through LDS with the next
// slice's global loads in flight during the current slice's MFMAs.  Ragged
// edges are zero-filled on load and masked on store.
constexpr int GB = 64, GK = 16;

__device__ __forceinline__ int find_task(const int64_t *__restrict__ start, int n, int64_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_gemm_batched(const GemmTask *__restrict__ tasks,
                                                      const int64_t *__restrict__ start, int ntask) {
  __shared__ double As[GK][GB + 2];
  __shared__ double Bs[GK][GB + 2];
  const int t = find_task(start, ntask, blockIdx.x);
  const GemmTask tk = tasks[t];
  const int mt = (tk.M + GB - 1) / GB;
  const int64_t local = (int64_t)blockIdx.x - start[t];
  const int m0 = (int)(local % mt) * GB, n0 = (int)(local / mt) * GB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1, l16 = lane & 15, lk = lane >> 4;
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int m, k;
      if (!tk.ta) { m = tid & 63; k = (tid >> 6) + 4 * i; }
      else { k = tid & 15; m = (tid >> 4) + 16 * i; }
      const int gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      // stored element (row, col) = (gm, gk), or (gk, gm) when transposed
      const bool zero_tri = tk.tri && (tk.ta ? gm > gk : gk > gm);
      if (gm < tk.M && gk < tk.K && !zero_tri)
        v = tk.ta ? tk.A[(int64_t)gm * tk.lda + gk] : tk.A[(int64_t)gk * tk.lda + gm];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int n, k;
      if (tk.tb) { n = tid & 63; k = (tid >> 6) + 4 * i; }
      else { k = tid & 15; n = (tid >> 4) + 16 * i; }
      const int gn = n0 + n, gk = k0 + k;
      double v = 0.0;
      if (gn < tk.N && gk < tk.K)
        v = tk.tb ? tk.B[(int64_t)gk * tk.ldb + gn] : tk.B[(int64_t)gn * tk.ldb + gk];
      rb[i] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!tk.ta) As[(tid >> 6) + 4 * i][tid & 63] = ra[i];
      else As[tid & 15][(tid >> 4) + 16 * i] = ra[i];
      if (tk.tb) Bs[(tid >> 6) + 4 * i][tid & 63] = rb[i];
      else Bs[tid & 15][(tid >> 4) + 16 * i] = rb[i];
    }
  };
  dbl4t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4t{0.0, 0.0, 0.0, 0.0};
  if (tk.K > 0) load(0);
  for (int k0 = 0; k0 < tk.K; k0 += GK) {
    store();
    __syncthreads();
    if (k0 + GK < tk.K) load(k0 + GK);
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = As[ks + lk][wr * 32 + i * 16 + l16];
        b[i] = Bs[ks + lk][wc * 32 + i * 16 + l16];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[i][j] of a 16 x 16 tile: lane j + 16 (i % 4), element i / 4
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gm = m0 + wr * 32 + i * 16 + 4 * e + lk;
        const int gn = n0 + wc * 32 + j * 16 + l16;
        if (gm < tk.M && gn < tk.N) {
          double *c = tk.C + (int64_t)gn * tk.ldc + gm;
          const double v = tk.alpha * acc[i][j][e];
          *c = (tk.beta == 0.0) ? v : v + tk.beta * *c;
        }
      }
}

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
  const int m0 = (blockIdx.x % mblocks) * BG, n0 = (blockIdx.x / mblocks) * BG;
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

int launch_gemm_nt_sub(const double *A, int lda, const double *B, int ldb, double *C, int ldc,
                       int M, int N, int K, hipStream_t st) {
  if (M <= 0 || N <= 0) return 0;
  const int64_t mb = (M + BG - 1) / BG, nbk = (N + BG - 1) / BG;
  if (mb * nbk >= ((int64_t)1 << 31)) {
    set_error("GEMM: %lld blocks", (long long)(mb * nbk));
    return MVG_ERR_LIMIT;
  }
  hipLaunchKernelGGL(k_gemm_nt_sub, dim3((unsigned)(mb * nbk)), dim3(256), 0, st, A, lda, B, ldb,
                     C, ldc, M, N, K, (int)mb);
  return check_launch("gemm_nt_sub");
}

int launch_gemm_batched(const GemmTask *d_tasks, const int64_t *d_start, int ntask, int64_t nblocks,
                        hipStream_t st) {
  if (ntask <= 0 || nblocks <= 0) return 0;
  if (nblocks >= ((int64_t)1 << 31)) {
    set_error("batched GEMM: %lld blocks", (long long)nblocks);
    return MVG_ERR_LIMIT;
  }
  hipLaunchKernelGGL(k_gemm_batched, dim3((unsigned)nblocks), dim3(256), 0, st, d_tasks, d_start,
                     ntask);
  return check_launch("gemm_batched");
}

int64_t gemm_blocks(const GemmTask &t) {
  if (t.M <= 0 || t.N <= 0) return 0;
  return (int64_t)((t.M + GB - 1) / GB) * ((t.N + GB - 1) / GB);
}

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
// Requirements (checked by the launcher): m % 4 == 0, n + PQB <= m <= PQ_MAXM.
constexpr int PQB = 16;          // panel width
constexpr int PQ_MAXM = 1536;    // rows: 6 (3) per panel thread of 256 (512)
constexpr int PAP_CB = 32;       // columns per apply workgroup
constexpr int PAP_THREADS = 256; // apply workgroup (4 waves)

// T factors in tk.tau: panel p0 at rows p0 .. p0 + PQB - 1 of a PQB-wide
// row-major array ((n + PQB) x PQB doubles).
template <int RPT, int NT>
__global__ __launch_bounds__(NT) void k_qr_panel(const QrTask *__restrict__ tasks, int p0) {
  __shared__ double red_s[NT / 64];
  __shared__ double red_d[NT / 64][PQB];
  __shared__ double s_alpha;
  __shared__ double sT[PQB][PQB];
  const QrTask tk = tasks[blockIdx.x];
  const int m = tk.m, n = tk.n, lda = tk.lda;
  if (p0 >= n) return;  // uniform: this task has no panel here
  if (tk.rank && *tk.rank <= p0) return;  // pivoted form: truncated before this panel
  const int pb = min(PQB, n - p0);
  double *A = tk.A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // rows p0 + tid + 512 e of the panel columns: loaded together from clamped
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
  for (int jj = 0; jj < pb; ++jj) {
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
    for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
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
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int c = 0; c < PQB; ++c) d[c] += __shfl_xor(d[c], o);
    if (lane == 0)
#pragma unroll
      for (int c = 0; c < PQB; ++c) red_d[wave][c] = d[c];
    __syncthreads();
    {
      // lane c < PQB sums the waves' partials of column c in a fixed order,
      // then every lane takes the sums from those lanes (reading all of
      // red_d per lane would hold 128 values in registers)
      double part = 0.0;
      if (lane < PQB)
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) part += red_d[w][lane];
#pragma unroll
      for (int c = 0; c < PQB; ++c) d[c] = __shfl(part, c);
    }
    // rows >= j of the columns right of jj: a -= tau (v^T a) v
#pragma unroll
    for (int e = 0; e < RPT; ++e)
#pragma unroll
      for (int c = 0; c < PQB; ++c)
        if (c > jj) a[e][c] -= tau * d[c] * v[e];
    // column jj of T (thread c owns row c of T): T_jj = tau,
    // T[c][jj] = -tau sum_{c <= l < jj} T[c][l] (V[:, l]^T v_jj)
    if (tid < jj) {
      double t = 0.0;
      for (int l = tid; l < jj; ++l) {
        double dl = 0.0;
#pragma unroll
        for (int c = 0; c < PQB; ++c)
          if (c == l) dl = d[c];
        t += sT[tid][l] * dl;
      }
      sT[tid][jj] = -tau * t;
    } else if (tid == jj) {
      sT[jj][jj] = tau;
    }
  }
  // the panel back (R on and above the diagonal, reflectors below), and T
#pragma unroll
  for (int e = 0; e < RPT; ++e) {
    const int r = p0 + tid + NT * e;
    if (r < m)
#pragma unroll
      for (int c = 0; c < PQB; ++c)
        if (c < pb) A[(int64_t)(p0 + c) * lda + r] = a[e][c];
  }
  if (tid < PQB) {
    double *Tg = tk.tau + (int64_t)(p0 + tid) * PQB;
    for (int b = 0; b < PQB; ++b) Tg[b] = (tid < pb && b < pb && b >= tid) ? sT[tid][b] : 0.0;
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
template <int MODE>
__global__ __launch_bounds__(PAP_THREADS) void k_qr_apply(const QrTask *__restrict__ tasks, int p0,
                                                          int nblk) {
  __shared__ double sW[PAP_THREADS / 64][PQB][PAP_CB + 1];
  __shared__ double sN[PQB][PAP_CB + 1];  // -op(T) W
  __shared__ double sT[PQB][PQB + 1];
  __shared__ double sC[PAP_THREADS / 64][PAP_CB];
  const QrTask tk = tasks[blockIdx.x / nblk];
  const int b = blockIdx.x % nblk;
  const int m = tk.m, n = tk.n, lda = tk.lda;
  if (p0 >= n) return;
  if (MODE == 1 && !tk.Q) return;
  if (tk.rank && *tk.rank <= p0) return;  // pivoted form: truncated before this panel
  const int pb = min(PQB, n - p0);
  const int c0 = (MODE == 0 ? p0 + pb : p0) + PAP_CB * b;
  if (c0 >= n) return;  // uniform per workgroup
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
  constexpr int NW = PAP_THREADS / 64;
  for (int ch = wave; ch < nchunk; ch += 2 * NW) {
    double vv[2][4], x0[2][4], x1[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int rl = min(16 * (ch + u * NW) + 4 * lk, M - 4);  // in bounds (M % 4 == 0)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        vv[u][s] = V[(int64_t)qv * lda + rl + s];
        x0[u][s] = X[(int64_t)xc0 * ldx + p0 + rl + s];
        x1[u][s] = X[(int64_t)xc1 * ldx + p0 + rl + s];
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
  for (int o = tid; o < PQB * PAP_CB; o += PAP_THREADS) {
    const int q = o / PAP_CB, c = o % PAP_CB;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < PAP_THREADS / 64; ++w) t += sW[w][q][c];
    sW[0][q][c] = t;
  }
  __syncthreads();
  for (int o = tid; o < PQB * PAP_CB; o += PAP_THREADS) {
    const int q = o / PAP_CB, c = o % PAP_CB;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < PQB; ++k) t += (MODE == 0 ? sT[k][q] : sT[q][k]) * sW[0][k][c];
    sN[q][c] = -t;
  }
  __syncthreads();
  // ---- X -= V W'  (accumulators start from the X tiles); with tk.work
  // (pivoted form, MODE 0) also the squared norms of the updated columns
  // below the panel's rows (rows p0 + pb ..), for the truncation test
  double css[2] = {0.0, 0.0};
  double nq[4][2];  // -W' operands of this lane: rows 4 s + lk, columns 16 h + l16
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int h = 0; h < 2; ++h) nq[s][h] = sN[4 * s + lk][16 * h + l16];
  for (int ch = wave; ch < nchunk; ch += 2 * NW) {
    double va[2][4];
    dbl4t xt[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r0 = 16 * (ch + u * NW);
      const int rv = min(r0 + l16, M - 1);      // V row of this lane (A operand)
#pragma unroll
      for (int s = 0; s < 4; ++s) va[u][s] = V[(int64_t)min(4 * s + lk, pb - 1) * lda + rv];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rx = min(r0 + 4 * e + lk, M - 1);
        xt[u][0][e] = X[(int64_t)xc0 * ldx + p0 + rx];
        xt[u][1][e] = X[(int64_t)xc1 * ldx + p0 + rx];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int r0 = 16 * (ch + u * NW);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int q = 4 * s + lk, r = r0 + l16;
        double vq = va[u][s];
        if (r < q) vq = 0.0;
        else if (r == q) vq = 1.0;
        if (r >= M || q >= pb) vq = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
          xt[u][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(vq, nq[s][h], xt[u][h], 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rx = r0 + 4 * e + lk;
        if (rx < M) {
          if (xok0) X[(int64_t)xc0 * ldx + p0 + rx] = xt[u][0][e];
          if (xok1) X[(int64_t)xc1 * ldx + p0 + rx] = xt[u][1][e];
          if (rx >= pb) {
            css[0] += xt[u][0][e] * xt[u][0][e];
            css[1] += xt[u][1][e] * xt[u][1][e];
          }
        }
      }
    }
  }
  if (MODE == 0 && tk.work) {
    // the four lanes of a column (l16 + 16 lk) in a fixed order, then the
    // waves in a fixed order
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      css[h] += __shfl_xor(css[h], 16);
      css[h] += __shfl_xor(css[h], 32);
    }
    if (lk == 0) {
      sC[wave][l16] = css[0];
      sC[wave][16 + l16] = css[1];
    }
    __syncthreads();
    if (tid < PAP_CB && c0 + tid < n) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < PAP_THREADS / 64; ++w) t += sC[w][tid];
      tk.work[(int64_t)QRS_ROWS * (m + n) + c0 + tid] = t;
    }
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
__global__ __launch_bounds__(PAP_THREADS) void k_qr_sample(const QrTask *__restrict__ tasks, int q0,
                                                           int nblk) {
  __shared__ double sW[PAP_THREADS / 64][QRS_ROWS][PAP_CB + 1];
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
  for (int ch = wave; ch < nchunk; ch += PAP_THREADS / 64) {
    const int rr = 16 * ch + 4 * lk;
    const int rl = min(rr, M - 4);
    double o0[4], o1[4], x0[4], x1[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      o0[s] = Om[(int64_t)l16 * m + rl + s];
      o1[s] = Om[(int64_t)(16 + l16) * m + rl + s];
      x0[s] = tk.A[(int64_t)xc0 * lda + q0 + rl + s];
      x1[s] = tk.A[(int64_t)xc1 * lda + q0 + rl + s];
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
  for (int o = tid; o < QRS_ROWS * PAP_CB; o += PAP_THREADS) {
    const int q = o % QRS_ROWS, c = o / QRS_ROWS;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < PAP_THREADS / 64; ++w) t += sW[w][q][c];
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
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
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
  // the swaps on A and on the column order, in sequence
  for (int t = 0; t < steps; ++t) {
    const int pcol = sswap[t];
    if (pcol != t) {
      double *ca = tk.A + (int64_t)(p0 + t) * lda, *cb = tk.A + (int64_t)(p0 + pcol) * lda;
      for (int r = tid; r < m; r += PICK_THREADS) {
        const double a = ca[r];
        ca[r] = cb[r];
        cb[r] = a;
      }
      if (tid == 0) {
        const int a = tk.piv[p0 + t];
        tk.piv[p0 + t] = tk.piv[p0 + pcol];
        tk.piv[p0 + pcol] = a;
      }
    }
    __syncthreads();
  }
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
// (MVG_QR_PANEL_THREADS=512, experiments).
static int panel_threads() {
  static const int t = [] {
    const char *e = getenv("MVG_QR_PANEL_THREADS");
    return e && atoi(e) == 512 ? 512 : 256;
  }();
  return t;
}

static void launch_panel(const QrTask *d_tasks, int ntask, int mmax, int p0, hipStream_t st) {
  const dim3 g(ntask);
  if (panel_threads() == 512) {
    const int rpt = (mmax + 511) / 512;
    if (rpt == 1)
      hipLaunchKernelGGL((k_qr_panel<1, 512>), g, dim3(512), 0, st, d_tasks, p0);
    else if (rpt == 2)
      hipLaunchKernelGGL((k_qr_panel<2, 512>), g, dim3(512), 0, st, d_tasks, p0);
    else
      hipLaunchKernelGGL((k_qr_panel<3, 512>), g, dim3(512), 0, st, d_tasks, p0);
    return;
  }
  const int rpt = (mmax + 255) / 256;
  switch (rpt) {
    case 1: hipLaunchKernelGGL((k_qr_panel<1, 256>), g, dim3(256), 0, st, d_tasks, p0); break;
    case 2: hipLaunchKernelGGL((k_qr_panel<2, 256>), g, dim3(256), 0, st, d_tasks, p0); break;
    case 3: hipLaunchKernelGGL((k_qr_panel<3, 256>), g, dim3(256), 0, st, d_tasks, p0); break;
    case 4: hipLaunchKernelGGL((k_qr_panel<4, 256>), g, dim3(256), 0, st, d_tasks, p0); break;
    case 5: hipLaunchKernelGGL((k_qr_panel<5, 256>), g, dim3(256), 0, st, d_tasks, p0); break;
    default: hipLaunchKernelGGL((k_qr_panel<6, 256>), g, dim3(256), 0, st, d_tasks, p0); break;
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
      hipLaunchKernelGGL((k_qr_apply<0>), dim3(ntask * nblk), dim3(PAP_THREADS), 0, st, d_tasks,
                         p0, nblk);
      if (int rc = check_launch("qr_apply")) return rc;
    }
  }
  if (!with_q) return 0;
  const int qb = (nmax + 63) / 64;
  hipLaunchKernelGGL(k_qr_qinit, dim3(ntask * qb), dim3(256), 0, st, d_tasks, qb);
  if (int rc = check_launch("qr_qinit")) return rc;
  for (int p0 = ((nmax - 1) / PQB) * PQB; p0 >= 0; p0 -= PQB) {
    const int nblk = (nmax - p0 + PAP_CB - 1) / PAP_CB;
    hipLaunchKernelGGL((k_qr_apply<1>), dim3(ntask * nblk), dim3(PAP_THREADS), 0, st, d_tasks, p0,
                       nblk);
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
    hipLaunchKernelGGL(k_qr_sample, dim3(ntask * sblk), dim3(PAP_THREADS), 0, st, d_tasks, p0, sblk);
    if (int rc = check_launch("qr_sample")) return rc;
    hipLaunchKernelGGL(k_qr_pick, dim3(ntask), dim3(PICK_THREADS), 0, st, d_tasks, p0);
    if (int rc = check_launch("qr_pick")) return rc;
    launch_panel(d_tasks, ntask, mmax, p0, st);
    if (int rc = check_launch("qr_panel")) return rc;
    const int rest = nmax - p0 - PQB;
    if (rest > 0) {
      const int nblk = (rest + PAP_CB - 1) / PAP_CB;
      hipLaunchKernelGGL((k_qr_apply<0>), dim3(ntask * nblk), dim3(PAP_THREADS), 0, st, d_tasks,
                         p0, nblk);
      if (int rc = check_launch("qr_apply")) return rc;
    }
    hipLaunchKernelGGL(k_qr_tail, dim3(ntask), dim3(256), 0, st, d_tasks, p0);
    if (int rc = check_launch("qr_tail")) return rc;
  }
  const int qb = (nmax + 63) / 64;
  hipLaunchKernelGGL(k_qr_qinit, dim3(ntask * qb), dim3(256), 0, st, d_tasks, qb);
  if (int rc = check_launch("qr_qinit")) return rc;
  for (int p0 = ((nmax - 1) / PQB) * PQB; p0 >= 0; p0 -= PQB) {
    const int nblk = (nmax - p0 + PAP_CB - 1) / PAP_CB;
    hipLaunchKernelGGL((k_qr_apply<1>), dim3(ntask * nblk), dim3(PAP_THREADS), 0, st, d_tasks, p0,
                       nblk);
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
