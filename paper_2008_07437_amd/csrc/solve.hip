// Triangular solves and products with a factored tile matrix (Eq. (1):
// L^-1 Z; Eq. (3)-(5) and Algorithm 1 of Section 5.4: L^-1 c0, Sigma^-1 c0,
// L^T w) for one or many right-hand sides, on dense FP64, mixed and TLR
// factors.
#include <algorithm>

#include "mvgeo_internal.h"
#include "tile_dev.h"
#include "tlr.h"

namespace mvg {

constexpr int VB = 64;  // rows per workgroup chunk of the per-column kernels

// ------------------------------------------------------- triangular solves
//
// Vectors are padded to Np = T nb; nrhs right-hand sides are stored column
// after column with leading dimension ldv, blockIdx.z selects the column.
// The diagonal tiles are solved with the inverses W_k kept by the
// factorisation: each step is a dense triangular matrix-vector product.

// y_k = W_k x_k (W_k lower triangular, column-major): 64 output rows per
// workgroup (nb / 64 workgroups per right-hand side), the four waves take a
// quarter of the columns c <= r each and are added in a fixed order.  Reads
// x from X, writes y to Y (out of place: other workgroups still read x).
__global__ __launch_bounds__(256) void k_trsv_tile_fwd(int nb, int k, const double *__restrict__ winv,
                                                       const double *__restrict__ X,
                                                       double *__restrict__ Y, int64_t ldv) {
  __shared__ double v[1024];
  __shared__ double part[4][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = blockIdx.x * 64, r = r0 + lane;
  const double *xk = X + (int64_t)blockIdx.z * ldv + (int64_t)k * nb;
  const double *W = winv + (int64_t)k * nb * nb;
  const int cend = r0 + 64;  // columns c < cend can meet rows r0..r0+63
  for (int c = tid; c < cend; c += 256) v[c] = xk[c];
  __syncthreads();
  const int q = cend / 4;    // a multiple of 16
  double s0 = 0.0, s1 = 0.0;
  for (int c = wave * q; c < wave * q + q; c += 2) {
    if (c <= r) s0 += W[(int64_t)c * nb + r] * v[c];
    if (c + 1 <= r) s1 += W[(int64_t)(c + 1) * nb + r] * v[c + 1];
  }
  part[wave][lane] = s0 + s1;
  __syncthreads();
  if (tid < 64)
    Y[(int64_t)blockIdx.z * ldv + (int64_t)k * nb + r0 + tid] =
        (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
}

// v_i -= L_ik y_k for tiles i in (k, T), y_k read from Y: 64 rows per
// workgroup, the four waves take a quarter of the columns each and are added
// in a fixed order.
__global__ __launch_bounds__(256) void k_gemv_fwd(TileMap M, int k, double *__restrict__ V,
                                                 const double *__restrict__ Y, int64_t ldv) {
  __shared__ double y[1024];
  __shared__ double part[4][64];
  const int nb = M.nb, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *Vc = V + (int64_t)blockIdx.z * ldv;
  const int chunks = nb / 64;
  const int i = k + 1 + blockIdx.x / chunks;
  const int r = (blockIdx.x % chunks) * 64 + lane;
  for (int c = tid; c < nb; c += 256) y[c] = Y[(int64_t)blockIdx.z * ldv + (int64_t)k * nb + c];
  __syncthreads();
  const int q = nb / 4;
  double s0 = 0.0, s1 = 0.0;
  if (tile_is_f32(M, i, k)) {  // mixed precision: off-band tiles in FP32
    const float *L = tile_ptr_f32(M, i, k) + r;
    for (int c = wave * q; c < wave * q + q; c += 2) {
      s0 += (double)L[(int64_t)c * nb] * y[c];
      s1 += (double)L[(int64_t)(c + 1) * nb] * y[c + 1];
    }
  } else {
    const double *L = tile_ptr(M, i, k) + r;
    for (int c = wave * q; c < wave * q + q; c += 2) {
      s0 += L[(int64_t)c * nb] * y[c];
      s1 += L[(int64_t)(c + 1) * nb] * y[c + 1];
    }
  }
  part[wave][lane] = s0 + s1;
  __syncthreads();
  if (tid < 64)
    Vc[(int64_t)i * nb + r] -= (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
}

// y_k = W_k^T x_k: output c = sum_{r >= c} W[r][c] x[r] (column c of W_k is
// contiguous); 64 outputs per workgroup (nb / 64 workgroups per right-hand
// side), one wave per output at a time, lanes over rows.  Out of place.
__global__ __launch_bounds__(256) void k_trsv_tile_bwd(int nb, int k, const double *__restrict__ winv,
                                                       const double *__restrict__ X,
                                                       double *__restrict__ Y, int64_t ldv) {
  __shared__ double v[1024];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = blockIdx.x * 64;
  const double *xk = X + (int64_t)blockIdx.z * ldv + (int64_t)k * nb;
  const double *W = winv + (int64_t)k * nb * nb;
  for (int r = c0 + tid; r < nb; r += 256) v[r] = xk[r];
  __syncthreads();
  for (int c = c0 + wave; c < c0 + 64; c += 4) {
    const double *col = W + (int64_t)c * nb;
    double t = 0.0;
    for (int r = c + lane; r < nb; r += 64) t += col[r] * v[r];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (lane == 0) Y[(int64_t)blockIdx.z * ldv + (int64_t)k * nb + c] = t;
  }
}

// v_j -= L_kj^T w_k for tiles j in [0, k), w_k read from Y: 64 columns per
// workgroup, one wave per column at a time, lanes over rows.
__global__ __launch_bounds__(256) void k_gemv_bwd(TileMap M, int k, double *__restrict__ V,
                                                 const double *__restrict__ Y, int64_t ldv) {
  __shared__ double w[1024];
  const int nb = M.nb, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *Vc = V + (int64_t)blockIdx.z * ldv;
  const int cb = nb / 64;
  const int j = blockIdx.x / cb;
  const int c0 = (blockIdx.x % cb) * 64;
  for (int r = tid; r < nb; r += 256) w[r] = Y[(int64_t)blockIdx.z * ldv + (int64_t)k * nb + r];
  __syncthreads();
  const bool f32 = tile_is_f32(M, k, j);
  for (int c = c0 + wave; c < c0 + 64; c += 4) {
    double s = 0.0;
    if (f32) {
      const float *col = tile_ptr_f32(M, k, j) + (int64_t)c * nb;
      for (int r = lane; r < nb; r += 64) s += (double)col[r] * w[r];
    } else {
      const double *col = tile_ptr(M, k, j) + (int64_t)c * nb;
      for (int r = lane; r < nb; r += 64) s += col[r] * w[r];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) Vc[(int64_t)j * nb + c] -= s;
  }
}

// Scratch of the per-column solves: the solved tiles (Np x nrhs).
static int solve_scratch(const mvg_mat *A, int nrhs, double **Y, hipStream_t st) {
  if (malloc_async((void **)Y, sizeof(double) * A->Np * nrhs, st) != hipSuccess) {
    hipGetLastError();
    set_error("solve workspace of %.3f GB failed", A->Np * nrhs * 8.0 / 1e9);
    return MVG_ERR_ALLOC;
  }
  return 0;
}

// Copy the solution back into V and release the scratch.
static int solve_finish(const mvg_mat *A, double *V, double *Y, int nrhs, int rc, hipStream_t st) {
  if (!rc && hipMemcpyAsync(V, Y, sizeof(double) * A->Np * nrhs, hipMemcpyDeviceToDevice, st) !=
                 hipSuccess)
    rc = MVG_ERR_LAUNCH;
  hipFreeAsync(Y, st);
  return rc;
}

static int solve_args_ok(const mvg_mat *A) {
  if (A->nb > 1024 || A->nb % VB || !A->d_winv) {
    set_error("triangular solve needs nb <= 1024, nb %% 64 == 0 and a factored matrix");
    return MVG_ERR_STATE;
  }
  return 0;
}

// Right-hand sides go in gridDim.z, at most 65535 per launch.
constexpr int MAX_RHS_LAUNCH = 65535;

// Many right-hand sides on an FP64 factor: the tile steps become GEMMs on
// FP64 MFMA (one pass over L for all columns instead of one per column).
//   forward  L X = B:   Y_k = W_k X_k,   X_i -= L_ik Y_k  (i > k)
//   backward L^T X = B: Y_k = W_k^T X_k, X_j -= L_kj^T Y_k (j < k)
//   product  Y = L^T X: Y_J = sum_{I >= J} L_IJ^T X_I, one launch per
//                       tile diagonal d = I - J (distinct outputs per task)
// Y (Np x nrhs) is the solution of the solves, copied back into X.
constexpr int GEMM_RHS_MIN = 4;
enum { TS_FORWARD = 0, TS_BACKWARD = 1, TS_TRMM_T = 2 };

static bool gemm_solve_ok(const mvg_mat *A, int nrhs) {
  return (A->precision == MVG_FP64 || A->precision == MVG_DST) && !A->tlr && A->h_off &&
         nrhs >= GEMM_RHS_MIN;
}

static int tile_gemm_solve(const mvg_mat *A, double *X, double *Y, int nrhs, int mode,
                           hipStream_t st) {
  const int T = A->T, nb = A->nb;
  const int ld = (int)A->Np;
  auto L = [&](int I, int J) {
    return (const double *)(A->arena + A->h_off[tidx(I, J, T)]);
  };
  auto W = [&](int k) { return (const double *)A->d_winv + (int64_t)k * nb * nb; };
  auto zero = [&](int I, int J) { return A->h_kind && A->h_kind[tidx(I, J, T)] == TK_ZERO; };
  auto task = [&](const double *a, int ta, int tri, const double *b, double *c, double alpha,
                  double beta) {
    return GemmTask{a, b, c, nb, nrhs, nb, nb, ld, ld, ta, 0, alpha, beta, tri};
  };
  // every launch: a segment of one task list (starts relative to the segment)
  std::vector<GemmTask> tasks;
  std::vector<int64_t> start;
  std::vector<int> seg;          // first task of each launch
  std::vector<int64_t> blocks;   // blocks of each launch
  auto close = [&](size_t first) {
    int64_t nbk = 0;
    for (size_t i = first; i < tasks.size(); ++i) {
      start.push_back(nbk);
      nbk += gemm_blocks(tasks[i]);
    }
    seg.push_back((int)first);
    blocks.push_back(nbk);
  };
  const int64_t tstride = (int64_t)nb;
  if (mode == TS_FORWARD) {
    for (int k = 0; k < T; ++k) {
      size_t f = tasks.size();
      tasks.push_back(task(W(k), 0, 1, X + k * tstride, Y + k * tstride, 1.0, 0.0));
      close(f);
      if (k + 1 < T) {
        f = tasks.size();
        for (int i = k + 1; i < T; ++i)
          if (!zero(i, k))
            tasks.push_back(task(L(i, k), 0, 0, Y + k * tstride, X + i * tstride, -1.0, 1.0));
        close(f);
      }
    }
  } else if (mode == TS_BACKWARD) {
    for (int k = T - 1; k >= 0; --k) {
      size_t f = tasks.size();
      tasks.push_back(task(W(k), 1, 1, X + k * tstride, Y + k * tstride, 1.0, 0.0));
      close(f);
      if (k > 0) {
        f = tasks.size();
        for (int j = 0; j < k; ++j)
          if (!zero(k, j))
            tasks.push_back(task(L(k, j), 1, 0, Y + k * tstride, X + j * tstride, -1.0, 1.0));
        close(f);
      }
    }
  } else {
    for (int d = 0; d < T; ++d) {
      const size_t f = tasks.size();
      for (int J = 0; J + d < T; ++J)
        if (d == 0 || !zero(J + d, J))
          tasks.push_back(task(L(J + d, J), 1, d == 0, X + (J + d) * tstride, Y + J * tstride,
                               1.0, d == 0 ? 0.0 : 1.0));
      close(f);
    }
  }
  HostLists H;
  int rc = 0;
  const GemmTask *dt =
      (const GemmTask *)H.stage(tasks.data(), tasks.size() * sizeof(GemmTask), st, &rc);
  const int64_t *ds = (const int64_t *)H.stage(start.data(), start.size() * 8, st, &rc);
  for (size_t s = 0; !rc && s < seg.size(); ++s) {
    const int n = (int)((s + 1 < seg.size() ? seg[s + 1] : (int)tasks.size()) - seg[s]);
    rc = launch_gemm_batched(dt + seg[s], ds + seg[s], n, blocks[s], st);
  }
  if (!rc && mode != TS_TRMM_T &&
      hipMemcpyAsync(X, Y, sizeof(double) * A->Np * nrhs, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    rc = MVG_ERR_LAUNCH;
  H.release(st);
  return rc;
}

static int gemm_solve_inplace(const mvg_mat *A, double *d_V, int nrhs, int mode, hipStream_t st) {
  double *Y = nullptr;
  if (malloc_async((void **)&Y, sizeof(double) * A->Np * nrhs, st) != hipSuccess) {
    hipGetLastError();
    set_error("solve workspace of %.2f GB failed", A->Np * nrhs * 8.0 / 1e9);
    return MVG_ERR_ALLOC;
  }
  const int rc = tile_gemm_solve(A, d_V, Y, nrhs, mode, st);
  hipFreeAsync(Y, st);
  return rc;
}

int trsm_forward_multi(const mvg_mat *A, double *d_V, int nrhs, hipStream_t st) {
  if (A->tlr) return tlr_trsm_forward(A, d_V, nrhs, A->Np, st);
  if (int rc = solve_args_ok(A)) return rc;
  if (gemm_solve_ok(A, nrhs)) return gemm_solve_inplace(A, d_V, nrhs, TS_FORWARD, st);
  if (nrhs > MAX_RHS_LAUNCH) {
    for (int c = 0; c < nrhs; c += MAX_RHS_LAUNCH)
      if (int rc = trsm_forward_multi(A, d_V + (int64_t)c * A->Np, std::min(MAX_RHS_LAUNCH, nrhs - c),
                                      st))
        return rc;
    return 0;
  }
  // solved tiles go to Y (the tile solve is out of place), the updates to V;
  // Y is copied back at the end
  double *Y = nullptr;
  if (int rc = solve_scratch(A, nrhs, &Y, st)) return rc;
  const TileMap M = A->map();
  const int chunks = M.nb / 64;
  int rc = 0;
  for (int k = 0; k < M.T && !rc; ++k) {
    hipLaunchKernelGGL(k_trsv_tile_fwd, dim3(chunks, 1, nrhs), dim3(256), 0, st, M.nb, k,
                       (const double *)A->d_winv, (const double *)d_V, Y, A->Np);
    rc = check_launch("trsv_tile_fwd");
    if (!rc && k + 1 < M.T) {
      hipLaunchKernelGGL(k_gemv_fwd, dim3((M.T - k - 1) * chunks, 1, nrhs), dim3(256), 0, st, M, k,
                         d_V, (const double *)Y, A->Np);
      rc = check_launch("gemv_fwd");
    }
  }
  return solve_finish(A, d_V, Y, nrhs, rc, st);
}

int trsv_forward(const mvg_mat *A, double *d_v, hipStream_t st) {
  return trsm_forward_multi(A, d_v, 1, st);
}

int trsm_backward_multi(const mvg_mat *A, double *d_V, int nrhs, hipStream_t st) {
  if (A->tlr) {
    for (int c = 0; c < nrhs; ++c)
      if (int rc = tlr_trsv_backward(A, d_V + (int64_t)c * A->Np, st)) return rc;
    return 0;
  }
  if (int rc = solve_args_ok(A)) return rc;
  if (gemm_solve_ok(A, nrhs)) return gemm_solve_inplace(A, d_V, nrhs, TS_BACKWARD, st);
  if (nrhs > MAX_RHS_LAUNCH) {
    for (int c = 0; c < nrhs; c += MAX_RHS_LAUNCH)
      if (int rc = trsm_backward_multi(A, d_V + (int64_t)c * A->Np,
                                       std::min(MAX_RHS_LAUNCH, nrhs - c), st))
        return rc;
    return 0;
  }
  double *Y = nullptr;
  if (int rc = solve_scratch(A, nrhs, &Y, st)) return rc;
  const TileMap M = A->map();
  const int nb = M.nb;
  int rc = 0;
  for (int k = M.T - 1; k >= 0 && !rc; --k) {
    hipLaunchKernelGGL(k_trsv_tile_bwd, dim3(nb / 64, 1, nrhs), dim3(256), 0, st, nb, k,
                       (const double *)A->d_winv, (const double *)d_V, Y, A->Np);
    rc = check_launch("trsv_tile_bwd");
    if (!rc && k > 0) {
      hipLaunchKernelGGL(k_gemv_bwd, dim3(k * (nb / 64), 1, nrhs), dim3(256), 0, st, M, k, d_V,
                         (const double *)Y, A->Np);
      rc = check_launch("gemv_bwd");
    }
  }
  return solve_finish(A, d_V, Y, nrhs, rc, st);
}

int trsv_backward(const mvg_mat *A, double *d_v, hipStream_t st) {
  return trsm_backward_multi(A, d_v, 1, st);
}

// Y = L^T X for nrhs columns (ld Np), L the factor's lower tiles: output tile
// J, column c: sum_{I >= J} sum_r L_IJ[r][c] X_I[r] (rows r >= c in the
// diagonal tile).  One workgroup per (J, 64 output columns, right-hand side),
// one wave per output column at a time, lanes over rows; fixed order.
__global__ __launch_bounds__(256) void k_trmm_t(TileMap M, const double *__restrict__ X,
                                                double *__restrict__ Y, int64_t ldv) {
  const int nb = M.nb, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cb = nb / 64;
  const int J = blockIdx.x / cb;
  const int c0 = (blockIdx.x % cb) * 64;
  const double *Xc = X + (int64_t)blockIdx.z * ldv;
  double *Yc = Y + (int64_t)blockIdx.z * ldv;
  const bool f32 = M.kind != nullptr;
  for (int c = c0 + wave; c < c0 + 64; c += 4) {
    double s = 0.0;
    for (int I = J; I < M.T; ++I) {
      const double *x = Xc + (int64_t)I * nb;
      const int r0 = (I == J) ? c : 0;
      if (f32 && tile_is_f32(M, I, J)) {
        const float *col = tile_ptr_f32(M, I, J) + (int64_t)c * nb;
        for (int r = r0 + lane; r < nb; r += 64) s += (double)col[r] * x[r];
      } else {
        const double *col = tile_ptr(M, I, J) + (int64_t)c * nb;
        for (int r = r0 + lane; r < nb; r += 64) s += col[r] * x[r];
      }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) Yc[(int64_t)J * nb + c] = s;
  }
}

int launch_trmm_t(const mvg_mat *A, const double *d_X, double *d_Y, int nrhs, hipStream_t st) {
  if (A->tlr) {
    set_error("L^T products are not available for TLR factors");
    return MVG_ERR_STATE;
  }
  if (int rc = solve_args_ok(A)) return rc;
  if (gemm_solve_ok(A, nrhs))
    return tile_gemm_solve(A, const_cast<double *>(d_X), d_Y, nrhs, TS_TRMM_T, st);
  const TileMap M = A->map();
  for (int c = 0; c < nrhs; c += MAX_RHS_LAUNCH) {
    const int64_t off = (int64_t)c * A->Np;
    hipLaunchKernelGGL(k_trmm_t, dim3(M.T * (M.nb / 64), 1, std::min(MAX_RHS_LAUNCH, nrhs - c)),
                       dim3(256), 0, st, M, d_X + off, d_Y + off, A->Np);
    if (int rc = check_launch("trmm_t")) return rc;
  }
  return 0;
}

// out[c] = sum_i A[c Np + i] B[c Np + i] for ncols columns (fixed order)
__global__ __launch_bounds__(256) void k_dot_cols(const double *__restrict__ A,
                                                  const double *__restrict__ B, int64_t Np,
                                                  double *__restrict__ out) {
  __shared__ double r[256];
  const double *a = A + (int64_t)blockIdx.x * Np, *b = B + (int64_t)blockIdx.x * Np;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < Np; i += 256) s += a[i] * b[i];
  r[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) r[threadIdx.x] += r[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = r[0];
}

int launch_dot_cols(const double *d_A, const double *d_B, int64_t Np, int ncols, double *d_out,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_dot_cols, dim3(ncols), dim3(256), 0, st, d_A, d_B, Np, d_out);
  return check_launch("dot_cols");
}

}  // namespace mvg
