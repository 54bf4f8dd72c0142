// Covariance generation for the bivariate parsimonious Matern model (Eq. 2)
// and the cokriging predictor (Eq. 3-5) on gfx950.
//
// K_nu is evaluated by the trapezoidal rule on the integral representation
// K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt (DLMF 10.32.9), written as
// e^-x * int exp(-x (cosh t - 1)) cosh(nu t) dt so that large x does not
// underflow.  The integrand is analytic in a strip around the real axis, so
// the rule converges geometrically in 1/h; the step is refined with x (levels
// in mvgeo_internal.h) because the integrand narrows like 1/sqrt(x).  One
// exponential per node serves the three orders nu11, nu22, nu12, and the
// node-dependent factors cosh(nu t_k), cosh(t_k) - 1 come from a per-theta
// table held in LDS.  Half-integer orders 1/2, 3/2, 5/2 use their closed forms.
#include <algorithm>
#include <cmath>

#include "matern_dev.h"

namespace mvg {

int matern_setup(const mvg_theta *th, MaternArgs *P) {
  if (!th) return -1;
  const double v[6] = {th->sigma11_sq, th->sigma22_sq, th->a, th->nu11, th->nu22, th->beta};
  for (int i = 0; i < 5; ++i)
    if (!(v[i] > 0.0) || !std::isfinite(v[i])) return -(i + 1);
  if (th->nu11 > 5.0) return -4;
  if (th->nu22 > 5.0) return -5;
  if (!(std::fabs(th->beta) < 1.0)) return -6;
  P->a = th->a;
  P->nu[0] = th->nu11;
  P->nu[1] = th->nu22;
  P->nu[2] = 0.5 * (th->nu11 + th->nu22);
  // colocated correlation for d = 2: Gamma(nu + 1) / Gamma(nu) = nu
  const double rho = th->beta * std::sqrt(th->nu11 * th->nu22) / P->nu[2];
  P->coef[0] = th->sigma11_sq;
  P->coef[1] = th->sigma22_sq;
  P->coef[2] = rho * std::sqrt(th->sigma11_sq) * std::sqrt(th->sigma22_sq);
  P->any_quad = 0;
  for (int o = 0; o < 3; ++o) {
    const double nu = P->nu[o];
    P->lnorm[o] = -((nu - 1.0) * std::log(2.0) + std::lgamma(nu));
    P->closed[o] = nu == 0.5 ? 1 : nu == 1.5 ? 2 : nu == 2.5 ? 3 : 0;
    if (!P->closed[o]) P->any_quad = 1;
  }
  return 0;
}

__global__ void k_quad_table(MaternArgs P, double *__restrict__ q) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < QN) quad_entry(k, P, q);
}

int launch_quad_table(const MaternArgs &P, double *d_qtab, hipStream_t st) {
  hipLaunchKernelGGL(k_quad_table, dim3((QN + 255) / 256), dim3(256), 0, st, P, d_qtab);
  return check_launch("quad_table");
}


__device__ __forceinline__ void load_qtab(const double *__restrict__ q, double *sq) {
  for (int i = threadIdx.x; i < 4 * QN; i += blockDim.x) sq[i] = q[i];
  __syncthreads();
}

// One workgroup: a 32 x 32 block of location pairs of one lower tile.
// Thread layout: 32 consecutive pair-rows (coalesced column writes) x 8 groups
// of 4 pair-columns.
__global__ __launch_bounds__(256) void k_cov_tiles(MaternArgs P, const double *__restrict__ qtab,
                                                   const double *__restrict__ xs,
                                                   const double *__restrict__ ys, int64_t n_loc,
                                                   TileMap M, int tile_first, int spt) {
  __shared__ double sq[4 * QN];
  const int nsub = spt * spt;
  const int64_t tile = tile_first + blockIdx.x / nsub;
  const int sub = blockIdx.x % nsub;
  if (M.kind && M.kind[tile] == TK_ZERO) return;  // annihilated DST tile (whole workgroup)
  load_qtab(qtab, sq);
  int J = 0;
  int64_t t = tile;
  while (t >= M.T - J) {
    t -= M.T - J;
    ++J;
  }
  const int I = J + (int)t;
  const int nb = M.nb, hp = nb / 2;
  const int pl = (sub % spt) * 32 + (threadIdx.x & 31);
  if (pl >= hp) return;
  const int pc0 = (sub / spt) * 32 + (threadIdx.x >> 5) * 4;
  const int64_t gl = (int64_t)I * hp + pl;
  const bool lpad = gl >= n_loc;
  const double xl = lpad ? 0.0 : xs[gl], yl = lpad ? 0.0 : ys[gl];
  const int kind = M.kind ? M.kind[tile] : TK_F64;
  char *tb = M.base + M.off[tile];
  for (int q = 0; q < 4; ++q) {
    const int pr = pc0 + q;
    if (pr >= hp) break;
    const int64_t gr = (int64_t)J * hp + pr;
    double c[3];
    if (lpad || gr >= n_loc) {
      const double d = (gl == gr) ? 1.0 : 0.0;
      c[0] = d;
      c[1] = d;
      c[2] = 0.0;
    } else {
      cross_cov_block(xl, yl, xs[gr], ys[gr], P, sq, c);
    }
    const int64_t e0 = (int64_t)(2 * pr) * nb + 2 * pl;  // (row 2pl, col 2pr)
    if (kind == TK_F64) {
      double *T = reinterpret_cast<double *>(tb);
      *reinterpret_cast<double2 *>(T + e0) = make_double2(c[0], c[2]);
      *reinterpret_cast<double2 *>(T + e0 + nb) = make_double2(c[2], c[1]);
    } else {
      float *T = reinterpret_cast<float *>(tb);
      *reinterpret_cast<float2 *>(T + e0) = make_float2((float)c[0], (float)c[2]);
      *reinterpret_cast<float2 *>(T + e0 + nb) = make_float2((float)c[2], (float)c[1]);
    }
  }
}

int launch_cov_tiles(const MaternArgs &P, const double *d_qtab, const double *d_x,
                     const double *d_y, int64_t n_loc, TileMap M, int tile_first, int tile_count,
                     hipStream_t st) {
  if (tile_count <= 0) return 0;
  const int spt = (M.nb / 2 + 31) / 32;
  const int64_t nwg = (int64_t)tile_count * spt * spt;
  // split very large grids into several launches of < 2^31 workgroups
  const int64_t per = ((int64_t)1 << 30) / (spt * spt);
  for (int64_t t0 = 0; t0 < tile_count; t0 += per) {
    const int64_t cnt = tile_count - t0 < per ? tile_count - t0 : per;
    hipLaunchKernelGGL(k_cov_tiles, dim3((unsigned)(cnt * spt * spt)), dim3(256), 0, st, P,
                       d_qtab, d_x, d_y, n_loc, M, (int)(tile_first + t0), spt);
    int rc = check_launch("cov_tiles");
    if (rc) return rc;
  }
  (void)nwg;
  return 0;
}

// ------------------------------------------------------------ p variables

int matern_setup_p(const mvg_theta_p *th, MaternArgsP *P) {
  if (!th) return -1;
  const int p = th->p;
  if (p < 1 || p > PMAX) return -1;
  for (int i = 0; i < p; ++i)
    if (!(th->sigma_sq[i] > 0.0) || !std::isfinite(th->sigma_sq[i])) return -2;
  if (!(th->a > 0.0) || !std::isfinite(th->a)) return -3;
  for (int i = 0; i < p; ++i)
    if (!(th->nu[i] > 0.0) || !(th->nu[i] <= 5.0)) return -4;
  // beta: symmetric, unit diagonal, positive definite (Cholesky)
  double c[PMAX][PMAX];
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      const double b = th->beta[i * PMAX + j];
      if (!std::isfinite(b) || b != th->beta[j * PMAX + i]) return -5;
      if (i == j && b != 1.0) return -5;
      c[i][j] = b;
    }
  for (int j = 0; j < p; ++j) {
    double d = c[j][j];
    for (int k = 0; k < j; ++k) d -= c[j][k] * c[j][k];
    if (!(d > 0.0)) return -5;
    const double l = std::sqrt(d);
    c[j][j] = l;
    for (int i = j + 1; i < p; ++i) {
      double v = c[i][j];
      for (int k = 0; k < j; ++k) v -= c[i][k] * c[j][k];
      c[i][j] = v / l;
    }
  }
  P->p = p;
  P->no = p * (p + 1) / 2;
  P->a = th->a;
  P->any_quad = 0;
  for (int i = 0; i < p; ++i)
    for (int j = i; j < p; ++j) {
      const int o = pord(i, j, p);
      const double nu = 0.5 * (th->nu[i] + th->nu[j]);
      // colocated correlation for d = 2: Gamma(nu + 1) / Gamma(nu) = nu
      const double rho = i == j ? 1.0 : th->beta[i * PMAX + j] * std::sqrt(th->nu[i] * th->nu[j]) / nu;
      P->nu[o] = nu;
      P->coef[o] = rho * std::sqrt(th->sigma_sq[i]) * std::sqrt(th->sigma_sq[j]);
      P->lnorm[o] = -((nu - 1.0) * std::log(2.0) + std::lgamma(nu));
      P->closed[o] = nu == 0.5 ? 1 : nu == 1.5 ? 2 : nu == 2.5 ? 3 : 0;
      if (!P->closed[o]) P->any_quad = 1;
    }
  return 0;
}

__global__ void k_quad_table_p(MaternArgsP P, double *__restrict__ q) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < QN) quad_entry_p(k, P, q);
}

int launch_quad_table_p(const MaternArgsP &P, double *d_qtab, hipStream_t st) {
  hipLaunchKernelGGL(k_quad_table_p, dim3((QN + 255) / 256), dim3(256), 0, st, P, d_qtab);
  return check_launch("quad_table_p");
}

// One workgroup: up to 32 x 32 location pairs (l, r) whose P x P blocks meet
// lower tile (I, J); a thread takes one l and four r, evaluates all orders of
// a pair at once and writes the entries (P l + i, P r + j) that lie in the
// tile.  Every tile entry belongs to exactly one pair, so each is written
// once.  Rows / columns at or beyond N = P n are the identity padding.
template <int P>
__global__ __launch_bounds__(256) void k_cov_tiles_p(MaternArgsP A, const double *__restrict__ qtab,
                                                     const double *__restrict__ xs,
                                                     const double *__restrict__ ys, int64_t n_loc,
                                                     TileMap M, int64_t tile_first, int spt) {
  constexpr int NO = P * (P + 1) / 2;
  __shared__ double sq[(1 + NO) * QN];
  const int nsub = spt * spt;
  const int64_t tile = tile_first + blockIdx.x / nsub;
  const int sub = blockIdx.x % nsub;
  const int kind = M.kind ? M.kind[tile] : TK_F64;
  if (kind == TK_ZERO) return;  // annihilated DST tile (whole workgroup)
  for (int i = threadIdx.x; i < (1 + NO) * QN; i += blockDim.x) sq[i] = qtab[i];
  __syncthreads();
  int J = 0;
  int64_t t = tile;
  while (t >= M.T - J) {
    t -= M.T - J;
    ++J;
  }
  const int I = J + (int)t;
  const int nb = M.nb;
  const int64_t N = (int64_t)P * n_loc;
  const int64_t g0 = (int64_t)I * nb, c0 = (int64_t)J * nb;  // first row / column of the tile
  const int64_t lr0 = g0 / P, lr1 = (g0 + nb - 1) / P;       // row locations meeting the tile
  const int64_t lc0 = c0 / P, lc1 = (c0 + nb - 1) / P;
  const int64_t l = lr0 + (sub % spt) * 32 + (threadIdx.x & 31);
  if (l > lr1) return;
  const bool lreal = l < n_loc;
  const double xl = lreal ? xs[l] : 0.0, yl = lreal ? ys[l] : 0.0;
  char *tb = M.base + M.off[tile];
  const int64_t rbase = lc0 + (sub / spt) * 32 + (threadIdx.x >> 5) * 4;
  for (int q = 0; q < 4; ++q) {
    const int64_t r = rbase + q;
    if (r > lc1) break;
    const bool real = lreal && r < n_loc;
    double Mv[NO];
    bool zero_h = false;
    if (real) {
      const double dx = xl - xs[r], dy = yl - ys[r];
      const double h = sqrt(dx * dx + dy * dy);
      zero_h = h == 0.0;
      if (!zero_h) matern_p<NO>(h / A.a, A, sq, Mv);
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int64_t g = (int64_t)P * l + i;
      if (g < g0 || g >= g0 + nb) continue;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int64_t c = (int64_t)P * r + j;
        if (c < c0 || c >= c0 + nb) continue;
        double v;
        if (g >= N || c >= N) {
          v = g == c ? 1.0 : 0.0;
        } else {
          const int o = i <= j ? pord(i, j, P) : pord(j, i, P);
          v = zero_h ? A.coef[o] : A.coef[o] * Mv[o];
        }
        const int64_t e = (c - c0) * nb + (g - g0);
        if (kind == TK_F64)
          reinterpret_cast<double *>(tb)[e] = v;
        else
          reinterpret_cast<float *>(tb)[e] = (float)v;
      }
    }
  }
}

int launch_cov_tiles_p(const MaternArgsP &P, const double *d_qtab, const double *d_x,
                       const double *d_y, int64_t n_loc, TileMap M, hipStream_t st) {
  const int64_t nt = (int64_t)M.T * (M.T + 1) / 2;
  const int p = P.p;
  const int spt = (int)(((M.nb - 1) / p + 2 + 31) / 32);  // location rows per tile <= (nb-1)/p + 2
  const int64_t per = ((int64_t)1 << 30) / (spt * spt);
  for (int64_t t0 = 0; t0 < nt; t0 += per) {
    const int64_t cnt = std::min<int64_t>(per, nt - t0);
    const dim3 grid((unsigned)(cnt * spt * spt));
    switch (p) {
      case 1:
        hipLaunchKernelGGL(k_cov_tiles_p<1>, grid, dim3(256), 0, st, P, d_qtab, d_x, d_y, n_loc, M,
                           t0, spt);
        break;
      case 2:
        hipLaunchKernelGGL(k_cov_tiles_p<2>, grid, dim3(256), 0, st, P, d_qtab, d_x, d_y, n_loc, M,
                           t0, spt);
        break;
      case 3:
        hipLaunchKernelGGL(k_cov_tiles_p<3>, grid, dim3(256), 0, st, P, d_qtab, d_x, d_y, n_loc, M,
                           t0, spt);
        break;
      case 4:
        hipLaunchKernelGGL(k_cov_tiles_p<4>, grid, dim3(256), 0, st, P, d_qtab, d_x, d_y, n_loc, M,
                           t0, spt);
        break;
      default:
        set_error("p = %d variables is not supported", p);
        return MVG_ERR_STATE;
    }
    if (int rc = check_launch("cov_tiles_p")) return rc;
  }
  return 0;
}

// ---------------------------------------------------------------- cokriging

constexpr int CK_CHUNK = 2048;  // locations per workgroup

// part[(t * nchunk + chunk) * 2 + j] = sum over the chunk's locations r and
// i in {0,1} of C_ij(||s0_t - s_r||) w[2r+i].
__global__ __launch_bounds__(256) void k_cokrige_dot(MaternArgs P, const double *__restrict__ qtab,
                                                     const double *__restrict__ xs,
                                                     const double *__restrict__ ys, int64_t n_loc,
                                                     const double *__restrict__ x0,
                                                     const double *__restrict__ y0,
                                                     const double *__restrict__ w,
                                                     double *__restrict__ part, int nchunk) {
  __shared__ double sq[4 * QN];
  __shared__ double red[2][256];
  load_qtab(qtab, sq);
  const int64_t t = blockIdx.x / nchunk;
  const int chunk = blockIdx.x % nchunk;
  const double xt = x0[t], yt = y0[t];
  double a0 = 0.0, a1 = 0.0;
  const int64_t r0 = (int64_t)chunk * CK_CHUNK;
  for (int q = threadIdx.x; q < CK_CHUNK; q += 256) {
    const int64_t r = r0 + q;
    if (r >= n_loc) break;
    double c[3];
    cross_cov_block(xt, yt, xs[r], ys[r], P, sq, c);
    const double w0 = w[2 * r], w1 = w[2 * r + 1];
    a0 += c[0] * w0 + c[2] * w1;  // Zhat_1 += C11 w_1 + C21 w_2
    a1 += c[2] * w0 + c[1] * w1;  // Zhat_2 += C12 w_1 + C22 w_2
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[(t * nchunk + chunk) * 2 + 0] = red[0][0];
    part[(t * nchunk + chunk) * 2 + 1] = red[1][0];
  }
}

int launch_cokrige_dot(const MaternArgs &P, const double *d_qtab, const double *d_x,
                       const double *d_y, int64_t n_loc, const double *d_x0, const double *d_y0,
                       int64_t m, const double *d_w, double *d_part, int nchunk, hipStream_t st) {
  hipLaunchKernelGGL(k_cokrige_dot, dim3((unsigned)(m * nchunk)), dim3(256), 0, st, P, d_qtab,
                     d_x, d_y, n_loc, d_x0, d_y0, d_w, d_part, nchunk);
  return check_launch("cokrige_dot");
}

// c0 columns for the MSE: V[(2t + j) * Np + 2r + i] = C_ij(||s0_t - s_r||),
// padded rows 0.
__global__ __launch_bounds__(256) void k_cokrige_c0(MaternArgs P, const double *__restrict__ qtab,
                                                    const double *__restrict__ xs,
                                                    const double *__restrict__ ys, int64_t n_loc,
                                                    int64_t Np, const double *__restrict__ x0,
                                                    const double *__restrict__ y0,
                                                    double *__restrict__ V) {
  __shared__ double sq[4 * QN];
  load_qtab(qtab, sq);
  const int64_t t = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (2 * r >= Np) return;
  double c[3] = {0.0, 0.0, 0.0};
  if (r < n_loc) cross_cov_block(x0[t], y0[t], xs[r], ys[r], P, sq, c);
  double *v0 = V + (2 * t) * Np, *v1 = V + (2 * t + 1) * Np;
  v0[2 * r] = c[0];
  v0[2 * r + 1] = c[2];
  v1[2 * r] = c[2];
  v1[2 * r + 1] = c[1];
}

int launch_cokrige_c0(const MaternArgs &P, const double *d_qtab, const double *d_x,
                      const double *d_y, int64_t n_loc, int64_t Np, const double *d_x0,
                      const double *d_y0, int64_t m, double *d_c0, hipStream_t st) {
  const int64_t npair = Np / 2;
  hipLaunchKernelGGL(k_cokrige_c0, dim3((unsigned)((npair + 255) / 256), (unsigned)m), dim3(256),
                     0, st, P, d_qtab, d_x, d_y, n_loc, Np, d_x0, d_y0, d_c0);
  return check_launch("cokrige_c0");
}

}  // namespace mvg
