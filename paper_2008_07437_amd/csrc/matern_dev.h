// Device-side evaluation of the bivariate Matern covariance (Eq. 2): the
// per-theta quadrature table and the 2 x 2 covariance block of two locations.
// Shared by the generation, cokriging and batched small-problem kernels.
//
// K_nu is evaluated by the trapezoidal rule on the integral representation
// K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt (DLMF 10.32.9), written as
// e^-x * int exp(-x (cosh t - 1)) cosh(nu t) dt; see mvgeo_internal.h for the
// step levels.
#pragma once

#include "mvgeo_internal.h"

namespace mvg {

// Table entry k of the per-theta table q (4 x QN): cosh t_k - 1 and
// cosh(nu_o t_k) for the three orders.
__device__ __forceinline__ void quad_entry(int k, const MaternArgs &P, double *__restrict__ q) {
  int j = -1;
  for (int l = 0; l < QLEV; ++l)
    if (k >= qlev_off(l) && k < qlev_off(l) + qlev_cnt(l)) j = l;
  double cm1 = 0.0, c0 = 0.0, c1 = 0.0, c2 = 0.0;
  if (j >= 0) {
    const double t = (double)(k - qlev_off(j)) * qlev_h(j);
    const double s = sinh(0.5 * t);
    cm1 = 2.0 * s * s;  // cosh t - 1 without cancellation
    c0 = cosh(P.nu[0] * t);
    c1 = cosh(P.nu[1] * t);
    c2 = cosh(P.nu[2] * t);
  }
  q[k] = cm1;
  q[QN + k] = c0;
  q[2 * QN + k] = c1;
  q[3 * QN + k] = c2;
}

// Normalised Matern M(x; nu_o) for the three orders, x > 0.  sq: LDS table.
__device__ __forceinline__ void matern3(double x, const MaternArgs &P,
                                        const double *__restrict__ sq, double M[3]) {
  if (x > qlev_xmax(QLEV - 1)) {
    M[0] = M[1] = M[2] = 0.0;
    return;
  }
  const double ex = exp(-x);
  double s0 = 0.5, s1 = 0.5, s2 = 0.5, logh = 0.0;
  if (P.any_quad) {
    const int j = x <= qlev_xmax(0) ? 0 : x <= qlev_xmax(1) ? 1 : x <= qlev_xmax(2) ? 2
                : x <= qlev_xmax(3) ? 3 : 4;
    const int off = qlev_off(j), cnt = qlev_cnt(j);
    logh = log(qlev_h(j));
    // nodes in pairs, the stopping test on the second of each pair (the
    // test costs six FP64 operations against the node's ~25)
    for (int k = 1; k < cnt; k += 2) {
      const double e = exp(-x * sq[off + k]);
      s0 += e * sq[QN + off + k];
      s1 += e * sq[2 * QN + off + k];
      s2 += e * sq[3 * QN + off + k];
      if (k + 1 >= cnt) break;
      const double e2 = exp(-x * sq[off + k + 1]);
      const double t0 = e2 * sq[QN + off + k + 1];
      const double t1 = e2 * sq[2 * QN + off + k + 1];
      const double t2 = e2 * sq[3 * QN + off + k + 1];
      s0 += t0;
      s1 += t1;
      s2 += t2;
      if (t0 <= 1e-17 * s0 && t1 <= 1e-17 * s1 && t2 <= 1e-17 * s2) break;
    }
  }
  const double lx = log(x);
  const double s[3] = {s0, s1, s2};
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    switch (P.closed[o]) {
      case 1: M[o] = ex; break;
      case 2: M[o] = (1.0 + x) * ex; break;
      case 3: M[o] = (1.0 + x + x * x * (1.0 / 3.0)) * ex; break;
      default: M[o] = exp(P.nu[o] * lx - x + P.lnorm[o] + logh) * s[o]; break;
    }
  }
}

// 2x2 block C(||s_l - s_r||) of Representation I: c[0]=C11, c[1]=C22, c[2]=C12.
__device__ __forceinline__ void cross_cov_block(double xl, double yl, double xr, double yr,
                                                const MaternArgs &P, const double *sq,
                                                double c[3]) {
  const double dx = xl - xr, dy = yl - yr;
  const double h = sqrt(dx * dx + dy * dy);
  if (h == 0.0) {
    c[0] = P.coef[0];
    c[1] = P.coef[1];
    c[2] = P.coef[2];
    return;
  }
  double M[3];
  matern3(h / P.a, P, sq, M);
  c[0] = P.coef[0] * M[0];
  c[1] = P.coef[1] * M[1];
  c[2] = P.coef[2] * M[2];
}

// ------------------------------------------------------------ p variables

// Table entry k of the p-variate table ((1 + no) x QN).
__device__ __forceinline__ void quad_entry_p(int k, const MaternArgsP &P, double *__restrict__ q) {
  int j = -1;
  for (int l = 0; l < QLEV; ++l)
    if (k >= qlev_off(l) && k < qlev_off(l) + qlev_cnt(l)) j = l;
  double t = 0.0, cm1 = 0.0;
  if (j >= 0) {
    t = (double)(k - qlev_off(j)) * qlev_h(j);
    const double s = sinh(0.5 * t);
    cm1 = 2.0 * s * s;
  }
  q[k] = cm1;
  for (int o = 0; o < P.no; ++o) q[(1 + o) * QN + k] = j >= 0 ? cosh(P.nu[o] * t) : 0.0;
}

// Normalised Matern M(x; nu_o) for all NO orders of the p-variate model,
// x > 0 (one exponential per node for every order).
template <int NO>
__device__ __forceinline__ void matern_p(double x, const MaternArgsP &P,
                                         const double *__restrict__ sq, double M[NO]) {
  if (x > qlev_xmax(QLEV - 1)) {
#pragma unroll
    for (int o = 0; o < NO; ++o) M[o] = 0.0;
    return;
  }
  const double ex = exp(-x);
  double s[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) s[o] = 0.5;
  double logh = 0.0;
  if (P.any_quad) {
    const int j = x <= qlev_xmax(0) ? 0 : x <= qlev_xmax(1) ? 1 : x <= qlev_xmax(2) ? 2
                : x <= qlev_xmax(3) ? 3 : 4;
    const int off = qlev_off(j), cnt = qlev_cnt(j);
    logh = log(qlev_h(j));
    // nodes in pairs, the stopping test on the second of each pair
    for (int k = 1; k < cnt; k += 2) {
      const double e = exp(-x * sq[off + k]);
#pragma unroll
      for (int o = 0; o < NO; ++o) s[o] += e * sq[(1 + o) * QN + off + k];
      if (k + 1 >= cnt) break;
      const double e2 = exp(-x * sq[off + k + 1]);
      bool small = true;
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        const double tt = e2 * sq[(1 + o) * QN + off + k + 1];
        s[o] += tt;
        small = small && tt <= 1e-17 * s[o];
      }
      if (small) break;
    }
  }
  const double lx = log(x);
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    switch (P.closed[o]) {
      case 1: M[o] = ex; break;
      case 2: M[o] = (1.0 + x) * ex; break;
      case 3: M[o] = (1.0 + x + x * x * (1.0 / 3.0)) * ex; break;
      default: M[o] = exp(P.nu[o] * lx - x + P.lnorm[o] + logh) * s[o]; break;
    }
  }
}

}  // namespace mvg
