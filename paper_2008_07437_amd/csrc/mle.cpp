// Maximum-likelihood driver around Eq. (1) (Section 5.1: the optimiser that
// repeatedly evaluates the likelihood; the paper delegates it to NLopt and
// does not name the method).  Derivative-free Nelder-Mead simplex search
// (Nelder and Mead, Computer Journal 7, 1965) with the usual coefficients:
// reflection 1, expansion 2, contraction 1/2, shrink 1/2.  The objective is
// evaluated in batches: the starting simplex (dim + 1 points) and every shrink
// (dim points) go to the likelihood in one call, which runs them on one
// matrix, or in one persistent launch when the problem is small.
//
// Host code only (no kernels): the likelihood itself is the GPU path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "mvgeo_internal.h"

namespace mvg {

typedef mvg_batch_objective batch_objective;

// Minimise f from x0; returns 0 or the objective's first non-zero code.
static int nelder_mead(int dim, const double *x0, double step, batch_objective f, void *ctx,
                       int max_evals, double ftol, double xtol, double *x_best, double *f_best,
                       int *n_evals, int *n_iters, int *converged) {
  const int m = dim + 1;
  std::vector<double> X((size_t)m * dim), F(m);
  int evals = 0, iters = 0;
  *converged = 0;
  auto eval = [&](int cnt, const double *V, double *out) -> int {
    const int rc = f(cnt, V, out, ctx);
    for (int i = 0; i < cnt; ++i)
      if (!(out[i] == out[i])) out[i] = INFINITY;  // NaN: treat as infeasible
    evals += cnt;
    return rc;
  };
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < dim; ++j) X[(size_t)i * dim + j] = x0[j] + (i == j + 1 ? step : 0.0);
  int rc = eval(m, X.data(), F.data());
  std::vector<int> ord(m);
  std::vector<double> c(dim), xr(dim), xe(dim), xc(dim), tmp((size_t)m * dim), ftmp(m);
  while (!rc) {
    // order by objective (stable: ties keep their index order)
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return F[a] < F[b]; });
    for (int i = 0; i < m; ++i) {
      std::copy(&X[(size_t)ord[i] * dim], &X[(size_t)ord[i] * dim] + dim, &tmp[(size_t)i * dim]);
      ftmp[i] = F[ord[i]];
    }
    X.swap(tmp);
    F.swap(ftmp);
    double spread = 0.0;
    for (int i = 1; i < m; ++i)
      for (int j = 0; j < dim; ++j)
        spread = std::max(spread, std::fabs(X[(size_t)i * dim + j] - X[j]));
    if (std::isfinite(F[m - 1]) && F[m - 1] - F[0] <= ftol && spread <= xtol) {
      *converged = 1;
      break;
    }
    if (evals >= max_evals) break;
    ++iters;
    std::fill(c.begin(), c.end(), 0.0);
    for (int i = 0; i < dim; ++i)
      for (int j = 0; j < dim; ++j) c[j] += X[(size_t)i * dim + j] / dim;
    double *xw = &X[(size_t)dim * dim];
    for (int j = 0; j < dim; ++j) xr[j] = c[j] + (c[j] - xw[j]);
    double fr;
    if ((rc = eval(1, xr.data(), &fr))) break;
    if (fr < F[0]) {  // expansion
      for (int j = 0; j < dim; ++j) xe[j] = c[j] + 2.0 * (xr[j] - c[j]);
      double fe;
      if ((rc = eval(1, xe.data(), &fe))) break;
      if (fe < fr) {
        std::copy(xe.begin(), xe.end(), xw);
        F[dim] = fe;
      } else {
        std::copy(xr.begin(), xr.end(), xw);
        F[dim] = fr;
      }
      continue;
    }
    if (fr < F[dim - 1]) {  // accept the reflection
      std::copy(xr.begin(), xr.end(), xw);
      F[dim] = fr;
      continue;
    }
    const bool outside = fr < F[dim];
    for (int j = 0; j < dim; ++j)
      xc[j] = outside ? c[j] + 0.5 * (xr[j] - c[j]) : c[j] + 0.5 * (xw[j] - c[j]);
    double fc;
    if ((rc = eval(1, xc.data(), &fc))) break;
    if (outside ? fc <= fr : fc < F[dim]) {
      std::copy(xc.begin(), xc.end(), xw);
      F[dim] = fc;
      continue;
    }
    // shrink towards the best point (one batch)
    for (int i = 1; i < m; ++i)
      for (int j = 0; j < dim; ++j)
        X[(size_t)i * dim + j] = X[j] + 0.5 * (X[(size_t)i * dim + j] - X[j]);
    if ((rc = eval(dim, &X[dim], &F[1]))) break;
  }
  const int ib = (int)(std::min_element(F.begin(), F.end()) - F.begin());
  std::copy(&X[(size_t)ib * dim], &X[(size_t)ib * dim] + dim, x_best);
  *f_best = F[ib];
  *n_evals = evals;
  *n_iters = iters;
  return rc;
}

// theta <-> unconstrained coordinates: logs of the variances and the range,
// nu = 5 / (1 + e^-u) in (0, 5), beta = tanh u.
static void to_theta(const double *u, mvg_theta *t) {
  t->sigma11_sq = std::exp(u[0]);
  t->sigma22_sq = std::exp(u[1]);
  t->a = std::exp(u[2]);
  t->nu11 = 5.0 / (1.0 + std::exp(-u[3]));
  t->nu22 = 5.0 / (1.0 + std::exp(-u[4]));
  t->beta = std::tanh(u[5]);
}

static void from_theta(const mvg_theta &t, double *u) {
  u[0] = std::log(t.sigma11_sq);
  u[1] = std::log(t.sigma22_sq);
  u[2] = std::log(t.a);
  u[3] = -std::log(5.0 / t.nu11 - 1.0);
  u[4] = -std::log(5.0 / t.nu22 - 1.0);
  u[5] = std::atanh(t.beta);
}

struct FitCtx {
  const double *x, *y, *z;
  int64_t n;
  const mvg_opts *o;
  void *stream;
};

static int loglik_objective(int m, const double *V, double *f, void *vctx) {
  const FitCtx *c = static_cast<const FitCtx *>(vctx);
  std::vector<mvg_theta> th(m);
  for (int i = 0; i < m; ++i) to_theta(V + (size_t)i * 6, &th[i]);
  std::vector<double> ll(m);
  std::vector<int64_t> st(m);
  int bad = 0;
  for (int i = 0; i < m; ++i) {  // a coordinate can leave the admissible set numerically
    MaternArgs tmp;
    if (matern_setup(&th[i], &tmp)) bad = 1;
  }
  if (bad) {
    for (int i = 0; i < m; ++i) {
      MaternArgs tmp;
      if (matern_setup(&th[i], &tmp)) {
        f[i] = INFINITY;
        continue;
      }
      double l;
      int64_t s;
      if (int rc = loglik(c->x, c->y, c->z, c->n, &th[i], 1, c->o, &l, nullptr, nullptr, &s,
                          nullptr, c->stream))
        return rc;
      f[i] = -l;
    }
    return 0;
  }
  mvg_opts d{};
  if (c->o) d = *c->o;
  if (d.precision == MVG_FP64 && 2 * c->n <= MVG_SMALL_MAX_ROWS) {
    // small problems: every batch size in one persistent launch, so a theta
    // gets the same value whichever step evaluates it
    std::vector<mvg_task> tk(m);
    for (int i = 0; i < m; ++i) tk[i] = mvg_task{c->x, c->y, c->z, c->n, th[i]};
    if (int rc = loglik_many(tk.data(), m, ll.data(), nullptr, nullptr, st.data(), c->stream))
      return rc;
  } else if (int rc = loglik(c->x, c->y, c->z, c->n, th.data(), m, c->o, ll.data(), nullptr,
                             nullptr, st.data(), nullptr, c->stream)) {
    return rc;
  }
  for (int i = 0; i < m; ++i) f[i] = -ll[i];
  return 0;
}

}  // namespace mvg

using namespace mvg;

extern "C" {

int mvg_nelder_mead(int dim, const double *x0, double step, mvg_batch_objective f, void *ctx,
                    int max_evals, double ftol, double xtol, double *x_best, double *f_best,
                    int *n_evals, int *n_iters, int *converged) {
  if (dim < 1 || dim > 64) return -1;
  if (!x0) return -2;
  if (!(step > 0.0)) return -3;
  if (!f) return -4;
  if (max_evals < dim + 1) return -6;
  if (!(ftol >= 0.0) || !(xtol >= 0.0)) return -7;
  if (!x_best || !f_best || !n_evals || !n_iters || !converged) return -9;
  return nelder_mead(dim, x0, step, f, ctx, max_evals, ftol, xtol, x_best, f_best, n_evals,
                     n_iters, converged);
}

int mle_fit(const double *d_x, const double *d_y, const double *d_z, int64_t n_loc,
            const mvg_theta *th0, const mvg_opts *o, const mvg_mle_opts *mo, mvg_theta *th_hat,
            double *h_loglik, int *h_evals, int *h_iters, int *h_converged, void *hip_stream) {
  if (!d_x) return -1;
  if (!d_y) return -2;
  if (!d_z) return -3;
  if (n_loc < 1) return -4;
  MaternArgs tmp;
  if (!th0 || matern_setup(th0, &tmp)) return -5;
  if (th0->nu11 >= 5.0 || th0->nu22 >= 5.0) return -5;  // the transform needs nu < 5
  mvg_mle_opts m{};
  if (mo) m = *mo;
  if (m.max_evals <= 0) m.max_evals = 1000;
  if (m.ftol <= 0.0) m.ftol = 1e-6;
  if (m.xtol <= 0.0) m.xtol = 1e-5;
  if (m.step <= 0.0) m.step = 0.1;
  if (m.max_evals < 7) return -7;
  if (!th_hat || !h_loglik) return -8;
  FitCtx ctx{d_x, d_y, d_z, n_loc, o, hip_stream};
  double u0[6], ub[6], fb = 0.0;
  from_theta(*th0, u0);
  int evals = 0, iters = 0, conv = 0;
  const int rc = nelder_mead(6, u0, m.step, loglik_objective, &ctx, m.max_evals, m.ftol, m.xtol,
                             ub, &fb, &evals, &iters, &conv);
  if (rc) return rc;
  to_theta(ub, th_hat);
  *h_loglik = -fb;
  if (h_evals) *h_evals = evals;
  if (h_iters) *h_iters = iters;
  if (h_converged) *h_converged = conv;
  return 0;
}

}  // extern "C"
