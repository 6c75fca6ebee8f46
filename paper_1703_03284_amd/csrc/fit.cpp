// Maximum-likelihood fit on top of mipwa_eval (Sec. 2: the knot parameters and the resonance
// coefficients are determined by an unbinned ML fit; interpolation correlates them, so a robust
// quasi-Newton minimiser is used; Sec. 4: the normalisation is recomputed in every iteration).
//
// BFGS on the floated parameters: inverse-Hessian estimate B (scaled identity after the first step),
// search direction -B g, line search satisfying the strong Wolfe conditions (bracketing, then zoom
// with safeguarded cubic interpolation; Nocedal & Wright, Numerical Optimization, ch. 3), update
// B <- (I - rho s y^T) B (I - rho y s^T) + rho s s^T when s^T y > 0.  Convergence when
// EDM = g^T B g / 2 < tol.  Then H by central differences of the analytic gradient, cov = 2 H^-1
// (the objective is -2 ln L).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "minimizer.h"
#include "mipwa.h"

namespace mipwa {
namespace {

struct Objective {
  const FullEval* fg;
  std::vector<int> free;
  std::vector<double> full;
  std::vector<double> gfull;
  int n_eval = 0;
  // f = +inf for parameters outside the allowed domain or a non-finite likelihood
  int operator()(const std::vector<double>& x, double& f, std::vector<double>& g) {
    for (size_t i = 0; i < free.size(); ++i) full[free[i]] = x[i];
    ++n_eval;
    int rc = (*fg)(full.data(), f, gfull.data());
    if (rc) return rc;
    g.resize(free.size());
    for (size_t i = 0; i < free.size(); ++i) g[i] = gfull[free[i]];
    return MIPWA_OK;
  }
};

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

// y = B x for the symmetric BFGS matrix, accumulated row by row as y += x_j B[j, :]: every element is
// an independent multiply-add, so the loop vectorises (a row-dot form is a chain of dependent adds)
void matvec(const std::vector<double>& B, const std::vector<double>& x, std::vector<double>& y) {
  const size_t n = x.size();
  y.assign(n, 0.0);
  double* __restrict__ yy = y.data();
  for (size_t j = 0; j < n; ++j) {
    const double xj = x[j];
    const double* __restrict__ Bj = B.data() + j * n;
    for (size_t i = 0; i < n; ++i) yy[i] += xj * Bj[i];
  }
}

// minimiser of the cubic through (a, fa, da) and (b, fb, db), safeguarded to the inner 80% of [a, b]
double cubic_step(double a, double fa, double da, double b, double fb, double db) {
  const double lo = std::min(a, b), hi = std::max(a, b), w = hi - lo;
  double t = 0.5 * (a + b);
  if (std::isfinite(fb) && std::isfinite(db)) {
    const double d1 = da + db - 3.0 * (fa - fb) / (a - b);
    const double disc = d1 * d1 - da * db;
    if (disc >= 0) {
      const double d2 = std::copysign(std::sqrt(disc), b - a);
      const double den = db - da + 2.0 * d2;
      if (den != 0) t = b - (b - a) * (db + d2 - d1) / den;
    }
  }
  return std::min(std::max(t, lo + 0.1 * w), hi - 0.1 * w);
}

struct LineResult {
  bool ok = false;
  double alpha = 0, f = 0;
  std::vector<double> x, g;
};

// Line search along d from (x0, f0, g0) for a step meeting the strong Wolfe conditions (Nocedal &
// Wright, ch. 3: expansion until a bracket is found, then zoom by safeguarded cubic interpolation),
// with the sufficient-decrease test relaxed by eps_f, the noise of f.  The bracket is kept by the
// sign of the directional derivative, as in Hager & Zhang's line search (SIAM J. Optim. 16, 2005):
// lo always has phi' < 0 and f <= f0 + eps_f, hi has phi' >= 0 or f above f0 + eps_f.  Comparisons
// of f values that differ by less than the noise decide nothing, so near the minimum, where the
// decrease per step falls below the rounding noise of a mixed-precision f, the search is steered by
// the gradient, which stays accurate there.
int line_search(Objective& obj, const std::vector<double>& x0, double f0, const std::vector<double>& g0,
                const std::vector<double>& d, double alpha0, double eps_f, LineResult& out) {
  const double c1 = 1e-4, c2 = 0.9;
  const double dphi0 = dot(g0, d);
  const size_t n = x0.size();
  std::vector<double> x(n);
  auto eval = [&](double a, double& f, double& dphi, std::vector<double>& gx) -> int {
    for (size_t i = 0; i < n; ++i) x[i] = x0[i] + a * d[i];
    int rc = obj(x, f, gx);
    if (rc) return rc;
    dphi = std::isfinite(f) ? dot(gx, d) : NAN;
    return MIPWA_OK;
  };
  auto accept = [&](double a, double f, const std::vector<double>& gx) {
    out.ok = true;
    out.alpha = a;
    out.f = f;
    out.x = x;
    out.g = gx;
  };
  auto wolfe = [&](double a, double f, double dp) {
    return f <= f0 + c1 * a * dphi0 + eps_f && std::fabs(dp) <= -c2 * dphi0;
  };
  // lo: phi' < 0 and f <= f0 + eps_f (a = 0 qualifies); hi: the other end of the bracket
  auto zoom = [&](double lo, double flo, double dlo, double hi, double fhi, double dhi) -> int {
    for (int it = 0; it < 30; ++it) {
      const double a = cubic_step(lo, flo, dlo, hi, fhi, dhi);
      double f, dp;
      std::vector<double> gx;
      int rc = eval(a, f, dp, gx);
      if (rc) return rc;
      if (std::isfinite(f) && wolfe(a, f, dp)) {
        accept(a, f, gx);
        return MIPWA_OK;
      }
      if (!std::isfinite(f) || dp >= 0 || f > f0 + eps_f) {
        hi = a;
        fhi = f;
        dhi = dp;
      } else {
        lo = a;
        flo = f;
        dlo = dp;
      }
      if (std::fabs(hi - lo) < 1e-16 * std::max(1.0, std::fabs(lo))) break;
    }
    // no point met both conditions: move to lo if it lies beyond the start (its f is within the
    // noise of f0 or below, and the function still descends there)
    if (lo > 0) {
      double f, dp;
      std::vector<double> gx;
      int rc = eval(lo, f, dp, gx);
      if (rc) return rc;
      if (std::isfinite(f) && f <= f0 + eps_f) accept(lo, f, gx);
    }
    return MIPWA_OK;
  };
  double a_prev = 0.0, f_prev = f0, d_prev = dphi0;
  double a = alpha0;
  for (int it = 0; it < 30; ++it) {
    double f, dp;
    std::vector<double> gx;
    int rc = eval(a, f, dp, gx);
    if (rc) return rc;
    if (std::isfinite(f) && wolfe(a, f, dp)) {
      accept(a, f, gx);
      return MIPWA_OK;
    }
    if (!std::isfinite(f) || dp >= 0 || f > f0 + eps_f) return zoom(a_prev, f_prev, d_prev, a, f, dp);
    a_prev = a;
    f_prev = f;
    d_prev = dp;
    a *= 2.0;
  }
  return MIPWA_OK;
}

bool cholesky_inverse(std::vector<double> A, size_t n, std::vector<double>& inv) {
  // A = L L^T in place (lower), then inv = L^-T L^-1
  for (size_t j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (size_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    A[j * n + j] = d;
    for (size_t i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (size_t k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
  }
  std::vector<double> Linv(n * n, 0.0);
  for (size_t i = 0; i < n; ++i) {
    Linv[i * n + i] = 1.0 / A[i * n + i];
    for (size_t j = 0; j < i; ++j) {
      double s = 0.0;
      for (size_t k = j; k < i; ++k) s -= A[i * n + k] * Linv[k * n + j];
      Linv[i * n + j] = s / A[i * n + i];
    }
  }
  inv.assign(n * n, 0.0);
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j <= i; ++j) {
      double s = 0.0;
      for (size_t k = i; k < n; ++k) s += Linv[k * n + i] * Linv[k * n + j];
      inv[i * n + j] = inv[j * n + i] = s;
    }
  return true;
}

}  // namespace

int bfgs_fit(const FullEval& fg, int P, const std::vector<int>& polar_pairs, const std::vector<unsigned char>& fixed,
             const double* theta0,
             double tol, int max_iter, bool want_hess, double eps_rel, FitOut& out) {
  Objective obj{&fg, {}, std::vector<double>(theta0, theta0 + P), std::vector<double>(P), 0};
  for (int p = 0; p < P; ++p)
    if (!fixed[p]) obj.free.push_back(p);
  const size_t n = obj.free.size();
  if (n == 0) {
    out.err = "every parameter is fixed";
    return MIPWA_E_INVAL;
  }
  std::vector<double> x(n), g;
  for (size_t i = 0; i < n; ++i) x[i] = theta0[obj.free[i]];
  double f = 0.0;
  int rc = obj(x, f, g);
  if (rc) return rc;
  if (!std::isfinite(f)) {
    out.err = "-2 ln L is not finite at the start point";
    return MIPWA_E_DOMAIN;
  }
  std::vector<double> B(n * n, 0.0);
  const double gmax = std::max(1e-300, std::fabs(*std::max_element(g.begin(), g.end(), [](double a, double b) {
    return std::fabs(a) < std::fabs(b);
  })));
  const double b0 = 0.1 / gmax;  // first step moves the steepest parameter by about 0.1
  for (size_t i = 0; i < n; ++i) B[i * n + i] = b0;
  // Bg = B g for the current B.  It is kept up to date through each update, so an iteration takes one
  // matrix-vector product (B g' with the B the step was taken with; B y = B g' - B g).
  std::vector<double> d(n), Bg, Bgn, s(n), y(n), By(n), w(n), t(n);
  matvec(B, g, Bg);
  auto restart = [&](double b) {  // B = b I
    std::fill(B.begin(), B.end(), 0.0);
    for (size_t i = 0; i < n; ++i) B[i * n + i] = b, Bg[i] = b * g[i];
  };
  int iter = 0, status = MIPWA_E_NOCONV;
  double edm = 0.0;
  bool scaled = false;
  for (; iter < max_iter; ++iter) {
    edm = 0.5 * dot(g, Bg);
    if (edm < tol) {
      status = MIPWA_OK;
      break;
    }
    for (size_t i = 0; i < n; ++i) d[i] = -Bg[i];
    if (dot(g, d) >= 0) {  // lost positive definiteness: restart from a scaled identity
      restart(b0);
      for (size_t i = 0; i < n; ++i) d[i] = -Bg[i];
    }
    LineResult lr;
    rc = line_search(obj, x, f, g, d, 1.0, eps_rel * std::fabs(f), lr);
    if (rc) return rc;
    if (!lr.ok) {
      // retry once along steepest descent before giving up
      restart(b0);
      for (size_t i = 0; i < n; ++i) d[i] = -Bg[i];
      rc = line_search(obj, x, f, g, d, 1.0, eps_rel * std::fabs(f), lr);
      if (rc) return rc;
      if (!lr.ok) break;
    }
    for (size_t i = 0; i < n; ++i) {
      s[i] = lr.x[i] - x[i];
      y[i] = lr.g[i] - g[i];
    }
    const double sy = dot(s, y);
    if (!scaled && sy > 0) {
      restart(sy / dot(y, y));
      scaled = true;
    }
    matvec(B, lr.g, Bgn);
    if (sy > 1e-12 * std::sqrt(dot(s, s) * dot(y, y))) {
      const double rho = 1.0 / sy;
      for (size_t i = 0; i < n; ++i) By[i] = Bgn[i] - Bg[i];
      const double yBy = dot(y, By);
      // B + (rho^2 y^T B y + rho) s s^T - rho (B y s^T + s y^T B), as B_ij += w_i s_j - s_i t_j with
      // w = (rho^2 y^T B y + rho) s - rho B y and t = rho B y (two multiply-adds per element).  The
      // change is symmetric: it is formed on and above the diagonal and mirrored, so B stays exactly
      // symmetric and B^T x (what matvec forms) is B x.
      const double a = rho * rho * yBy + rho;
      for (size_t i = 0; i < n; ++i) {
        w[i] = a * s[i] - rho * By[i];
        t[i] = rho * By[i];
      }
      for (size_t i = 0; i < n; ++i) {
        const double wi = w[i], si = s[i];
        double* Bi = B.data() + i * n;
        for (size_t j = i; j < n; ++j) Bi[j] += wi * s[j] - si * t[j];
      }
      for (size_t i = 1; i < n; ++i)
        for (size_t j = 0; j < i; ++j) B[i * n + j] = B[j * n + i];
      // the updated B times g' = B g' + w (s . g') - s (t . g')
      const double sg = dot(s, lr.g), tg = dot(t, lr.g);
      for (size_t i = 0; i < n; ++i) Bgn[i] += w[i] * sg - s[i] * tg;
    }
    Bg.swap(Bgn);
    x = lr.x;
    f = lr.f;
    g = lr.g;
  }
  if (iter >= max_iter) {
    matvec(B, g, Bg);
    edm = 0.5 * dot(g, Bg);
    if (edm < tol) status = MIPWA_OK;
  }
  // covariance
  std::vector<double> V(n * n);
  for (size_t i = 0; i < n * n; ++i) V[i] = 2.0 * B[i];
  if (want_hess) {
    std::vector<double> H(n * n), xp, gp, gm;
    double fp, fm;
    for (size_t i = 0; i < n; ++i) {
      const double h = 1e-4 * std::max(1.0, std::fabs(x[i]));
      xp = x;
      xp[i] += h;
      rc = obj(xp, fp, gp);
      if (rc) return rc;
      xp[i] = x[i] - h;
      rc = obj(xp, fm, gm);
      if (rc) return rc;
      for (size_t j = 0; j < n; ++j) H[j * n + i] = (gp[j] - gm[j]) / (2.0 * h);
    }
    for (size_t i = 0; i < n; ++i)
      for (size_t j = 0; j < i; ++j) H[i * n + j] = H[j * n + i] = 0.5 * (H[i * n + j] + H[j * n + i]);
    std::vector<double> Hinv;
    if (cholesky_inverse(H, n, Hinv)) {
      for (size_t i = 0; i < n * n; ++i) V[i] = 2.0 * Hinv[i];
      matvec(Hinv, g, Bg);
      edm = 0.5 * dot(g, Bg);
    }
  }
  out.theta.assign(theta0, theta0 + P);
  for (size_t i = 0; i < n; ++i) out.theta[obj.free[i]] = x[i];
  out.cov.assign((size_t)P * P, 0.0);
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < n; ++j) out.cov[(size_t)obj.free[i] * P + obj.free[j]] = V[i * n + j];
  // fold (magnitude, phase) pairs: magnitude >= 0, phase in (-pi, pi]; a sign flip of a magnitude flips
  // its covariance row and column
  for (const int i : polar_pairs) {
    double a = out.theta[i], p = out.theta[i + 1];
    if (a < 0) {
      a = -a;
      p += M_PI;
      for (int q = 0; q < P; ++q) {
        out.cov[(size_t)i * P + q] = -out.cov[(size_t)i * P + q];
        out.cov[(size_t)q * P + i] = -out.cov[(size_t)q * P + i];
      }
    }
    p = M_PI - std::fmod(std::fmod(M_PI - p, 2.0 * M_PI) + 2.0 * M_PI, 2.0 * M_PI);
    out.theta[i] = a;
    out.theta[i + 1] = p;
  }
  out.nll = f;
  out.edm = edm;
  out.n_iter = iter;
  out.n_eval = obj.n_eval;
  out.status = status;
  return MIPWA_OK;
}

}  // namespace mipwa

extern "C" int mipwa_fit(mipwa_ctx* ctx, const mipwa_fit_opts* opts, double* theta_inout, double* cov_out,
                         mipwa_fit_info* info) {
  using namespace mipwa;
  if (!ctx) return MIPWA_E_INVAL;
  if (!theta_inout) return ctx->fail(MIPWA_E_INVAL, "theta is NULL");
  const int P = ctx->ext_P();
  const double tol = opts && opts->tol_edm > 0 ? opts->tol_edm : 1e-6;
  const int max_iter = opts && opts->max_iter > 0 ? opts->max_iter : 1000;
  const bool want_hess = opts ? opts->hessian != 0 : true;
  FullEval fg = [ctx, P](const double* th, double& f, double* g) -> int {
    int rc = mipwa_set_params(ctx, th, P);
    if (rc == MIPWA_E_INVAL) {
      f = INFINITY;
      return MIPWA_OK;
    }
    if (rc) return rc;
    rc = mipwa_eval(ctx, &f, g);
    if (rc == MIPWA_E_DOMAIN) {
      f = INFINITY;
      return MIPWA_OK;
    }
    return rc;
  };
  const double eps_rel = ctx->fp64 ? kNoiseRelFp64 : kNoiseRelMixed;
  FitOut out;
  // (magnitude, phase) pairs of the external layout: the polar knots, c_NR of the isobar form, the c_r
  std::vector<int> pairs;
  if (ctx->swave == kSwavePolar)
    for (int k = 0; k < ctx->mh.N; ++k) pairs.push_back(2 * k);
  if (ctx->swave == kSwaveIsobar) pairs.push_back(0);
  for (int r = 0; r < ctx->mh.R; ++r) pairs.push_back(ctx->ext_res_off() + 2 * r);
  int rc = bfgs_fit(fg, P, pairs, ctx->fixed, theta_inout, tol, max_iter, want_hess, eps_rel, out);
  if (rc) return ctx->fail(rc, out.err.empty() ? std::string(ctx->err) : out.err);
  std::copy(out.theta.begin(), out.theta.end(), theta_inout);
  (void)mipwa_set_params(ctx, theta_inout, P);
  if (cov_out) std::copy(out.cov.begin(), out.cov.end(), cov_out);
  if (info) {
    info->nll = out.nll;
    info->edm = out.edm;
    info->n_iter = out.n_iter;
    info->n_eval = out.n_eval;
    info->status = out.status;
  }
  if (out.status != MIPWA_OK)
    return ctx->fail(MIPWA_E_NOCONV, "EDM above tolerance after max_iter iterations or a failed line search");
  return MIPWA_OK;
}
