// The fit's BFGS minimiser (csrc/fit.cpp) on objectives whose answers are known in closed form, built
// by tests/test_minimizer.py under AddressSanitizer and UBSan.  Prints one line per failed check and
// a final count; exits non-zero on any failure.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "minimizer.h"
#include "mipwa.h"

using namespace mipwa;

static int fails = 0;
static void check(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL %s\n", what);
    ++fails;
  }
}

// x = A^-1 b for a small dense SPD A (Gauss-Jordan, fine at these sizes)
static std::vector<double> solve(std::vector<double> A, std::vector<double> b, int n) {
  for (int c = 0; c < n; ++c) {
    const double p = A[c * n + c];
    for (int j = 0; j < n; ++j) A[c * n + j] /= p;
    b[c] /= p;
    for (int r = 0; r < n; ++r)
      if (r != c) {
        const double f = A[r * n + c];
        for (int j = 0; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
        b[r] -= f * b[c];
      }
  }
  return b;
}

int main() {
  std::mt19937_64 rng(5);
  std::uniform_real_distribution<double> u(-1.0, 1.0);

  // f = (x - a)^T A (x - a), A = L L^T + I: minimum a, Hessian 2A, covariance 2 H^-1 = A^-1
  const int n = 6;
  std::vector<double> L(n * n), A(n * n, 0.0), a(n);
  for (auto& v : L) v = u(rng);
  for (int i = 0; i < n; ++i) {
    a[i] = 2.0 * u(rng);
    for (int j = 0; j < n; ++j) {
      for (int k = 0; k < n; ++k) A[i * n + j] += L[i * n + k] * L[j * n + k];
      if (i == j) A[i * n + j] += 1.0;
    }
  }
  FullEval quad = [&](const double* x, double& f, double* g) {
    f = 0.0;
    for (int i = 0; i < n; ++i) {
      double Ad = 0.0;
      for (int j = 0; j < n; ++j) Ad += A[i * n + j] * (x[j] - a[j]);
      f += (x[i] - a[i]) * Ad;
      g[i] = 2.0 * Ad;
    }
    return MIPWA_OK;
  };
  {
    std::vector<double> x0(n, 0.0);
    FitOut out;
    const int rc = bfgs_fit(quad, n, {}, std::vector<unsigned char>(n, 0), x0.data(), 1e-14, 500, true, 1e-13, out);
    check(rc == MIPWA_OK && out.status == MIPWA_OK, "quadratic: converges");
    double dx = 0.0, dc = 0.0, cmax = 0.0;
    for (int i = 0; i < n; ++i) {
      dx = std::max(dx, std::fabs(out.theta[i] - a[i]));
      std::vector<double> e(n, 0.0);
      e[i] = 1.0;
      const std::vector<double> col = solve(A, e, n);  // column i of A^-1
      for (int j = 0; j < n; ++j) {
        dc = std::max(dc, std::fabs(out.cov[j * n + i] - col[j]));
        cmax = std::max(cmax, std::fabs(col[j]));
      }
    }
    check(dx < 1e-6, "quadratic: minimum");
    check(dc < 1e-6 * cmax, "quadratic: covariance = A^-1");
    check(std::fabs(out.nll) < 1e-12, "quadratic: f at the minimum");
    check(out.n_eval > 0 && out.n_iter > 0 && out.n_iter <= 3 * n, "quadratic: iteration count");
  }

  // held parameters: x_2 and x_4 fixed off their optimum; the free ones reach the conditional minimum
  // x_f = a_f - A_ff^-1 A_fh (x_h - a_h)
  {
    std::vector<unsigned char> fx(n, 0);
    fx[2] = fx[4] = 1;
    std::vector<double> x0(n, 0.0);
    x0[2] = a[2] + 0.7;
    x0[4] = a[4] - 0.4;
    FitOut out;
    const int rc = bfgs_fit(quad, n, {}, fx, x0.data(), 1e-14, 500, false, 1e-13, out);
    check(rc == MIPWA_OK && out.status == MIPWA_OK, "held: converges");
    check(out.theta[2] == x0[2] && out.theta[4] == x0[4], "held: values unchanged");
    std::vector<int> fr;
    for (int i = 0; i < n; ++i)
      if (!fx[i]) fr.push_back(i);
    const int m = (int)fr.size();
    std::vector<double> Aff(m * m), rhs(m);
    for (int i = 0; i < m; ++i) {
      for (int j = 0; j < m; ++j) Aff[i * m + j] = A[fr[i] * n + fr[j]];
      rhs[i] = -(A[fr[i] * n + 2] * (x0[2] - a[2]) + A[fr[i] * n + 4] * (x0[4] - a[4]));
    }
    const std::vector<double> dxf = solve(Aff, rhs, m);
    double err = 0.0;
    for (int i = 0; i < m; ++i) err = std::max(err, std::fabs(out.theta[fr[i]] - (a[fr[i]] + dxf[i])));
    check(err < 1e-6, "held: conditional minimum");
    double covh = 0.0;
    for (int q = 0; q < n; ++q) covh += std::fabs(out.cov[2 * n + q]) + std::fabs(out.cov[q * n + 4]);
    check(covh == 0.0, "held: zero covariance rows and columns");
  }

  // Rosenbrock, 2 and 10 dimensions: minimum at (1, ..., 1)
  for (int d : {2, 10}) {
    FullEval rb = [d](const double* x, double& f, double* g) {
      f = 0.0;
      for (int i = 0; i < d; ++i) g[i] = 0.0;
      for (int i = 0; i + 1 < d; ++i) {
        const double t = x[i + 1] - x[i] * x[i], v = 1.0 - x[i];
        f += 100.0 * t * t + v * v;
        g[i] += -400.0 * x[i] * t - 2.0 * v;
        g[i + 1] += 200.0 * t;
      }
      return MIPWA_OK;
    };
    std::vector<double> x0(d);
    for (int i = 0; i < d; ++i) x0[i] = i % 2 ? 1.0 : -1.2;
    FitOut out;
    const int rc = bfgs_fit(rb, d, {}, std::vector<unsigned char>(d, 0), x0.data(), 1e-16, 2000, false, 1e-13, out);
    check(rc == MIPWA_OK && out.status == MIPWA_OK, "rosenbrock: converges");
    double err = 0.0;
    for (int i = 0; i < d; ++i) err = std::max(err, std::fabs(out.theta[i] - 1.0));
    check(err < 1e-5, "rosenbrock: minimum at ones");
    // the iteration limit: status E_NOCONV with the best point so far, the call itself succeeds
    FitOut lim;
    const int rc2 = bfgs_fit(rb, d, {}, std::vector<unsigned char>(d, 0), x0.data(), 1e-16, 3, false, 1e-13, lim);
    check(rc2 == MIPWA_OK && lim.status == MIPWA_E_NOCONV && lim.n_iter == 3, "rosenbrock: iteration limit");
  }

  // a (magnitude, phase) pair reaching a negative magnitude is folded to (|r|, phase + pi) in (-pi, pi],
  // and its covariance row and column change sign with the magnitude
  {
    const double tu = -0.8, tv = 0.3;  // target point r (cos p, sin p) = (tu, tv) * r0 with r0 < 0 reachable
    FullEval pol = [&](const double* x, double& f, double* g) {
      const double c = std::cos(x[1]), s = std::sin(x[1]);
      const double ex = x[0] * c - tu, ey = x[0] * s - tv, ez = x[2] - 0.25 * x[0];
      f = ex * ex + ey * ey + ez * ez;
      g[0] = 2.0 * (ex * c + ey * s) - 0.5 * ez;
      g[1] = 2.0 * (-ex * x[0] * s + ey * x[0] * c);
      g[2] = 2.0 * ez;
      return MIPWA_OK;
    };
    const double x0[3] = {-0.7, -0.3, 0.0};  // near r = -|t|, p = atan2(tv, tu) - pi
    FitOut plain, folded;
    const std::vector<unsigned char> none(3, 0);
    const int rc1 = bfgs_fit(pol, 3, {}, none, x0, 1e-16, 500, true, 1e-13, plain);
    const int rc2 = bfgs_fit(pol, 3, {0}, none, x0, 1e-16, 500, true, 1e-13, folded);
    check(rc1 == MIPWA_OK && rc2 == MIPWA_OK && plain.status == MIPWA_OK, "polar: converges");
    check(plain.theta[0] < 0.0, "polar: unfolded magnitude negative");
    const double r = std::hypot(tu, tv);
    check(std::fabs(folded.theta[0] - r) < 1e-6, "polar: folded magnitude");
    check(std::fabs(folded.theta[1] - std::atan2(tv, tu)) < 1e-6, "polar: folded phase");
    check(folded.theta[1] > -M_PI && folded.theta[1] <= M_PI, "polar: phase range");
    check(std::fabs(folded.cov[0 * 3 + 2] + plain.cov[0 * 3 + 2]) < 1e-9 &&
              std::fabs(folded.cov[2 * 3 + 0] + plain.cov[2 * 3 + 0]) < 1e-9 &&
              std::fabs(folded.cov[1 * 3 + 2] - plain.cov[1 * 3 + 2]) < 1e-9,
          "polar: covariance signs");
  }

  // +inf outside the domain: f = x^2 - ln x, minimum at 1/sqrt(2); the first trial steps overshoot
  // into x <= 0 and must be pulled back
  {
    FullEval dom = [](const double* x, double& f, double* g) {
      if (!(x[0] > 0.0)) {
        f = INFINITY;
        g[0] = 0.0;
        return MIPWA_OK;
      }
      f = x[0] * x[0] - std::log(x[0]);
      g[0] = 2.0 * x[0] - 1.0 / x[0];
      return MIPWA_OK;
    };
    const double x0 = 30.0;
    FitOut out;
    const int rc = bfgs_fit(dom, 1, {}, std::vector<unsigned char>(1, 0), &x0, 1e-16, 200, false, 1e-13, out);
    check(rc == MIPWA_OK && out.status == MIPWA_OK, "domain: converges");
    check(std::fabs(out.theta[0] - std::sqrt(0.5)) < 1e-6, "domain: minimum");
  }

  // errors: a callback failure aborts with its status; nothing floated; a non-finite start
  {
    int calls = 0;
    FullEval bad = [&](const double* x, double& f, double* g) -> int {
      if (++calls == 4) return MIPWA_E_HIP;
      return quad(x, f, g);
    };
    std::vector<double> x0(n, 0.0);
    FitOut out;
    check(bfgs_fit(bad, n, {}, std::vector<unsigned char>(n, 0), x0.data(), 1e-14, 500, false, 1e-13, out) ==
              MIPWA_E_HIP,
          "errors: callback status returned");
    check(bfgs_fit(quad, n, {}, std::vector<unsigned char>(n, 1), x0.data(), 1e-14, 500, false, 1e-13, out) ==
              MIPWA_E_INVAL,
          "errors: every parameter held");
    FullEval nan = [](const double*, double& f, double* g) {
      f = NAN;
      g[0] = 0.0;
      return MIPWA_OK;
    };
    const double z = 1.0;
    check(bfgs_fit(nan, 1, {}, std::vector<unsigned char>(1, 0), &z, 1e-14, 500, false, 1e-13, out) ==
              MIPWA_E_DOMAIN,
          "errors: non-finite start");
  }

  std::printf("minimizer: %d failures\n", fails);
  return fails ? 1 : 0;
}
