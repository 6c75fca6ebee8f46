// BFGS fit over a full-parameter evaluation callback; used by mipwa_fit (one context) and by the
// serving loop (evaluations batched across jobs).  Internal.
#pragma once

#include <functional>
#include <string>
#include <vector>

namespace mipwa {

// theta: P doubles -> f (may be +inf for an invalid or non-finite point) and the P-gradient.
// A non-zero return aborts the fit with that status.
using FullEval = std::function<int(const double* theta, double& f, double* grad)>;

struct FitOut {
  std::vector<double> theta, cov;  // folded theta; P x P covariance (zero rows for fixed parameters)
  double nll = 0, edm = 0;
  int n_iter = 0, n_eval = 0, status = 0;
  std::string err;
};

// Noise of f, relative to |f|, that the line search tolerates.  In mixed precision the per-point FP32
// rounding of ln|A|^2 and |A|^2 sums to ~1e-5 absolute at 10^4 events (f ~ 2.5e4) and grows with the
// event count; 1e-8 |f| covers it at every size, and the search then decides by the gradient's sign.
constexpr double kNoiseRelFp64 = 1e-13, kNoiseRelMixed = 1e-8;

// polar_pairs: indices i of (magnitude, phase) pairs (theta[i], theta[i+1]) folded to magnitude >= 0,
// phase in (-pi, pi] at the end
int bfgs_fit(const FullEval& fg, int P, const std::vector<int>& polar_pairs, const std::vector<unsigned char>& fixed,
             const double* theta0, double tol, int max_iter, bool hessian, double eps_rel, FitOut& out);

}  // namespace mipwa
