// Host-side model code (spline setup, evaluation and resonance tables, intervals, region test) under
// AddressSanitizer and UBSan, built by tests/test_host_memory.py: exact-size heap buffers for every
// table routine, models from 2 to 128 knots with 0 to 4 resonances of every spin.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "host.h"

using namespace mipwa;

int main() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  const double M = 1.86966, m = 0.13957;
  const double smin = 4 * m * m, smax = (M - m) * (M - m);
  int checked = 0;
  for (int N : {2, 3, 4, 5, 17, 50, 127, 128}) {
    for (int R : {0, 1, 2, 3, 4}) {
      std::vector<double> knots(N);
      for (int k = 0; k < N; ++k) knots[k] = smin + (smax - smin) * k / (N - 1);
      std::vector<mipwa_res> res(R);
      const double masses[4] = {0.775, 1.275, 0.98, 1.465}, widths[4] = {0.149, 0.185, 0.07, 0.4};
      for (int r = 0; r < R; ++r) res[r] = mipwa_res{r % 3 == 2 ? 0 : 1 + r % 2, masses[r], widths[r], 1.5};
      mipwa_model md{M, m, m, m, 5.0, N, knots.data(), R, res.data()};
      ModelHost mh;
      std::string err;
      if (mh.init(&md, err) != 0) {
        std::printf("init N=%d R=%d failed: %s\n", N, R, err.c_str());
        return 1;
      }
      std::vector<double> theta(mh.P);
      for (int k = 0; k < N; ++k) {
        theta[2 * k] = 0.5 + 1.5 * u(rng);
        theta[2 * k + 1] = -3.0 + 6.0 * u(rng);
      }
      for (int r = 0; r < R; ++r) {
        theta[2 * N + 2 * r] = 0.2 + u(rng);
        theta[2 * N + 2 * r + 1] = -3.0 + 6.0 * u(rng);
        theta[2 * N + 2 * R + 2 * r] = masses[r];
        theta[2 * N + 2 * R + 2 * r + 1] = widths[r];
      }
      if (mh.check_theta(theta.data(), err) != 0) {
        std::printf("check_theta N=%d R=%d: %s\n", N, R, err.c_str());
        return 1;
      }
      std::vector<double> zr(N), zi(N), Mr(N), Mi(N);
      for (int k = 0; k < N; ++k) {
        zr[k] = u(rng);
        zi[k] = u(rng);
      }
      mh.second_derivs(zr.data(), zi.data(), Mr.data(), Mi.data());
      std::vector<double> poly((size_t)8 * (N - 1));
      mh.poly_table(theta.data(), poly.data());
      std::vector<double> rt((size_t)kResWords * R);
      mh.res_table(theta.data(), rt.data());
      for (bool fp64 : {true, false})
        for (bool residues : {true, false}) {
          const size_t bytes = (size_t)table_real_words(N - 1, R, fp64) * (fp64 ? 8 : 4);
          std::vector<unsigned char> tab(bytes);
          mh.eval_table(theta.data(), fp64, tab.data(), residues);
        }
      for (int i = 0; i < 1000; ++i) {
        const double s = smin - 0.1 + (smax - smin + 0.2) * u(rng);
        const int j = mh.interval(s);
        if (j < 0 || j > N - 2) {
          std::printf("interval out of range\n");
          return 1;
        }
        (void)mh.inside(s, smin + (smax - smin) * u(rng), 1e-9);
      }
      ++checked;
    }
  }
  std::printf("host model code: %d models checked\n", checked);
  return 0;
}
