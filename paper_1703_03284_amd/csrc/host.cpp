// Host FP64 setup: model validation, the natural-spline operator, per-evaluation tables and the
// cell-sorting point loader.
#include "host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

namespace mipwa {

namespace {

double barrier_poly(int L, double z) {
  if (L == 1) return 1.0 + z;
  if (L == 2) return (z + 3.0) * z + 9.0;
  return 1.0;
}

double barrier_poly_d(int L, double z) {
  if (L == 1) return 1.0;
  if (L == 2) return 2.0 * z + 3.0;
  return 0.0;
}

template <typename Real>
void fill_kin(Kin<Real>& k, double M, double m1, double m2, double m3, double rD) {
  const double M2 = M * M, a = m1 * m1, b = m2 * m2, c = m3 * m3;
  k.sum = Real(M2 + a + b + c);
  k.thr_hi = Real((m1 + m2) * (m1 + m2));
  k.thr_lo = Real((m1 - m2) * (m1 - m2));
  k.pb_hi = Real((M + m3) * (M + m3));
  k.pb_lo = Real((M - m3) * (M - m3));
  k.t1corr = Real((M2 - c) * (a - b));
  k.t2a = Real(2.0 * M2 + 2.0 * c);
  k.t2b = Real((M2 - c) * (M2 - c));
  k.t2c = Real(2.0 * a + 2.0 * b);
  k.t2d = Real((a - b) * (a - b));
  k.rD2 = Real(rD * rD);
}

}  // namespace

int ModelHost::init(const mipwa_model* m, std::string& err) {
  std::ostringstream os;
  if (!m) {
    err = "model is NULL";
    return MIPWA_E_INVAL;
  }
  if (!(m->M > 0 && m->m1 > 0 && m->m2 > 0 && m->m3 > 0) || !std::isfinite(m->M) || !std::isfinite(m->m1)) {
    err = "masses must be positive and finite";
    return MIPWA_E_INVAL;
  }
  if (m->m2 != m->m3) {
    err = "the two h+ must have equal masses (m2 == m3) for Bose symmetrisation";
    return MIPWA_E_INVAL;
  }
  if (!(m->M > m->m1 + m->m2 + m->m3)) {
    err = "M must exceed m1 + m2 + m3";
    return MIPWA_E_INVAL;
  }
  if (!(m->rD >= 0) || !std::isfinite(m->rD)) {
    err = "rD must be >= 0";
    return MIPWA_E_INVAL;
  }
  if (m->n_knots < 2 || m->n_knots > MIPWA_MAX_KNOTS || !m->knots) {
    os << "n_knots must be in [2, " << MIPWA_MAX_KNOTS << "]";
    err = os.str();
    return MIPWA_E_INVAL;
  }
  if (m->n_res < 0 || m->n_res > MIPWA_MAX_RES || (m->n_res > 0 && !m->res)) {
    os << "n_res must be in [0, " << MIPWA_MAX_RES << "]";
    err = os.str();
    return MIPWA_E_INVAL;
  }
  M = m->M;
  m1 = m->m1;
  m2 = m->m2;
  m3 = m->m3;
  rD = m->rD;
  N = m->n_knots;
  R = m->n_res;
  P = 2 * N + 4 * R;
  knots.assign(m->knots, m->knots + N);
  for (int k = 0; k < N; ++k) {
    if (!std::isfinite(knots[k]) || (k > 0 && !(knots[k] > knots[k - 1]))) {
      err = "knots must be finite and strictly increasing";
      return MIPWA_E_INVAL;
    }
  }
  res.assign(m->res, m->res + R);
  for (int r = 0; r < R; ++r) {
    const mipwa_res& q = res[r];
    if (q.spin < 0 || q.spin > 2 || !(q.width > 0) || !(q.radius >= 0) || !std::isfinite(q.mass) ||
        !std::isfinite(q.width) || !std::isfinite(q.radius)) {
      os << "resonance " << r << ": spin must be 0..2, width > 0, radius >= 0";
      err = os.str();
      return MIPWA_E_INVAL;
    }
    if (!(q.mass > m1 + m2) || !(q.mass < M - m3)) {
      os << "resonance " << r << ": mass must lie between m1 + m2 and M - m3";
      err = os.str();
      return MIPWA_E_INVAL;
    }
  }
  h.resize(N - 1);
  for (int j = 0; j < N - 1; ++j) h[j] = knots[j + 1] - knots[j];
  // Thomas factorisation of the interior system
  //   h_{k-1} M_{k-1} + 2 (h_{k-1} + h_k) M_k + h_k M_{k+1} = rhs_k,  k = 1..N-2,  M_0 = M_{N-1} = 0.
  const int n = N - 2;
  th_c.assign(std::max(n, 1), 0.0);
  th_d.assign(std::max(n, 1), 0.0);
  for (int i = 0; i < n; ++i) {
    const int k = i + 1;
    const double a = h[k - 1], b = 2.0 * (h[k - 1] + h[k]), c = h[k];
    const double den = b - (i > 0 ? a * th_c[i - 1] : 0.0);
    th_d[i] = den;
    th_c[i] = c / den;
  }
  inv_h.resize(N - 1);
  for (int j = 0; j < N - 1; ++j) inv_h[j] = 1.0 / h[j];
  inv_d.assign(th_d.size(), 0.0);
  for (int i = 0; i < n; ++i) inv_d[i] = 1.0 / th_d[i];
  fill_kin(kin64, M, m1, m2, m3, rD);
  fill_kin(kin32, M, m1, m2, m3, rD);
  return MIPWA_OK;
}

void ModelHost::second_derivs(const double* zr, const double* zi, double* Mr, double* Mi) const {
  const int n = N - 2;
  Mr[0] = Mi[0] = Mr[N - 1] = Mi[N - 1] = 0.0;
  if (n <= 0) return;
  double yr[kMaxKnots], yi[kMaxKnots];
  for (int i = 0; i < n; ++i) {
    const int k = i + 1;
    const double rr = 6.0 * ((zr[k + 1] - zr[k]) * inv_h[k] - (zr[k] - zr[k - 1]) * inv_h[k - 1]);
    const double ri = 6.0 * ((zi[k + 1] - zi[k]) * inv_h[k] - (zi[k] - zi[k - 1]) * inv_h[k - 1]);
    const double a = h[k - 1];
    yr[i] = (rr - (i > 0 ? a * yr[i - 1] : 0.0)) * inv_d[i];
    yi[i] = (ri - (i > 0 ? a * yi[i - 1] : 0.0)) * inv_d[i];
  }
  for (int i = n - 1; i >= 0; --i) {
    if (i < n - 1) {
      yr[i] -= th_c[i] * yr[i + 1];
      yi[i] -= th_c[i] * yi[i + 1];
    }
    Mr[i + 1] = yr[i];
    Mi[i + 1] = yi[i];
  }
}

void ModelHost::poly_table(const double* theta, double* out) const {
  double zr[kMaxKnots], zi[kMaxKnots], Mr[kMaxKnots], Mi[kMaxKnots];
  for (int k = 0; k < N; ++k) {
    const double a = theta[2 * k], ph = theta[2 * k + 1];
    double sn, cs;
    sincos(ph, &sn, &cs);
    zr[k] = a * cs;
    zi[k] = a * sn;
  }
  second_derivs(zr, zi, Mr, Mi);
  // S on interval j with t = (s - s_j)/h_j:  S = P0 + P1 t + P2 t^2 + P3 t^3 with
  //   P0 = z_j, P1 = z_{j+1} - z_j - (h^2/6)(2 M_j + M_{j+1}), P2 = (h^2/2) M_j, P3 = (h^2/6)(M_{j+1} - M_j).
  for (int j = 0; j < N - 1; ++j) {
    const double c6 = h[j] * h[j] / 6.0;
    double* p = out + 8 * j;
    p[0] = zr[j];
    p[1] = zi[j];
    p[2] = zr[j + 1] - zr[j] - c6 * (2.0 * Mr[j] + Mr[j + 1]);
    p[3] = zi[j + 1] - zi[j] - c6 * (2.0 * Mi[j] + Mi[j + 1]);
    p[4] = 3.0 * c6 * Mr[j];
    p[5] = 3.0 * c6 * Mi[j];
    p[6] = c6 * (Mr[j + 1] - Mr[j]);
    p[7] = c6 * (Mi[j + 1] - Mi[j]);
  }
}

void ModelHost::res_table(const double* theta, double* out) const {
  const double thr_hi = (m1 + m2) * (m1 + m2), thr_lo = (m1 - m2) * (m1 - m2);
  const double pb_hi = (M + m3) * (M + m3), pb_lo = (M - m3) * (M - m3);
  for (int r = 0; r < R; ++r) {
    const int L = res[r].spin;
    const double m = theta[2 * N + 2 * R + 2 * r], G = theta[2 * N + 2 * R + 2 * r + 1];
    const double rho2 = res[r].radius * res[r].radius, rD2 = rD * rD;
    const double s = m * m;
    const double q2 = (s - thr_hi) * (s - thr_lo) / (4.0 * s);
    const double p2 = (s - pb_hi) * (s - pb_lo) / (4.0 * s);
    const double dq2_dm = 2.0 * m * (((s - thr_lo) + (s - thr_hi)) / (4.0 * s) - q2 / s);
    const double dp2_dm = 2.0 * m * (((s - pb_lo) + (s - pb_hi)) / (4.0 * s) - p2 / s);
    const double zq = rho2 * q2, zp = rD2 * p2;
    const double K1 = barrier_poly(L, zq), K2 = barrier_poly(L, zp);
    const double dK1 = barrier_poly_d(L, zq) * rho2 * dq2_dm;
    const double dK2 = barrier_poly_d(L, zp) * rD2 * dp2_dm;
    const double kappa = std::sqrt(K1 * K2);
    double qpow = std::sqrt(q2);  // q^(2L+1)
    for (int l = 0; l < L; ++l) qpow *= q2;
    const double delta = G * s * K1 / qpow;
    const double dln_delta = 2.0 / m + dK1 / K1 - 0.5 * (2 * L + 1) * dq2_dm / q2;
    double* o = out + kResWords * r;
    o[0] = s;
    o[1] = kappa;
    o[2] = delta;
    o[3] = rho2;
    o[4] = (double)L;
    o[5] = m;
    o[6] = 0.5 * (dK1 / K1 + dK2 / K2);
    o[7] = delta * dln_delta;
    o[8] = s * K1 / qpow;
    o[9] = 0.0;
  }
}

void ModelHost::eval_table(const double* theta, bool fp64, void* out, bool residues) const {
  const int nint = N - 1, tw = table_words(nint, R);
  double tab[table_words(kMaxKnots - 1, kMaxRes)];
  poly_table(theta, tab);
  for (int r = 0; r < R; ++r) {
    const double cm = theta[2 * N + 2 * r], ca = theta[2 * N + 2 * r + 1];
    double sn, cs;
    sincos(ca, &sn, &cs);
    tab[8 * nint + 2 * r] = cm * cs;
    tab[8 * nint + 2 * r + 1] = cm * sn;
  }
  res_table(theta, tab + 8 * nint + 2 * R);
  if (fp64) {
    std::memcpy(out, tab, (size_t)tw * sizeof(double));
    return;
  }
  float* f = static_cast<float*>(out);
  for (int i = 0; i < tw; ++i) f[i] = (float)tab[i];
  float* lo = f + tw;
  if (!residues) {
    std::memset(lo, 0, (size_t)table_lo_words(nint, R) * sizeof(float));
    return;
  }
  for (int j = 0; j < nint; ++j)
    for (int m = 0; m < 4; ++m) lo[4 * j + m] = (float)(tab[8 * j + m] - (double)f[8 * j + m]);
  for (int k = 0; k < 2 * R; ++k) lo[4 * nint + k] = (float)(tab[8 * nint + k] - (double)f[8 * nint + k]);
}

int ModelHost::upload_res64(const double* theta, DevBuf& d, hipStream_t st) const {
  std::vector<double> r((size_t)kResWords * std::max(R, 1), 0.0);
  res_table(theta, r.data());
  if (d.alloc(r.size() * sizeof(double)) != hipSuccess) return MIPWA_E_NOMEM;
  if (st) {
    if (hipMemcpyAsync(d.p, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return MIPWA_E_HIP;
  } else if (hipMemcpy(d.p, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    return MIPWA_E_HIP;
  }
  return MIPWA_OK;
}

int ModelHost::interval(double s) const {
  // number of knots <= s, minus one, clamped to [0, N-2]
  const int c = (int)(std::upper_bound(knots.begin(), knots.end(), s) - knots.begin());
  return std::min(std::max(c - 1, 0), N - 2);
}

bool ModelHost::inside(double s12, double s13, double tol) const {
  if (!(s12 >= smin() - tol && s12 <= smax() + tol)) return false;
  const double x = std::min(std::max(s12, smin()), smax());
  const double rs = std::sqrt(x);
  const double e1 = (x - m2 * m2 + m1 * m1) / (2.0 * rs);
  const double e3 = (M * M - x - m3 * m3) / (2.0 * rs);
  const double p1 = std::sqrt(std::max(e1 * e1 - m1 * m1, 0.0));
  const double p3 = std::sqrt(std::max(e3 * e3 - m3 * m3, 0.0));
  const double es = (e1 + e3) * (e1 + e3);
  return s13 >= es - (p1 + p3) * (p1 + p3) - tol && s13 <= es - (p1 - p3) * (p1 - p3) + tol;
}

int ModelHost::check_theta(const double* theta, std::string& err) const {
  for (int p = 0; p < P; ++p)
    if (!std::isfinite(theta[p])) {
      err = "theta[" + std::to_string(p) + "] is not finite";
      return MIPWA_E_INVAL;
    }
  for (int r = 0; r < R; ++r) {
    const double m = theta[2 * N + 2 * R + 2 * r], G = theta[2 * N + 2 * R + 2 * r + 1];
    if (!(G > 0)) {
      err = "width of resonance " + std::to_string(r) + " must be > 0";
      return MIPWA_E_INVAL;
    }
    if (!(m > m1 + m2) || !(m < M - m3)) {
      err = "mass of resonance " + std::to_string(r) + " outside (m1 + m2, M - m3)";
      return MIPWA_E_INVAL;
    }
  }
  return MIPWA_OK;
}

}  // namespace mipwa
