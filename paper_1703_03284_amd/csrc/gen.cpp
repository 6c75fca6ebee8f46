// Toy Monte Carlo on the device: Philox candidates, accept-reject on |A|^2 eff, order-preserving
// compaction (Sec. 4 toy samples generated from the Dalitz-plot PDF).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "mipwa.h"

using namespace mipwa;

namespace {

constexpr int kChunk = 1 << 20;

struct GenState {
  DevBuf tab, c12, c13, f, flag, counts, offsets, total, exceeded, o12, o13, of;
  GenArgs g{};
};

int gen_setup(mipwa_ctx* ctx, const double* ext_theta, int n_theta, uint64_t seed, double fmax, int mode, GenState& s) {
  const ModelHost& mh = ctx->mh;
  if (!ext_theta || n_theta != ctx->ext_P()) return ctx->fail(MIPWA_E_INVAL, "theta must have P entries");
  std::vector<double> internal(mh.P);
  ctx->to_internal(ext_theta, internal.data());
  const double* theta = internal.data();
  int rc = mh.check_theta(theta, ctx->err);
  if (rc) return rc;
  const int nint = mh.N - 1;
  std::vector<double> tab(8 * nint + mh.N + 2 * mh.R + kResWords * mh.R);
  mh.poly_table(theta, tab.data());
  std::copy(mh.knots.begin(), mh.knots.end(), tab.begin() + 8 * nint);
  double* c = tab.data() + 8 * nint + mh.N;
  for (int r = 0; r < mh.R; ++r) {
    const double cm = theta[2 * mh.N + 2 * r], ca = theta[2 * mh.N + 2 * r + 1];
    c[2 * r] = cm * std::cos(ca);
    c[2 * r + 1] = cm * std::sin(ca);
  }
  mh.res_table(theta, c + 2 * mh.R);
  const size_t nb = (kChunk + kGenBlock - 1) / kGenBlock;
  if (s.tab.alloc(tab.size() * 8) || s.c12.alloc(kChunk * 8) || s.c13.alloc(kChunk * 8) || s.f.alloc(kChunk * 8) ||
      s.flag.alloc(kChunk) || s.counts.alloc(nb * 4) || s.offsets.alloc(nb * 4) || s.total.alloc(16) ||
      s.exceeded.alloc(16) || s.o12.alloc(kChunk * 8) || s.o13.alloc(kChunk * 8) || s.of.alloc(kChunk * 8))
    return ctx->fail(MIPWA_E_NOMEM, "generator buffers");
  if (hipMemcpy(s.tab.p, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(s.exceeded.p, 0, 16) != hipSuccess)
    return ctx->fail(MIPWA_E_HIP, "generator table upload");
  const double* d = s.tab.as<double>();
  GenArgs& g = s.g;
  g.poly = d;
  g.knots = d + 8 * nint;
  g.c = d + 8 * nint + mh.N;
  g.res = g.c + 2 * mh.R;
  g.eff = ctx->eff.set() ? ctx->eff.d.as<float>() : nullptr;
  g.N = mh.N;
  g.R = mh.R;
  g.nx = ctx->eff.nx;
  g.ny = ctx->eff.ny;
  g.eff_lo = ctx->eff.lo;
  g.eff_hi = ctx->eff.hi;
  g.M = mh.M;
  g.m1 = mh.m1;
  g.m2 = mh.m2;
  g.m3 = mh.m3;
  g.smin = mh.smin();
  g.span = mh.smax() - mh.smin();
  g.seed = seed;
  g.fmax = fmax;
  g.mode = mode;
  return MIPWA_OK;
}

// evaluate one chunk of candidates and compact the kept ones; returns the number kept
int gen_chunk(mipwa_ctx* ctx, GenState& s, long long first, int* kept) {
  hipStream_t st = ctx->stream;
  if (launch_generate_chunk(s.g, &ctx->mh.kin64, first, kChunk, s.c12.as<double>(), s.c13.as<double>(),
                            s.f.as<double>(), s.flag.as<unsigned char>(), s.counts.as<int>(), s.exceeded.as<int>(),
                            st) != hipSuccess ||
      launch_compact(s.flag.as<unsigned char>(), kChunk, s.counts.as<int>(), s.offsets.as<int>(), s.total.as<int>(),
                     s.c12.as<double>(), s.c13.as<double>(), s.f.as<double>(), s.o12.as<double>(),
                     s.o13.as<double>(), s.of.as<double>(), st) != hipSuccess)
    return ctx->fail(MIPWA_E_HIP, "generator kernels");
  if (hipMemcpyAsync(kept, s.total.p, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return ctx->fail(MIPWA_E_HIP, "generator count");
  return MIPWA_OK;
}

}  // namespace

extern "C" {

int mipwa_generate(mipwa_ctx* ctx, const double* theta, int n_theta, uint64_t seed, double fmax, int64_t n,
                   double* s12_out, double* s13_out, int* exceeded, int64_t* n_candidates) {
  if (!ctx) return MIPWA_E_INVAL;
  if (n < 1 || !(fmax > 0) || !s12_out || !s13_out) return ctx->fail(MIPWA_E_INVAL, "need n >= 1, fmax > 0 and outputs");
  (void)hipSetDevice(ctx->device);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return ctx->fail(MIPWA_E_HIP, "stream sync");
  GenState s;
  int rc = gen_setup(ctx, theta, n_theta, seed, fmax, 0, s);
  if (rc) return rc;
  long long have = 0, first = 0;
  while (have < n) {
    int kept = 0;
    rc = gen_chunk(ctx, s, first, &kept);
    if (rc) return rc;
    const long long take = std::min<long long>(kept, n - have);
    if (take > 0 && (hipMemcpy(s12_out + have, s.o12.p, take * 8, hipMemcpyDeviceToHost) != hipSuccess ||
                     hipMemcpy(s13_out + have, s.o13.p, take * 8, hipMemcpyDeviceToHost) != hipSuccess))
      return ctx->fail(MIPWA_E_HIP, "generator copy");
    have += take;
    first += kChunk;
  }
  int exc = 0;
  if (hipMemcpy(&exc, s.exceeded.p, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return ctx->fail(MIPWA_E_HIP, "generator flag copy");
  if (exceeded) *exceeded = exc;
  if (n_candidates) *n_candidates = first;
  return MIPWA_OK;
}

int mipwa_density_max(mipwa_ctx* ctx, const double* theta, int n_theta, uint64_t seed, int64_t n_probe,
                      double* fmax_out) {
  if (!ctx) return MIPWA_E_INVAL;
  if (n_probe < 1 || !fmax_out) return ctx->fail(MIPWA_E_INVAL, "need n_probe >= 1 and an output");
  (void)hipSetDevice(ctx->device);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return ctx->fail(MIPWA_E_HIP, "stream sync");
  GenState s;
  int rc = gen_setup(ctx, theta, n_theta, seed, 1.0, 1, s);
  if (rc) return rc;
  long long seen = 0, first = 0;
  double best = 0.0;
  std::vector<double> f;
  while (seen < n_probe) {
    int kept = 0;
    rc = gen_chunk(ctx, s, first, &kept);
    if (rc) return rc;
    const long long take = std::min<long long>(kept, n_probe - seen);
    f.resize(take);
    if (take > 0 && hipMemcpy(f.data(), s.of.p, take * 8, hipMemcpyDeviceToHost) != hipSuccess)
      return ctx->fail(MIPWA_E_HIP, "generator copy");
    for (double v : f) best = std::max(best, v);
    seen += take;
    first += kChunk;
  }
  *fmax_out = best;
  return MIPWA_OK;
}

int mipwa_toy(mipwa_ctx* ctx, const double* theta, int n_theta, uint64_t seed, int64_t n_probe, int64_t n,
              double* s12_out, double* s13_out, double* fmax_out) {
  if (!ctx) return MIPWA_E_INVAL;
  if (n_probe < 1) return ctx->fail(MIPWA_E_INVAL, "need n_probe >= 1");
  double fmax = 0.0;
  int rc = mipwa_density_max(ctx, theta, n_theta, seed + 1000, n_probe, &fmax);
  if (rc) return rc;
  if (!(fmax > 0.0) || !std::isfinite(fmax)) return ctx->fail(MIPWA_E_INVAL, "the density is zero or not finite over the probe");
  fmax *= 1.5;
  for (;;) {
    int exceeded = 0;
    rc = mipwa_generate(ctx, theta, n_theta, seed, fmax, n, s12_out, s13_out, &exceeded, nullptr);
    if (rc) return rc;
    if (!exceeded) break;
    fmax *= 2.0;
  }
  if (fmax_out) *fmax_out = fmax;
  return MIPWA_OK;
}

}  // extern "C"
