// Point loading on the device: validation, canonical order s12 <= s13, spline cells, a stable sort
// of the points by cell, local spline coordinates and weights.  Same order and the same FP64
// arithmetic as a host counting sort would give (floating-point contraction is off here).
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "engine.h"
#include "host.h"

#pragma clang fp contract(off)

namespace mipwa {
namespace {

struct RegionArgs {
  double M, m1, m2, m3, smin, smax, tol;
};

__device__ bool inside_dev(const RegionArgs& g, double s12, double s13) {
  if (!(s12 >= g.smin - g.tol && s12 <= g.smax + g.tol)) return false;
  const double x = fmin(fmax(s12, g.smin), g.smax);
  const double rs = sqrt(x);
  const double e1 = (x - g.m2 * g.m2 + g.m1 * g.m1) / (2.0 * rs);
  const double e3 = (g.M * g.M - x - g.m3 * g.m3) / (2.0 * rs);
  const double p1 = sqrt(fmax(e1 * e1 - g.m1 * g.m1, 0.0));
  const double p3 = sqrt(fmax(e3 * e3 - g.m3 * g.m3, 0.0));
  const double es = (e1 + e3) * (e1 + e3);
  return s13 >= es - (p1 + p3) * (p1 + p3) - g.tol && s13 <= es - (p1 - p3) * (p1 - p3) + g.tol;
}

// number of knots <= s, minus one, clamped to [0, N-2] (a point on a knot belongs to the interval above)
__device__ int interval_dev(const double* kn, int N, double s) {
  int lo = 0, hi = N;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (kn[mid] <= s) lo = mid + 1;
    else hi = mid;
  }
  return min(max(lo - 1, 0), N - 2);
}

__global__ __launch_bounds__(256) void k_prepare(const double* __restrict__ s12, const double* __restrict__ s13,
                                                 const double* __restrict__ w, const double* __restrict__ eff,
                                                 long long n, const double* __restrict__ knots, int N, RegionArgs g,
                                                 double* __restrict__ a, double* __restrict__ b,
                                                 unsigned* __restrict__ key, unsigned* __restrict__ idx,
                                                 unsigned long long* bad) {
  // bad[0]: first point outside the region or with a bad weight; bad[1]: first bad efficiency
  __shared__ double kn[kMaxKnots];
  for (int i = threadIdx.x; i < N; i += blockDim.x) kn[i] = knots[i];
  __syncthreads();
  const int nint = N - 1;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double x = s12[i], y = s13[i];
    bool ok = isfinite(x) && isfinite(y) && inside_dev(g, x, y);
    if (w) ok = ok && w[i] > 0 && isfinite(w[i]);
    if (!ok) atomicMin(&bad[0], (unsigned long long)i);
    if (eff && !(eff[i] > 0 && isfinite(eff[i]))) atomicMin(&bad[1], (unsigned long long)i);
    const double lo = fmin(x, y), hi = fmax(x, y);
    a[i] = lo;
    b[i] = hi;
    const int j12 = ok ? interval_dev(kn, N, lo) : 0, j13 = ok ? interval_dev(kn, N, hi) : 0;
    key[i] = (unsigned)(j12 * nint + j13);
    idx[i] = (unsigned)i;
  }
}

// first sorted position of every cell that holds points (the others keep -1)
__global__ __launch_bounds__(256) void k_cell_starts(const unsigned* __restrict__ key, long long n,
                                                     int* __restrict__ start) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    if (i == 0 || key[i - 1] != key[i]) start[key[i]] = (int)i;
}

template <typename Real>
__global__ __launch_bounds__(256) void k_gather(const unsigned* __restrict__ key, const unsigned* __restrict__ idx,
                                                const double* __restrict__ a, const double* __restrict__ b,
                                                const double* __restrict__ w, const double* __restrict__ eps,
                                                long long n, const double* __restrict__ knots,
                                                const double* __restrict__ h, int nint, Real* __restrict__ tt,
                                                double* __restrict__ ss, Real* __restrict__ wsorted,
                                                Real* __restrict__ wplain) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const unsigned o = idx[i], k = key[i];
    const int j12 = (int)(k / nint), j13 = (int)(k % nint);
    const double x = a[o], y = b[o];
    tt[2 * i] = Real((x - knots[j12]) / h[j12]);
    tt[2 * i + 1] = Real((y - knots[j13]) / h[j13]);
    ss[2 * i] = x;
    ss[2 * i + 1] = y;
    if (w) {
      wplain[i] = Real(w[o]);
      wsorted[i] = Real(w[o] * (eps ? eps[o] : 1.0));
    }
  }
}

int grid_for(long long n) { return (int)std::min<long long>((n + 255) / 256, 4096); }

// Scratch memory of one load, allocated and freed in stream order (from the given pool, else the
// device's default one): a plain free would wait for every stream on the device, including the
// evaluations of other jobs.
struct StreamBuf {
  void* p = nullptr;
  hipStream_t st = nullptr;
  hipMemPool_t pool = nullptr;
  explicit StreamBuf(hipMemPool_t pl) : pool(pl) {}
  StreamBuf(const StreamBuf&) = delete;
  StreamBuf& operator=(const StreamBuf&) = delete;
  ~StreamBuf() {
    if (p) (void)hipFreeAsync(p, st);
  }
  bool alloc(size_t n, hipStream_t s) {
    st = s;
    const hipError_t e = pool ? hipMallocFromPoolAsync(&p, n ? n : 16, pool, s) : hipMallocAsync(&p, n ? n : 16, s);
    if (e != hipSuccess) p = nullptr;
    return e != hipSuccess;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

#define LCHK(expr, what)                                  \
  do {                                                    \
    if ((expr) != hipSuccess) {                           \
      err = what;                                         \
      return MIPWA_E_HIP;                                 \
    }                                                     \
  } while (0)

}  // namespace

int load_points(const ModelHost& mh, bool fp64, int kind, const double* s12, const double* s13, const double* w,
                const double* eff, long long n, const EffTable& et, hipStream_t st, PointSet& ps, std::string& err,
                hipMemPool_t pool, hipStream_t free_st) {
  ps.loaded = false;
  if (n < 1 || !s12 || !s13 || (kind == 1 && !w)) {
    err = kind == 1 ? "need n >= 1 points with s12, s13 and w" : "need n >= 1 events with s12 and s13";
    return MIPWA_E_INVAL;
  }
  if (n > (1LL << 31) - kTile) {
    err = "at most 2^31 points per set";
    return MIPWA_E_INVAL;
  }
  const int N = mh.N, nint = N - 1;
  const size_t ncell = (size_t)nint * nint;
  (void)hipGetLastError();
  StreamBuf d12(pool), d13(pool), dw(pool), deff(pool), dkn(pool), dh(pool), da(pool), db(pool), dkey(pool),
      didx(pool), dkey2(pool), didx2(pool), dstart(pool), dbad(pool);
  if (d12.alloc(n * 8, st) || d13.alloc(n * 8, st) || (kind == 1 && dw.alloc(n * 8, st)) ||
      (eff && deff.alloc(n * 8, st)) || dkn.alloc(N * 8, st) || dh.alloc(nint * 8, st) || da.alloc(n * 8, st) ||
      db.alloc(n * 8, st) || dkey.alloc(n * 4, st) || didx.alloc(n * 4, st) || dkey2.alloc(n * 4, st) ||
      didx2.alloc(n * 4, st) || dstart.alloc(ncell * 4, st) || dbad.alloc(16, st)) {
    err = "device allocation failed while loading points";
    return MIPWA_E_NOMEM;
  }
  LCHK(hipMemcpyAsync(d12.p, s12, n * 8, hipMemcpyHostToDevice, st), "upload of s12 failed");
  LCHK(hipMemcpyAsync(d13.p, s13, n * 8, hipMemcpyHostToDevice, st), "upload of s13 failed");
  if (kind == 1) LCHK(hipMemcpyAsync(dw.p, w, n * 8, hipMemcpyHostToDevice, st), "upload of weights failed");
  if (eff) LCHK(hipMemcpyAsync(deff.p, eff, n * 8, hipMemcpyHostToDevice, st), "upload of efficiencies failed");
  LCHK(hipMemcpyAsync(dkn.p, mh.knots.data(), N * 8, hipMemcpyHostToDevice, st), "upload of knots failed");
  LCHK(hipMemcpyAsync(dh.p, mh.h.data(), nint * 8, hipMemcpyHostToDevice, st), "upload of knot spacings failed");
  const unsigned long long none[2] = {~0ull, ~0ull};
  LCHK(hipMemcpyAsync(dbad.p, none, 16, hipMemcpyHostToDevice, st), "flag upload failed");
  LCHK(hipMemsetAsync(dstart.p, 0xff, ncell * 4, st), "cell start reset failed");
  const RegionArgs g{mh.M, mh.m1, mh.m2, mh.m3, mh.smin(), mh.smax(), 1e-9 * mh.smax()};
  k_prepare<<<grid_for(n), 256, 0, st>>>(d12.as<double>(), d13.as<double>(), kind == 1 ? dw.as<double>() : nullptr,
                                         eff ? deff.as<double>() : nullptr, n, dkn.as<double>(), N, g, da.as<double>(),
                                         db.as<double>(), dkey.as<unsigned>(), didx.as<unsigned>(),
                                         dbad.as<unsigned long long>());
  LCHK(hipGetLastError(), "point preparation kernel failed");
  unsigned long long bad[2] = {0, 0};
  LCHK(hipMemcpyAsync(bad, dbad.p, 16, hipMemcpyDeviceToHost, st), "flag download failed");
  LCHK(hipStreamSynchronize(st), "point preparation failed");
  if (bad[0] != none[0]) {
    const long long i = (long long)bad[0];
    if (kind == 1 && std::isfinite(s12[i]) && std::isfinite(s13[i]) && mh.inside(s12[i], s13[i], 1e-9 * mh.smax()) &&
        !(w[i] > 0 && std::isfinite(w[i])))
      err = "weight " + std::to_string(i) + " must be positive and finite";
    else
      err = "point " + std::to_string(i) + " (" + std::to_string(s12[i]) + ", " + std::to_string(s13[i]) +
            ") is outside the Dalitz region";
    return MIPWA_E_INVAL;
  }
  if (bad[1] != none[1]) {
    err = "efficiency " + std::to_string((long long)bad[1]) + " must be positive and finite";
    return MIPWA_E_INVAL;
  }
  // efficiency: given, or looked up in the table at the points as given (not the swapped coordinates)
  const double* d_eps = eff ? deff.as<double>() : nullptr;
  StreamBuf dlook(pool);
  if (!eff && et.set()) {
    if (dlook.alloc(n * 8, st)) {
      err = "device allocation failed for the efficiency lookup";
      return MIPWA_E_NOMEM;
    }
    LCHK(launch_eff_lookup(d12.as<double>(), d13.as<double>(), n, et.d.as<float>(), et.nx, et.ny, et.lo, et.hi,
                           dlook.as<double>(), st),
         "efficiency lookup on the device failed");
    d_eps = dlook.as<double>();
  }
  // stable sort of (cell, index) by cell
  int end_bit = 1;
  while ((1ull << end_bit) < ncell) ++end_bit;
  size_t temp = 0;
  LCHK(rocprim::radix_sort_pairs(nullptr, temp, dkey.as<unsigned>(), dkey2.as<unsigned>(), didx.as<unsigned>(),
                                 didx2.as<unsigned>(), (size_t)n, 0, end_bit, st),
       "sort setup failed");
  StreamBuf dtemp(pool);
  if (dtemp.alloc(temp, st)) {
    err = "device allocation failed for the sort";
    return MIPWA_E_NOMEM;
  }
  LCHK(rocprim::radix_sort_pairs(dtemp.p, temp, dkey.as<unsigned>(), dkey2.as<unsigned>(), didx.as<unsigned>(),
                                 didx2.as<unsigned>(), (size_t)n, 0, end_bit, st),
       "sort of points by cell failed");
  k_cell_starts<<<grid_for(n), 256, 0, st>>>(dkey2.as<unsigned>(), n, dstart.as<int>());
  LCHK(hipGetLastError(), "cell start kernel failed");
  // point arrays in sorted order
  const size_t real = fp64 ? 8 : 4;
  if (ps.tt.alloc_from(2 * n * real, pool, st, free_st) || ps.ss.alloc_from(2 * n * 8, pool, st, free_st) ||
      ps.cache.alloc_from((size_t)std::max(mh.R, 1) * 2 * n * real, pool, st, free_st) ||
      (kind == 1 &&
       (ps.w.alloc_from(n * real, pool, st, free_st) || ps.wplain.alloc_from(n * real, pool, st, free_st)))) {
    err = "device allocation failed for points";
    return MIPWA_E_NOMEM;
  }
  if (fp64)
    k_gather<double><<<grid_for(n), 256, 0, st>>>(dkey2.as<unsigned>(), didx2.as<unsigned>(), da.as<double>(),
                                                   db.as<double>(), kind == 1 ? dw.as<double>() : nullptr, d_eps, n,
                                                   dkn.as<double>(), dh.as<double>(), nint, ps.tt.as<double>(),
                                                   ps.ss.as<double>(), ps.w.as<double>(), ps.wplain.as<double>());
  else
    k_gather<float><<<grid_for(n), 256, 0, st>>>(dkey2.as<unsigned>(), didx2.as<unsigned>(), da.as<double>(),
                                                  db.as<double>(), kind == 1 ? dw.as<double>() : nullptr, d_eps, n,
                                                  dkn.as<double>(), dh.as<double>(), nint, ps.tt.as<float>(),
                                                  ps.ss.as<double>(), ps.w.as<float>(), ps.wplain.as<float>());
  LCHK(hipGetLastError(), "gather kernel failed");
  std::vector<int> starts(ncell);
  LCHK(hipMemcpyAsync(starts.data(), dstart.p, ncell * 4, hipMemcpyDeviceToHost, st), "cell start download failed");
  // events: c_eps = -2 sum ln eff over the events (efficiencies given or looked up)
  std::vector<double> eps_host;
  if (kind == 0 && !eff && d_eps) {
    eps_host.resize(n);
    LCHK(hipMemcpyAsync(eps_host.data(), d_eps, n * 8, hipMemcpyDeviceToHost, st), "efficiency download failed");
  }
  LCHK(hipStreamSynchronize(st), "loading points failed");
  double c_eps = 0.0;
  if (kind == 0) {
    const double* e = eff ? eff : (eps_host.empty() ? nullptr : eps_host.data());
    if (e)
      for (long long i = 0; i < n; ++i) c_eps += -2.0 * std::log(e[i]);
  }
  // tiles of <= kTile points within each cell, and the cells that hold points
  // a cell's points end where the next occupied cell's begin
  std::vector<long long> ends(ncell, 0);
  for (long long c = (long long)ncell - 1, next = n; c >= 0; --c)
    if (starts[c] >= 0) {
      ends[c] = next;
      next = starts[c];
    }
  std::vector<Tile> tiles, cells;
  tiles.reserve(n / kTile + ncell);
  for (size_t c = 0; c < ncell; ++c) {
    if (starts[c] < 0) continue;
    const long long lo = starts[c], hi = ends[c];
    cells.push_back(Tile{(int)(c / nint), (int)(c % nint), (int)tiles.size(), 0});
    for (long long t = lo; t < hi; t += kTile)
      tiles.push_back(Tile{(int)(c / nint), (int)(c % nint), (int)t, (int)std::min<long long>(kTile, hi - t)});
    cells.back().count = (int)tiles.size() - cells.back().start;
  }
  if (ps.tiles.alloc_from(tiles.size() * sizeof(Tile), pool, st, free_st) ||
      ps.cells.alloc_from(std::max<size_t>(cells.size(), 1) * sizeof(Tile), pool, st, free_st)) {
    err = "device allocation failed for tiles";
    return MIPWA_E_NOMEM;
  }
  LCHK(hipMemcpyAsync(ps.tiles.p, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, st),
       "copy of tiles failed");
  LCHK(hipMemcpyAsync(ps.cells.p, cells.data(), cells.size() * sizeof(Tile), hipMemcpyHostToDevice, st),
       "upload of the cell list failed");
  LCHK(hipStreamSynchronize(st), "upload of the tiles failed");
  if (kind == 0) {
    ps.w.release();
    ps.wplain.release();
  }
  ps.n = n;
  ps.n_tiles = (int)tiles.size();
  ps.n_cells = (int)cells.size();
  ps.c_eps = c_eps;
  ps.loaded = true;
  return MIPWA_OK;
}

}  // namespace mipwa
