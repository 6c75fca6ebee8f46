// Host-side FP64 pieces of the library: spline setup, resonance constants, point loading, and the
// context that owns every device buffer.  Internal; the public boundary is include/mipwa.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "engine.h"
#include "mipwa.h"

namespace mipwa {

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  // memory from a stream-ordered pool: released by a free in the order of free_st, which, unlike a
  // plain free, does not wait for the whole device
  hipMemPool_t pool = nullptr;
  hipStream_t free_st = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), pool(o.pool), free_st(o.free_st) {
    o.p = nullptr;
    o.bytes = 0;
    o.pool = nullptr;
    o.free_st = nullptr;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      pool = o.pool;
      free_st = o.free_st;
      o.p = nullptr;
      o.bytes = 0;
      o.pool = nullptr;
      o.free_st = nullptr;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)(pool ? hipFreeAsync(p, free_st) : hipFree(p));
    p = nullptr;
    bytes = 0;
    pool = nullptr;
    free_st = nullptr;
  }
  hipError_t alloc(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, n ? n : 16);
    if (e == hipSuccess) bytes = n;
    else p = nullptr;
    return e;
  }
  // from `pl` in the order of stream `st` (a plain allocation when pl is null); the memory is later
  // freed in the order of `fst`
  hipError_t alloc_from(size_t n, hipMemPool_t pl, hipStream_t st, hipStream_t fst) {
    if (!pl) return alloc(n);
    release();
    hipError_t e = hipMallocFromPoolAsync(&p, n ? n : 16, pl, st);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = n;
    pool = pl;
    free_st = fst;
    return hipSuccess;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// Pinned host allocation; a mapped, coherent one also has a device address (dev).
struct HostBuf {
  void* p = nullptr;
  void* dev = nullptr;
  size_t bytes = 0;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = dev = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t n, bool mapped_coherent = false) {
    if (n <= bytes && p && (dev || !mapped_coherent)) return hipSuccess;
    release();
    hipError_t e = hipHostMalloc(&p, n ? n : 16,
                                 mapped_coherent ? (hipHostMallocMapped | hipHostMallocCoherent) : hipHostMallocDefault);
    if (e == hipSuccess && mapped_coherent) e = hipHostGetDevicePointer(&dev, p, 0);
    if (e == hipSuccess) {
      bytes = n;
    } else {
      if (p) (void)hipHostFree(p);
      p = dev = nullptr;
    }
    return e;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// The static part of a model: kinematics, knots, resonances and the factorised spline operator.
struct ModelHost {
  double M = 0, m1 = 0, m2 = 0, m3 = 0, rD = 0;
  std::vector<double> knots, h;  // N knots, N-1 interval lengths
  std::vector<mipwa_res> res;
  int N = 0, R = 0, P = 0;
  std::vector<double> th_c;      // Thomas factors (interior unknowns)
  std::vector<double> th_d;
  std::vector<double> inv_h, inv_d;  // 1/h and 1/th_d: the per-evaluation staging multiplies
  Kin<double> kin64{};
  Kin<float> kin32{};

  int init(const mipwa_model* m, std::string& err);
  double smin() const { return (m1 + m2) * (m1 + m2); }
  double smax() const { return (M - m3) * (M - m3); }
  // second derivatives M (complex, as re/im arrays) from knot values z
  void second_derivs(const double* zr, const double* zi, double* Mr, double* Mi) const;
  // spline polynomial coefficients per interval: 8 doubles (P0..P3 re/im) per interval
  void poly_table(const double* theta, double* out) const;
  // per-resonance constants (kResWords doubles each) at the given masses/widths in theta
  void res_table(const double* theta, double* out) const;
  // the evaluation table at theta in the working precision: table_real_words(N - 1, R, fp64) words
  // (doubles, or floats followed by their residues; zeros in place of the residues when `residues` is
  // false) at out
  void eval_table(const double* theta, bool fp64, void* out, bool residues = true) const;
  // FP64 resonance constants at theta into a device buffer (synchronous; the copy is made in the
  // order of stream st when one is given, for memory allocated in that order)
  int upload_res64(const double* theta, DevBuf& d, hipStream_t st = nullptr) const;
  int interval(double s) const;
  bool inside(double s12, double s13, double tol) const;
  int check_theta(const double* theta, std::string& err) const;
};

struct PointSet {
  long long n = 0;
  int n_tiles = 0;
  int n_cells = 0;          // spline cells (j12, j13) holding points: Tile{j12, j13, first tile, tiles}
  DevBuf tt, ss, w, wplain, cache, tiles, cells;
  double c_eps = 0.0;       // -2 sum ln eff (events)
  bool loaded = false;
};

// Load host points into a point set, on the device: validate, swap each pair to s12 <= s13, locate
// the spline cells, stable sort by cell, compute local coordinates in FP64; the host cuts the tiles.
// When no eff array is given and a table is set, eff is looked up on the device.
struct EffTable {
  std::vector<float> tab;
  int nx = 0, ny = 0;
  double lo = 0, hi = 0;
  DevBuf d;
  bool set() const { return nx > 0; }
};

// With a pool, the point set's memory and the scratch of the load come from it in the order of st,
// and the point set's memory is freed in the order of free_st.
int load_points(const ModelHost& mh, bool fp64, int kind, const double* s12, const double* s13, const double* w,
                const double* eff, long long n, const EffTable& et, hipStream_t st, PointSet& ps,
                std::string& err, hipMemPool_t pool = nullptr, hipStream_t free_st = nullptr);

}  // namespace mipwa
