// gfx950 kernels of the MIPWA likelihood.
//
// What is computed (see include/mipwa.h for the method and its readings):
//   A(s12,s13) = S(s12) + S(s13) + sum_r c_r R_r(s12,s13)            (Sec. 2 Eq. 1, Sec. 4 symmetrisation)
//   data:  sum ln|A|^2 and the adjoint seed g = -4 A/|A|^2
//   norm:  sum w eff |A|^2 and the seed g = 4 w eff A (scaled by n/I in the finish)
//   adjoint: per spline interval j and power m, sum g t^m; per resonance sum g conj(R_r) and, when
//   masses/widths float, sum g conj(dR_r/dm), sum g conj(dR_r/dGamma).
//
// Layout: points are sorted at load time by spline cell (j12, j13) and cut into tiles of at most kTile
// points of one cell, so the interval indices and the spline polynomials are wave-uniform (scalar
// registers).  Point streams are SoA pairs (t12,t13), (s12,s13), w, and one complex plane per
// resonance, read coalesced.  Each wave owns a contiguous range of tiles, keeps its adjoint partials
// in registers while the cell does not change, and folds them into a wave-private LDS histogram of
// spline intervals when it does.  Blocks write fixed-size FP64 records; two more kernels reduce them
// in a fixed order (bitwise reproducible): group sums of 32 records, then one block per job that sums
// the groups and runs the FP64 finish.
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "engine.h"

namespace mipwa {

template <typename Real>
struct Ops;

template <>
struct Ops<float> {
  using V2 = float2;
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
  static __device__ __forceinline__ float log(float x) { return __logf(x); }
  // a wave-uniform value held in a scalar register
  static __device__ __forceinline__ float uniform(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
  }
};

template <>
struct Ops<double> {
  using V2 = double2;
  static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
  static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double rsqrt(double x) { return ::rsqrt(x); }
  static __device__ __forceinline__ double log(double x) { return ::log(x); }
  static __device__ __forceinline__ double uniform(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
  }
};

// Pointers into device memory that the compiler may treat as global (not generic) addresses: loads
// then take a wave-uniform base in scalar registers plus a 32-bit lane offset.
#define MIPWA_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const MIPWA_GLOBAL T* global_ptr(const T* p) {
  return (const MIPWA_GLOBAL T*)p;
}

// Streaming load of a point's data.  The weights and every FP64 element carry the non-temporal hint:
// each point is read once per evaluation and a point set is larger than the caches.  The FP32
// coordinate and amplitude pairs (float2) do not: the mixed-precision sweep alternates its part order
// between evaluations so that the part read last is read first next time, from the Infinity Cache,
// which non-temporal lines do not stay in (headline mixed: 97 us plain, 102 us with the hint on these
// loads; the weights' hint is neutral).
template <typename T>
__device__ __forceinline__ T nt_load(const MIPWA_GLOBAL T* p) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "4-, 8- or 16-byte element");
  if constexpr (std::is_same_v<T, float2>) {
    return __builtin_bit_cast(T, *(const MIPWA_GLOBAL unsigned long long*)p);
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_nontemporal_load((const MIPWA_GLOBAL unsigned*)p));
  } else if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_nontemporal_load((const MIPWA_GLOBAL unsigned long long*)p));
  } else {
    using U4v = unsigned __attribute__((ext_vector_type(4)));
    return __builtin_bit_cast(T, __builtin_nontemporal_load((const MIPWA_GLOBAL U4v*)p));
  }
}

// A pointer or count that is the same for the whole wave, held in scalar registers.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ long long uniform_ll(long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)x);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// Tile descriptors through the constant address space, so that a wave-uniform index becomes a scalar load.
using ConstTiles = const __attribute__((address_space(4))) Tile*;

__device__ __forceinline__ Tile load_tile(ConstTiles tiles, int i) {
  return Tile{tiles[i].j12, tiles[i].j13, tiles[i].start, tiles[i].count};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Breit-Wigner amplitudes of all R resonances for one pairing: x is the resonant h-h+ invariant, y
// the other one (Sec. 2: relativistic Breit-Wigner times a real angular factor; the readings are the
// running width with Blatt-Weisskopf factors and Zemach tensors).  With the per-resonance constants
// kappa = sqrt(N_L(z_qr) N_L(z_pr)) and delta = Gamma_r m_r^2 N_L(z_qr) / q_r^(2L+1):
//   BW = kappa f(x) T_L(x,y) / (m_r^2 - x - i delta u(x)),
//   f = 1/sqrt(N_L(rho^2 q^2) N_L(rD^2 p^2)),  u = q^(2L+1) / (sqrt(x) N_L(rho^2 q^2)),
// which is B_L(q) B_L(p) T_L / (m_r^2 - x - i m_r Gamma(x)).  The mass and width partials are
//   dBW/dm = dln kappa/dm BW - 2 m_r E + i (ddelta/dm) F,   dBW/dGamma = i (ddelta/dGamma) F,
// with E = BW / D and F = u BW / D.  The constants are per resonance, so with DER the pairing adds
// E and F to (er, ei) and (fr, fi) and the constants are applied once to the reduced sums.
template <typename Real, int R, bool DER>
__device__ __forceinline__ void bw_pairing(const Kin<Real>& k, const Real* __restrict__ res, Real x, Real y,
                                           Real* br, Real* bi, Real* er, Real* ei, Real* fr, Real* fi) {
  using O = Ops<Real>;
  // FP32: one reciprocal square root gives both 1/x and sqrt(x) (a quarter-rate operation fewer);
  // FP64 keeps the correctly rounded division and root
  Real ix, sx, isx = Real(0);
  if constexpr (sizeof(Real) == 4) {
    isx = O::rsqrt(x);
    sx = x * isx;
    ix = isx * isx;
  } else {
    ix = O::rcp(x);
    sx = O::sqrt(x);
  }
  Real q2 = (x - k.thr_hi) * (x - k.thr_lo) * (Real(0.25) * ix);
  Real p2 = (x - k.pb_hi) * (x - k.pb_lo) * (Real(0.25) * ix);
  q2 = q2 > Real(0) ? q2 : Real(0);
  p2 = p2 > Real(0) ? p2 : Real(0);
  const Real q = O::sqrt(q2);
  const Real t1 = k.sum - x - y - y + k.t1corr * ix;
  const Real t2 = t1 * t1 - (x - k.t2a + k.t2b * ix) * (x - k.t2c + k.t2d * ix) * Real(1.0 / 3.0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const Real* c = res + r * kResWords;
    const Real m2 = c[0], kappa = c[1], delta = c[2], rho2 = c[3];
    const int L = (int)c[4];
    const Real zq = rho2 * q2, zp = k.rD2 * p2;
    Real nq, np, qp, T;
    if (L == 1) {
      nq = Real(1) + zq;
      np = Real(1) + zp;
      qp = q2 * q;
      T = t1;
    } else if (L == 2) {
      nq = (zq + Real(3)) * zq + Real(9);
      np = (zp + Real(3)) * zp + Real(9);
      qp = q2 * q2 * q;
      T = t2;
    } else {
      nq = Real(1);
      np = Real(1);
      qp = q;
      T = Real(1);
    }
    const Real f = O::rsqrt(nq * np);
    // u = q^(2L+1) / (sqrt(x) N_L(q)); in FP32 1/N_L(q) = f^2 N_L(p) saves the reciprocal
    Real u;
    if constexpr (sizeof(Real) == 4) u = qp * isx * (f * f * np);
    else u = qp * O::rcp(sx * nq);
    const Real dre = m2 - x, dim = -delta * u;
    const Real idd = O::rcp(dre * dre + dim * dim);
    const Real num = kappa * f * T * idd;
    const Real vr = num * dre, vi = -num * dim;
    br[r] += vr;
    bi[r] += vi;
    if constexpr (DER) {
      const Real ire = dre * idd, iim = -dim * idd;  // 1/D
      const Real wr = vr * ire - vi * iim, wi = vr * iim + vi * ire;  // E = BW / D
      er[r] += wr;
      ei[r] += wi;
      fr[r] += u * wr;
      fi[r] += u * wi;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// K1: symmetrised resonance amplitudes R_r = BW_r(s12,s13) + BW_r(s13,s12) at every point.

// Computed in FP64 from the FP64 coordinates in both precisions and rounded once when stored (the cache
// is rebuilt only when a mass or width changes, so its cost does not enter an evaluation; FP64 keeps
// m_r^2 - x accurate next to narrow poles).
template <typename Real, int R>
__global__ __launch_bounds__(256) void k_cache(Segment sg, const double* __restrict__ res, Kin<double> kin) {
  using V2 = typename Ops<Real>::V2;
  constexpr int R1 = R > 0 ? R : 1;
  const double2* __restrict__ ss = (const double2*)sg.ss;
  V2* __restrict__ cache = (V2*)sg.cache;
  const long long n = sg.n;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const double2 s = ss[p];
    double br[R1] = {}, bi[R1] = {};
    bw_pairing<double, R, false>(kin, res, s.x, s.y, br, bi, nullptr, nullptr, nullptr, nullptr);
    bw_pairing<double, R, false>(kin, res, s.y, s.x, br, bi, nullptr, nullptr, nullptr, nullptr);
#pragma unroll
    for (int r = 0; r < R; ++r) cache[(long long)r * n + p] = V2{(Real)br[r], (Real)bi[r]};
  }
}

// ---------------------------------------------------------------------------------------------
// K2: fused forward + adjoint over the tiles of one segment, persistent waves.

// bins: this wave's `parts` interval histograms, stride doubles apart; scal: its `parts` sets of nsc
// scalars.  order 0 / 1: the parts of the wave's tile range are swept in ascending / descending order.
template <typename Real, int R, bool OTF, int KIND>
__device__ __forceinline__ void run_segment(const Segment& sg, const Kin<Real>& kin, const Real* tab, double* bins,
                                            double* scal, int wave, int lane, int waves, int local_block, int stride,
                                            int parts, int order) {
  using O = Ops<Real>;
  using V2 = typename O::V2;
  constexpr int R1 = R > 0 ? R : 1;
  constexpr int IT = kTile / 64;
  const Real* __restrict__ cv = tab + 8 * sg.nint;
  const Real* __restrict__ res = cv + 2 * R;
  // FP32: the residues of P_0, P_1 and c_r follow the table (zeros when the host gives none); the
  // floated-shape sweep, bound by the vector ALU, leaves them out
  constexpr bool kLo = sizeof(Real) < sizeof(double) && !OTF;
  const Real* __restrict__ lo = tab + table_words(sg.nint, R);
  Real cre[R1], cim[R1], cre_lo[R1], cim_lo[R1];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    cre[r] = O::uniform(cv[2 * r]);
    cim[r] = O::uniform(cv[2 * r + 1]);
    cre_lo[r] = kLo ? O::uniform(lo[4 * sg.nint + 2 * r]) : Real(0);
    cim_lo[r] = kLo ? O::uniform(lo[4 * sg.nint + 2 * r + 1]) : Real(0);
  }
  const V2* __restrict__ tt = uniform_ptr((const V2*)sg.tt);
  const double2* __restrict__ ss = uniform_ptr((const double2*)sg.ss);
  const Real* __restrict__ ww = uniform_ptr((const Real*)sg.w);
  const V2* __restrict__ cache = uniform_ptr((const V2*)sg.cache);
  const long long n = uniform_ll(sg.n);

  const long long nw = (long long)sg.n_blocks * waves;
  const long long gw = (long long)local_block * waves + wave;
  const int t0 = (int)(sg.n_tiles * gw / nw);
  const int t1 = (int)(sg.n_tiles * (gw + 1) / nw);

  double q12[8], q13[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) q12[m] = q13[m] = 0.0;
  double acc = 0.0;
  double agc[2 * R1], ahm[2 * R1], ahg[2 * R1];
#pragma unroll
  for (int r = 0; r < 2 * R1; ++r) agc[r] = ahm[r] = ahg[r] = 0.0;

  // FP32 streams: per-tile partial sums in FP32, folded into the FP64 accumulators once per tile.
  // FP64 streams: the "tile" arrays are the accumulators themselves (never folded per tile).
  constexpr bool kTilePartial = sizeof(Real) < sizeof(double);
  Real tq12[8], tq13[8], tgc[2 * R1], thm[2 * R1], thg[2 * R1];
  Real tacc = Real(0);
#pragma unroll
  for (int m = 0; m < 8; ++m) tq12[m] = tq13[m] = Real(0);
#pragma unroll
  for (int r = 0; r < 2 * R1; ++r) tgc[r] = thm[r] = thg[r] = Real(0);

  int cj12 = -1, cj13 = -1;
  // e: residues of P_1 (elements 2, 3) of the two intervals, e0: the sum of their P_0 residues
  Real p12[8], p13[8], e12[4], e13[4], e0r = Real(0), e0i = Real(0);
#pragma unroll
  for (int m = 0; m < 8; ++m) p12[m] = p13[m] = Real(0);
#pragma unroll
  for (int m = 0; m < 4; ++m) e12[m] = e13[m] = Real(0);
  double* hb = bins;  // interval histogram of the part being swept

  auto flush = [&]() {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      double u = q12[m], v = q13[m];
      if constexpr (!kTilePartial) {
        u += (double)tq12[m];
        v += (double)tq13[m];
        tq12[m] = tq13[m] = Real(0);
      }
      const double a = wave_sum(u);
      const double b = wave_sum(v);
      q12[m] = 0.0;
      q13[m] = 0.0;
      if (lane == 0) {
        hb[8 * cj12 + m] += a;
        hb[8 * cj13 + m] += b;
      }
    }
  };

  // One point: both spline axes, the resonance terms, |A|^2, the seed g of the adjoint, and its
  // products with the spline powers and the resonance amplitudes (and, on the fly, with the sums E
  // and F of the mass and width partials).  Invalid lanes contribute zero.
  auto accumulate = [&](Real x12, Real x13, const Real* rr, const Real* ri, const Real* er, const Real* ei,
                        const Real* fr, const Real* fi, Real wv, bool valid) {
    Real ar = p12[0] + x12 * (p12[2] + x12 * (p12[4] + x12 * p12[6]));
    Real ai = p12[1] + x12 * (p12[3] + x12 * (p12[5] + x12 * p12[7]));
    ar += p13[0] + x13 * (p13[2] + x13 * (p13[4] + x13 * p13[6]));
    ai += p13[1] + x13 * (p13[3] + x13 * (p13[5] + x13 * p13[7]));
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ar += cre[r] * rr[r] - cim[r] * ri[r];
      ai += cre[r] * ri[r] + cim[r] * rr[r];
    }
    if constexpr (kLo) {
      // the residue terms, all small, summed among themselves and then added once
      Real dr = e0r + x12 * e12[2] + x13 * e13[2];
      Real di = e0i + x12 * e12[3] + x13 * e13[3];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        dr += cre_lo[r] * rr[r] - cim_lo[r] * ri[r];
        di += cre_lo[r] * ri[r] + cim_lo[r] * rr[r];
      }
      ar += dr;
      ai += di;
    }
    const Real a2 = ar * ar + ai * ai;
    Real gr, gi;
    if constexpr (KIND == 0) {
      const Real l = O::log(a2);
      tacc += valid ? l : Real(0);
      const Real sc = valid ? Real(-4) * O::rcp(a2) : Real(0);
      gr = sc * ar;
      gi = sc * ai;
    } else {
      const Real w = valid ? wv : Real(0);
      tacc += w * a2;
      gr = Real(4) * w * ar;
      gi = Real(4) * w * ai;
    }
    {
      const Real x = x12, x2 = x * x, x3 = x2 * x;
      tq12[0] += gr;
      tq12[1] += gi;
      tq12[2] += gr * x;
      tq12[3] += gi * x;
      tq12[4] += gr * x2;
      tq12[5] += gi * x2;
      tq12[6] += gr * x3;
      tq12[7] += gi * x3;
    }
    {
      const Real x = x13, x2 = x * x, x3 = x2 * x;
      tq13[0] += gr;
      tq13[1] += gi;
      tq13[2] += gr * x;
      tq13[3] += gi * x;
      tq13[4] += gr * x2;
      tq13[5] += gi * x2;
      tq13[6] += gr * x3;
      tq13[7] += gi * x3;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      tgc[2 * r] += gr * rr[r] + gi * ri[r];
      tgc[2 * r + 1] += gi * rr[r] - gr * ri[r];
      if constexpr (OTF) {
        thm[2 * r] += gr * er[r] + gi * ei[r];
        thm[2 * r + 1] += gi * er[r] - gr * ei[r];
        thg[2 * r] += gr * fr[r] + gi * fi[r];
        thg[2 * r + 1] += gi * fr[r] - gr * fi[r];
      }
    }
  };
  auto enter_cell = [&](int j12, int j13) {
    if (j12 != cj12 || j13 != cj13) {
      if (cj12 >= 0) flush();
      cj12 = j12;
      cj13 = j13;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        p12[m] = O::uniform(tab[8 * cj12 + m]);
        p13[m] = O::uniform(tab[8 * cj13 + m]);
      }
      if constexpr (kLo) {
#pragma unroll
        for (int m = 2; m < 4; ++m) {
          e12[m] = O::uniform(lo[4 * cj12 + m]);
          e13[m] = O::uniform(lo[4 * cj13 + m]);
        }
        e0r = O::uniform(lo[4 * cj12] + lo[4 * cj13]);
        e0i = O::uniform(lo[4 * cj12 + 1] + lo[4 * cj13 + 1]);
      }
    }
  };
  auto fold_tile = [&]() {
    if constexpr (kTilePartial) {
      acc += (double)tacc;
      tacc = Real(0);
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        q12[m] += (double)tq12[m];
        q13[m] += (double)tq13[m];
        tq12[m] = tq13[m] = Real(0);
      }
#pragma unroll
      for (int r = 0; r < 2 * R; ++r) {
        agc[r] += (double)tgc[r];
        tgc[r] = Real(0);
        if constexpr (OTF) {
          ahm[r] += (double)thm[r];
          ahg[r] += (double)thg[r];
          thm[r] = thg[r] = Real(0);
        }
      }
    }
  };

  // Closes the sweep of part h of the wave's tiles: flushes the cell in progress, folds the running
  // sums of the FP64 streams, and stores the wave's reduced scalars in slot h; the accumulators start
  // again from zero.
  const int nsc = 1 + 2 * R + (OTF ? 4 * R : 0);
  auto end_half = [&](int h) {
    if constexpr (!kTilePartial) {
      acc += (double)tacc;
      tacc = Real(0);
#pragma unroll
      for (int r = 0; r < 2 * R; ++r) {
        agc[r] += (double)tgc[r];
        tgc[r] = Real(0);
        if constexpr (OTF) {
          ahm[r] += (double)thm[r];
          ahg[r] += (double)thg[r];
          thm[r] = thg[r] = Real(0);
        }
      }
    }
    if (cj12 >= 0) flush();
    cj12 = cj13 = -1;
    if constexpr (OTF) {
      // g conj(dR/dm) = dlk g conj(R) - 2 m g conj(E) - i ddm g conj(F),  g conj(dR/dGamma) = -i ddg g conj(F)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const Real* c = res + r * kResWords;
        const double m2 = 2.0 * (double)c[5], dlk = (double)c[6], ddm = (double)c[7], ddg = (double)c[8];
        const double er = ahm[2 * r], ei = ahm[2 * r + 1], fr = ahg[2 * r], fi = ahg[2 * r + 1];
        ahm[2 * r] = dlk * agc[2 * r] - m2 * er + ddm * fi;
        ahm[2 * r + 1] = dlk * agc[2 * r + 1] - m2 * ei - ddm * fr;
        ahg[2 * r] = ddg * fi;
        ahg[2 * r + 1] = -ddg * fr;
      }
    }
    double* my = scal + h * nsc;
    {
      const double v = wave_sum(acc);
      if (lane == 0) my[0] = v;
      acc = 0.0;
    }
#pragma unroll
    for (int r = 0; r < 2 * R; ++r) {
      const double v = wave_sum(agc[r]);
      if (lane == 0) my[1 + r] = v;
      agc[r] = 0.0;
      if constexpr (OTF) {
        const double a = wave_sum(ahm[r]);
        const double b = wave_sum(ahg[r]);
        if (lane == 0) {
          my[1 + 2 * R + r] = a;
          my[1 + 4 * R + r] = b;
        }
        ahm[r] = ahg[r] = 0.0;
      }
    }
  };

  if constexpr (!OTF) {
    // Cached amplitudes: the sweep is bound by HBM reads (non-temporal loads), so every step keeps
    // loads in flight.  A tile is taken in two halves of HB points per lane; the loads of the next
    // half (the second half of this tile, then the first half of the next tile) are issued before
    // the current half is used, and the next tile's descriptor is requested a tile ahead.  Lanes past
    // the tile end re-read its last point and contribute zero.
    constexpr int HB = IT / 2;
    static_assert(IT % 2 == 0, "a tile holds an even number of wave-widths");
    struct Half {
      V2 t[HB];
      V2 r[HB][R1];
      Real w[HB];
    };
    // the tile's base addresses are wave-uniform (scalar registers); lanes add a 32-bit offset
    auto load_half = [&](Half& h, const Tile& td, int part) {
      const MIPWA_GLOBAL V2* tb = global_ptr(tt + td.start);
      const MIPWA_GLOBAL Real* wb = global_ptr(ww + td.start);
#pragma unroll
      for (int k = 0; k < HB; ++k) {
        const int i = (part * HB + k) * 64 + lane;
        // offset within the tile (count >= 1), bounded so that it fits a 32-bit lane offset
        static_assert((kTile & (kTile - 1)) == 0, "the tile size is a power of two");
        const unsigned j = (unsigned)(i < td.count ? i : td.count - 1) & (unsigned)(kTile - 1);
        h.t[k] = nt_load(tb + j);
#pragma unroll
        for (int r = 0; r < R; ++r) h.r[k][r] = nt_load(global_ptr(cache + ((long long)r * n + td.start)) + j);
        if constexpr (KIND == 1) h.w[k] = nt_load(wb + j);
      }
    };
    auto use_half = [&](const Half& h, const Tile& td, int part) {
#pragma unroll
      for (int k = 0; k < HB; ++k) {
        Real rr[R1], ri[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) {
          rr[r] = r < R ? h.r[k][r].x : Real(0);
          ri[r] = r < R ? h.r[k][r].y : Real(0);
        }
        const bool valid = (part * HB + k) * 64 + lane < td.count;
        accumulate(h.t[k].x, h.t[k].y, rr, ri, nullptr, nullptr, nullptr, nullptr, KIND == 1 ? h.w[k] : Real(0),
                   valid);
      }
    };
    // The wave's tiles are swept as `parts` equal consecutive parts, each with its own accumulators and
    // interval histogram, combined in a fixed order at the end: the result does not depend on the
    // order the parts are taken in.  Consecutive evaluations alternate ascending and descending part
    // order, so each starts on the parts the previous one read last, while they are still in the
    // Infinity Cache.
    auto sweep = [&](int a0, int a1) {
      if (a0 >= a1) return;
      Half a, b;
      const ConstTiles tiles = (ConstTiles)uniform_ptr(sg.tiles);
      Tile td = load_tile(tiles, a0);
      load_half(a, td, 0);
#pragma unroll 1
      for (int ti = a0; ti < a1; ++ti) {
        // the next descriptor (clamped to this part's last tile) is requested a tile ahead
        const Tile tn = load_tile(tiles, min(ti + 1, a1 - 1));
        load_half(b, td, 1);
        enter_cell(td.j12, td.j13);
        use_half(a, td, 0);
        if (ti + 1 < a1) load_half(a, tn, 0);
        use_half(b, td, 1);
        fold_tile();
        td = tn;
      }
    };
#pragma unroll 1
    for (int pass = 0; pass < parts; ++pass) {
      const int h = order ? parts - 1 - pass : pass;
      hb = bins + h * stride;
      sweep(t0 + (int)((long long)(t1 - t0) * h / parts), t0 + (int)((long long)(t1 - t0) * (h + 1) / parts));
      end_half(h);
    }
  } else {
    // Shapes floated: amplitudes and their derivatives on the fly.  ALU-bound; one point per lane
    // at a time keeps the register file within one wave's share, and the loads of the next point
    // (the next in this tile, else the first of the next tile, whose descriptor is requested a
    // tile ahead) are issued before the current point is computed.  Lanes past a tile's end
    // re-read its last point and contribute zero.
    if (t0 < t1) {
      auto issue = [&](const Tile& t, int b, V2& tv, double2& sv, Real& wv) {
        const int i = b * 64 + lane;
        const long long p = (long long)t.start + (i < t.count ? i : t.count - 1);
        tv = tt[p];
        sv = ss[p];
        if constexpr (KIND == 1) wv = ww[p];
      };
      Tile td = sg.tiles[t0];
      Tile tn = sg.tiles[min(t0 + 1, t1 - 1)];
      V2 tv;
      double2 sv;
      Real wv = Real(0);
      issue(td, 0, tv, sv, wv);
#pragma unroll 1
      for (int ti = t0; ti < t1; ++ti) {
        enter_cell(td.j12, td.j13);
#pragma unroll 1
        for (int ib = 0; ib < IT; ++ib) {
          const bool valid = ib * 64 + lane < td.count;
          V2 tv2;
          double2 sv2;
          Real wv2 = Real(0);
          if (ib + 1 < IT) issue(td, ib + 1, tv2, sv2, wv2);
          else issue(tn, 0, tv2, sv2, wv2);  // the last tile's own first point when none follows
          Real rr[R1], ri[R1], er[R1], ei[R1], fr[R1], fi[R1];
#pragma unroll
          for (int r = 0; r < R1; ++r) rr[r] = ri[r] = er[r] = ei[r] = fr[r] = fi[r] = Real(0);
          const Real x12s = (Real)sv.x, x13s = (Real)sv.y;
          bw_pairing<Real, R, true>(kin, res, x12s, x13s, rr, ri, er, ei, fr, fi);
          bw_pairing<Real, R, true>(kin, res, x13s, x12s, rr, ri, er, ei, fr, fi);
          accumulate(tv.x, tv.y, rr, ri, er, ei, fr, fi, wv, valid);
          tv = tv2;
          sv = sv2;
          wv = wv2;
        }
        fold_tile();
        td = tn;
        tn = sg.tiles[min(ti + 2, t1 - 1)];
      }
    }
    end_half(0);
  }
}
// ---------------------------------------------------------------------------------------------
// Normalisation as a quadratic form (fixed shapes).  In cell c the amplitude is linear in
// v = (P_0..3 of interval j12, P_0..3 of interval j13, c_1..c_R) with the per-point functions phi of
// the moments, so I_c = sum_p w |phi . v|^2 = sum_ij v_i M_ij conj(v_j) and the complex partials of I
// are 2 (M^T v).  A wave takes a contiguous run of cells; lane l < K forms Y_l = (M^T v)_l, adds
// 4 Y into the interval bins and c_r partials (the form the point sweep uses, seed 4 w A) and
// Re(conj(v_l) Y_l) into I.

template <typename Real, int R>
__device__ void run_qform(const Segment& sg, const Real* tab, double* bins, double* scal, int wave, int lane,
                          int waves, int local_block) {
  constexpr int K = 8 + R;
  const long long nw = (long long)sg.n_blocks * waves;
  const long long gw = (long long)local_block * waves + wave;
  const int c0 = (int)(sg.n_tiles * gw / nw);
  const int c1 = (int)(sg.n_tiles * (gw + 1) / nw);
  const double* __restrict__ mom = (const double*)sg.cache;
  // (the quadratic form is given tables without residues: the data sweep it pairs with must see the
  // same coefficients, and its FP32 arithmetic would keep only part of them)
  const Real* cv = tab + 8 * sg.nint;
  double acc = 0.0, gre = 0.0, gim = 0.0;
  for (int c = c0; c < c1; ++c) {
    const Tile cell = sg.tiles[c];
    double vr[K], vi[K];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      vr[m] = (double)tab[8 * cell.j12 + 2 * m];
      vi[m] = (double)tab[8 * cell.j12 + 2 * m + 1];
      vr[4 + m] = (double)tab[8 * cell.j13 + 2 * m];
      vi[4 + m] = (double)tab[8 * cell.j13 + 2 * m + 1];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      vr[8 + r] = (double)cv[2 * r];
      vi[8 + r] = (double)cv[2 * r + 1];
    }
    double yr = 0.0, yi = 0.0, ur = 0.0, ui = 0.0;
    if (lane < K) {
      const double* Mc = mom + (long long)c * K * K * 2;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const double mr = Mc[2 * (i * K + lane)], mi = Mc[2 * (i * K + lane) + 1];
        yr += mr * vr[i] - mi * vi[i];
        yi += mr * vi[i] + mi * vr[i];
      }
#pragma unroll
      for (int i = 0; i < K; ++i)
        if (i == lane) {
          ur = vr[i];
          ui = vi[i];
        }
      acc += ur * yr + ui * yi;
    }
    // interval bins: the j12 lanes and the j13 lanes in two steps (the same interval when j12 == j13)
    if (lane < 4) {
      bins[8 * cell.j12 + 2 * lane] += 4.0 * yr;
      bins[8 * cell.j12 + 2 * lane + 1] += 4.0 * yi;
    }
    if (lane >= 4 && lane < 8) {
      bins[8 * cell.j13 + 2 * (lane - 4)] += 4.0 * yr;
      bins[8 * cell.j13 + 2 * (lane - 4) + 1] += 4.0 * yi;
    }
    if (lane >= 8 && lane < K) {
      gre += 4.0 * yr;
      gim += 4.0 * yi;
    }
  }
  double* my = scal;  // this wave's first slot
  {
    const double v = wave_sum(acc);
    if (lane == 0) my[0] = v;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double a = wave_sum(lane == 8 + r ? gre : 0.0);
    const double b = wave_sum(lane == 8 + r ? gim : 0.0);
    if (lane == 0) {
      my[1 + 2 * r] = a;
      my[2 + 2 * r] = b;
    }
  }
}

// One block per cell.  The cell's points are contiguous in the sorted arrays; they are taken in
// chunks of kMomChunk: each thread loads one point and writes its K functions phi (complex FP64) to
// LDS, then thread k < K*K forms M[i][j] (i = k / K, j = k % K) over the chunk from LDS, adding the
// points in order.
constexpr int kMomChunk = 256;

template <typename Real, int R>
__global__ __launch_bounds__(kMomChunk) void k_moments(Segment sg, const Tile* __restrict__ cells,
                                                       double* __restrict__ mom) {
  constexpr int K = 8 + R;
  static_assert(K * K <= kMomChunk, "one thread per moment");
  using V2 = typename Ops<Real>::V2;
  __shared__ double2 phi[kMomChunk * K];
  __shared__ double pw[kMomChunk];
  const Tile cell = cells[blockIdx.x];
  const Tile first = sg.tiles[cell.start], last = sg.tiles[cell.start + cell.count - 1];
  const long long p0 = first.start, p1 = (long long)last.start + last.count;
  const V2* __restrict__ tt = (const V2*)sg.tt;
  const Real* __restrict__ ww = (const Real*)sg.w;
  const V2* __restrict__ cache = (const V2*)sg.cache;
  const int k = threadIdx.x;
  const int i = k / K, j = k % K;
  double sr = 0.0, si = 0.0;
  for (long long c0 = p0; c0 < p1; c0 += kMomChunk) {
    const int m = (int)min((long long)kMomChunk, p1 - c0);
    __syncthreads();  // the previous chunk is consumed
    if (k < m) {
      const long long p = c0 + k;
      const V2 x = tt[p];
      const double t12 = (double)x.x, t13 = (double)x.y;
      double2* f = phi + k * K;
      f[0] = double2{1.0, 0.0};
      f[1] = double2{t12, 0.0};
      f[2] = double2{t12 * t12, 0.0};
      f[3] = double2{t12 * t12 * t12, 0.0};
      f[4] = double2{1.0, 0.0};
      f[5] = double2{t13, 0.0};
      f[6] = double2{t13 * t13, 0.0};
      f[7] = double2{t13 * t13 * t13, 0.0};
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const V2 c = cache[(long long)r * sg.n + p];
        f[8 + r] = double2{(double)c.x, (double)c.y};
      }
      pw[k] = (double)ww[p];
    }
    __syncthreads();
    if (k < K * K) {
      // w phi_i conj(phi_j)
      for (int q = 0; q < m; ++q) {
        const double2 a = phi[q * K + i], b = phi[q * K + j];
        const double w = pw[q];
        sr += w * (a.x * b.x + a.y * b.y);
        si += w * (a.y * b.x - a.x * b.y);
      }
    }
  }
  if (k < K * K) {
    double* out = mom + ((long long)blockIdx.x * K * K + k) * 2;
    out[0] = sr;
    out[1] = si;
  }
}

// ---------------------------------------------------------------------------------------------
// FP64 finish of one job, run by the job's block of k_job_finish once its records are reduced:
//   -2 ln L = -2 S_data + C_eps + 2 n ln I,  scale = n / I,
//   spline-polynomial partials -> knot values z and second derivatives M -> z through M = K z,
//   then the chain rule to (a_k, phi_k), (|c_r|, arg c_r), (m_r, Gamma_r).

// fin: the reduced data record followed by the reduced normalisation record (LDS); kc: the job's
// Thomas factors and interval widths staged in LDS (the solve below is a serial chain, so its
// operands must not come from global memory one dependent load at a time); th: the knot and
// coefficient parameters, staged in LDS with them.  The results are gathered in LDS and written out
// by the first wave, which alone then needs a fence before the sequence word is published.
__device__ void finish_job(const Job& jb, const double* fin, const double* kc, const double* th,
                           unsigned long long seq, double* out) {
  const int N = jb.N, nint = N - 1, R = jb.R;
  const double* fd = fin;
  const double* fn = fin + jb.rs;
  const int s0 = 8 * nint;
  const double I = fn[s0];
  const double scale = jb.n_ev / I;
  __shared__ double ob[1 + 2 * kMaxKnots + 4 * kMaxRes];
  const double* thc = kc;                // Thomas factors c'_i of the interior system
  const double* thinv = thc + (N - 2);   // 1 / pivot_i
  const double* h = thinv + (N - 2);
  __shared__ double gy[2 * kMaxKnots], gm[2 * kMaxKnots], u[2 * kMaxKnots];
  // spline-polynomial partials of interval j -> partials of z_j, z_{j+1}, M_j, M_{j+1}
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    double yr = 0, yi = 0, mr = 0, mi = 0;
    if (k < nint) {
      const double* a = fd + 8 * k;
      const double* b = fn + 8 * k;
      const double q0r = a[0] + scale * b[0], q0i = a[1] + scale * b[1];
      const double q1r = a[2] + scale * b[2], q1i = a[3] + scale * b[3];
      const double q2r = a[4] + scale * b[4], q2i = a[5] + scale * b[5];
      const double q3r = a[6] + scale * b[6], q3i = a[7] + scale * b[7];
      const double c = h[k] * h[k] / 6.0;
      yr += q0r - q1r;
      yi += q0i - q1i;
      mr += c * (-2.0 * q1r + 3.0 * q2r - q3r);
      mi += c * (-2.0 * q1i + 3.0 * q2i - q3i);
    }
    if (k > 0) {
      const int j = k - 1;
      const double* a = fd + 8 * j;
      const double* b = fn + 8 * j;
      const double q1r = a[2] + scale * b[2], q1i = a[3] + scale * b[3];
      const double q3r = a[6] + scale * b[6], q3i = a[7] + scale * b[7];
      const double c = h[j] * h[j] / 6.0;
      yr += q1r;
      yi += q1i;
      mr += c * (q3r - q1r);
      mi += c * (q3i - q1i);
    }
    gy[2 * k] = yr;
    gy[2 * k + 1] = yi;
    gm[2 * k] = mr;
    gm[2 * k + 1] = mi;
  }
  __syncthreads();
  // M = T^-1 D z on the interior knots, T symmetric tridiagonal: the z-partials through M are
  // D^T T^-1 g_M.  The Thomas solve of the n interior rows is two first-order linear recurrences,
  //   forward   y_i = A_i + B_i y_{i-1},  A_i = g_i / p_i,  B_i = -h_i / p_i,  y_{-1} = 0,
  //   backward  x_i = y_i + C_i x_{i+1},  C_i = -c'_i,  x_n = 0,
  // each taken as a scan of affine maps over the 64 lanes of one wave (re on wave 0, im on wave 1):
  // lane l composes its rows 2l and 2l + 1, six shuffle rounds compose the lanes' maps in a fixed
  // order, and the row a lane's map skips is filled in from its neighbour's result.
  const int n = N - 2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave < 2) {
    const int comp = wave;
    const int i0 = 2 * lane, i1 = 2 * lane + 1;
    const double A0 = i0 < n ? gm[2 * (i0 + 1) + comp] * thinv[i0] : 0.0;
    const double B0 = i0 < n && i0 > 0 ? -h[i0] * thinv[i0] : 0.0;
    const double A1 = i1 < n ? gm[2 * (i1 + 1) + comp] * thinv[i1] : 0.0;
    const double B1 = i1 < n ? -h[i1] * thinv[i1] : 0.0;
    double P = A1 + B1 * A0, Q = B1 * B0;  // y_{i1} = P + Q y_{i0 - 1}
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const double Pe = __shfl_up(P, d), Qe = __shfl_up(Q, d);  // the map of the rows before
      if (lane >= d) {
        P = P + Q * Pe;
        Q = Q * Qe;
      }
    }
    const double yb = __shfl_up(P, 1);  // y_{i0 - 1}, the previous lane's last row
    const double Y0 = i0 < n ? A0 + B0 * (lane > 0 ? yb : 0.0) : 0.0;
    const double Y1 = i1 < n ? P : 0.0;
    const double C0 = i0 < n - 1 ? -thc[i0] : 0.0;
    const double C1 = i1 < n - 1 ? -thc[i1] : 0.0;
    double X = Y0 + C0 * Y1, Z = C0 * C1;  // x_{i0} = X + Z x_{i1 + 1}
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const double Xa = __shfl_down(X, d), Za = __shfl_down(Z, d);  // the map of the rows after
      if (lane + d < 64) {
        X = X + Z * Xa;
        Z = Z * Za;
      }
    }
    const double xa = __shfl_down(X, 1);  // x_{i1 + 1}, the next lane's first row
    if (i0 < n) u[2 * (i0 + 1) + comp] = X;
    if (i1 < n) u[2 * (i1 + 1) + comp] = Y1 + C1 * (lane < 63 ? xa : 0.0);
    if (lane == 0) {
      u[comp] = 0.0;
      u[2 * (N - 1) + comp] = 0.0;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    double yr = gy[2 * k], yi = gy[2 * k + 1];
    // D[k', k] for interior rows k' in {k-1, k, k+1}
    if (k + 1 <= N - 2) {
      const double d = 6.0 / h[k];
      yr += d * u[2 * (k + 1)];
      yi += d * u[2 * (k + 1) + 1];
    }
    if (k >= 1 && k <= N - 2) {
      const double d = -6.0 / h[k] - 6.0 / h[k - 1];
      yr += d * u[2 * k];
      yi += d * u[2 * k + 1];
    }
    if (k - 1 >= 1) {
      const double d = 6.0 / h[k - 1];
      yr += d * u[2 * (k - 1)];
      yi += d * u[2 * (k - 1) + 1];
    }
    if (jb.swave == kSwavePolar) {
      const double a = th[2 * k], ph = th[2 * k + 1];
      double sn, cs;
      sincos(ph, &sn, &cs);
      ob[1 + 2 * k] = yr * cs + yi * sn;
      ob[2 + 2 * k] = a * (-yr * sn + yi * cs);
    } else if (jb.swave == kSwaveCartesian) {
      ob[1 + 2 * k] = yr;
      ob[2 + 2 * k] = yi;
    } else {
      gy[2 * k] = yr;  // isobar: combined below
      gy[2 * k + 1] = yi;
    }
  }
  // Isobar S-wave: a constant c_NR, carried as a two-knot spline with both knots at c_NR / 2 (which
  // the symmetrised sum S(s12) + S(s13) returns as c_NR).  Its partials are the two knots' z-partials
  // Y = y_0 + y_1 taken through z = c_NR / 2 to (|c_NR|, arg c_NR).
  if (jb.swave == kSwaveIsobar) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const double yr = gy[0] + gy[2], yi = gy[1] + gy[3];
      const double cm = 2.0 * th[0], ph = th[1];
      double sn, cs;
      sincos(ph, &sn, &cs);
      ob[1] = 0.5 * (yr * cs + yi * sn);
      ob[2] = 0.5 * cm * (-yr * sn + yi * cs);
    }
  }
  // external offset of the resonance block: after the knots, or after c_NR
  const int o = jb.swave == kSwaveIsobar ? 2 : 2 * N;
  // the resonances on wave 2 and -2 ln L on wave 3, beside the knots on waves 0 and 1
  for (int r = threadIdx.x - 128; r >= 0 && r < R; r += 64) {
    const double gr = fd[s0 + 1 + 2 * r] + scale * fn[s0 + 1 + 2 * r];
    const double gi = fd[s0 + 2 + 2 * r] + scale * fn[s0 + 2 + 2 * r];
    const double cm = th[2 * N + 2 * r], ca = th[2 * N + 2 * r + 1];
    double sn, cs;
    sincos(ca, &sn, &cs);
    ob[1 + o + 2 * r] = gr * cs + gi * sn;
    ob[2 + o + 2 * r] = cm * (-gr * sn + gi * cs);
    double dm = 0.0, dg = 0.0;
    if (jb.otf) {
      const int om = s0 + 1 + 2 * R + 2 * r, og = s0 + 1 + 4 * R + 2 * r;
      const double hmr = fd[om] + scale * fn[om], hmi = fd[om + 1] + scale * fn[om + 1];
      const double hgr = fd[og] + scale * fn[og], hgi = fd[og + 1] + scale * fn[og + 1];
      const double cr = cm * cs, ci = cm * sn;
      dm = cr * hmr + ci * hmi;
      dg = cr * hgr + ci * hgi;
    }
    ob[1 + o + 2 * R + 2 * r] = dm;
    ob[2 + o + 2 * R + 2 * r] = dg;
  }
  if (threadIdx.x == 192) ob[0] = -2.0 * fd[s0] + jb.c_eps + 2.0 * jb.n_ev * log(I);
  __syncthreads();
  if (threadIdx.x < 64) {
    const int nout = 1 + o + 4 * R;
    for (int i = threadIdx.x; i < nout; i += 64) out[i] = ob[i];
    if (jb.seq_out) {
      // The results may sit in host memory that a host thread polls: the wave's stores are made
      // visible system-wide before the sequence number that tells the host they are complete.
      // Results in device memory need no fence: the kernel's end orders them before later work.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
      if (threadIdx.x == 0) __hip_atomic_store(jb.seq_out, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// parts: the number of consecutive parts each wave's tile range is swept in (1 with shapes floated);
// order (0 or 1): ascending or descending part order.  The result is the same either way, bit for bit.
template <typename Real, int R, bool OTF>
__global__ __launch_bounds__(512) void k_eval(const Segment* __restrict__ segs, const int2* __restrict__ block_map,
                                              const Job* __restrict__ jobs, Kin<Real> kin, int max_nint,
                                              ArgTable targ, int parts, int order) {
  extern __shared__ double lds[];
  const int waves = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int2 bm = block_map[blockIdx.x];  // (segment, block index within the segment)
  const Segment sg = segs[bm.x];
  const int nsc = 1 + 2 * R + (OTF ? 4 * R : 0);
  const int stride = 8 * max_nint;
  // LDS: [evaluation table | interval histograms, `parts` per wave | sets of scalars, `parts` per wave]
  constexpr bool kF64 = sizeof(Real) == sizeof(double);
  const int tw = (table_real_words(max_nint, R, kF64) * (int)sizeof(Real) + 7) / 8;
  double* tab_lds = lds;
  double* bins = lds + tw;
  double* scal = bins + parts * waves * stride;
  {
    const unsigned* src = sg.table ? (const unsigned*)sg.table : (const unsigned*)targ.w;
    unsigned* dst = (unsigned*)tab_lds;
    const int words = table_real_words(sg.nint, R, kF64) * (int)sizeof(Real) / 4;
    for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
  }
  for (int i = threadIdx.x; i < parts * waves * (stride + nsc); i += blockDim.x) bins[i] = 0.0;
  __syncthreads();
  const Real* tab = (const Real*)tab_lds;
  double* wb = bins + parts * wave * stride;
  double* ws = scal + parts * wave * nsc;
  if (sg.kind == 0) {
    run_segment<Real, R, OTF, 0>(sg, kin, tab, wb, ws, wave, lane, waves, bm.y, stride, parts, order);
  } else if (sg.kind == 1) {
    run_segment<Real, R, OTF, 1>(sg, kin, tab, wb, ws, wave, lane, waves, bm.y, stride, parts, order);
  } else {
    // the quadratic form needs the resonance amplitudes fixed: never set up with shapes floated
    if constexpr (!OTF) run_qform<Real, R>(sg, tab, wb, ws, wave, lane, waves, bm.y);
  }
  __syncthreads();
  const int rs = sg.rs;
  double* rec = sg.records + (long long)bm.y * rs;
  const int nb = 8 * sg.nint;
  // waves in order, each wave's parts in order
  for (int f = threadIdx.x; f < nb + nsc; f += blockDim.x) {
    double s = 0.0;
    if (f < nb) {
      for (int w = 0; w < parts * waves; ++w) s += bins[w * stride + f];
    } else {
      for (int w = 0; w < parts * waves; ++w) s += scal[w * nsc + (f - nb)];
    }
    rec[f] = s;
  }

}

// ---------------------------------------------------------------------------------------------
// K3: group sums.  Group g of a segment: the records of its blocks [32 g, 32 g + 32), summed in block
// order into the job's group record.  No cross-block communication inside a kernel: the kernel
// boundary after the streaming kernel makes its records visible.  One block per task (segment, group)
// of `tasks`, or, with tasks == nullptr, per group of the single job described by `plan`.

__global__ __launch_bounds__(512) void k_group_sum(const Segment* __restrict__ segs, const Job* __restrict__ jobs,
                                                   const int2* __restrict__ tasks, GroupPlan plan) {
  const double* rb;
  double* go;
  int rs, gsz;
  if (tasks) {
    const int2 tk = tasks[blockIdx.x];
    const Segment& sg = segs[tk.x];
    const Job& jb = jobs[sg.job];
    const int g = tk.y;
    rs = sg.rs;
    gsz = min(kGroup, sg.n_blocks - g * kGroup);
    rb = sg.records + (long long)g * kGroup * rs;
    go = jb.grec + (long long)(sg.g0 + g) * rs;
  } else {
    const int k = (int)blockIdx.x < plan.G_d ? 0 : 1;
    const int g = k ? (int)blockIdx.x - plan.G_d : (int)blockIdx.x;
    rs = plan.rs;
    gsz = min(kGroup, plan.n_blocks[k] - g * kGroup);
    rb = plan.records[k] + (long long)g * kGroup * rs;
    go = plan.grec + (long long)(k ? plan.G_d + g : g) * rs;
  }
  for (int f = threadIdx.x; f < rs; f += blockDim.x) {
    // every load reads a valid record (the index is clamped into the group) and is issued without a
    // branch; records past the group's end are then dropped from the sum
    double v[kGroup];
#pragma unroll
    for (int b = 0; b < kGroup; ++b) v[b] = rb[(long long)min(b, gsz - 1) * rs + f];
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < kGroup; ++b) s += b < gsz ? v[b] : 0.0;
    go[f] = s;
  }
}

// K4: one block per job: sum the group records in order and run the FP64 finish.
constexpr int kMaxRecord = 8 * (kMaxKnots - 1) + 1 + 6 * kMaxRes;

constexpr int kMaxConsts = 3 * kMaxKnots - 5;
constexpr int kMaxTheta = 2 * kMaxKnots + 2 * kMaxRes;  // knot pairs and coefficient pairs
constexpr int kFinishThreads = 512;

// One block of kFinishThreads per job.  `jobs` == nullptr: a single job passed by value in `one`
// (saves the dependent load of its descriptor).
__global__ __launch_bounds__(kFinishThreads) void k_job_finish(const Job* __restrict__ jobs, Job one, ArgTable targ,
                                                              unsigned long long seq, double* out_override) {
  __shared__ double fin[2 * kMaxRecord];
  __shared__ double kc[kMaxConsts];
  __shared__ double thl[kMaxTheta];
  const Job jb = jobs ? jobs[blockIdx.x] : one;
  const int rs = jb.rs, nf = 2 * rs, nkc = 3 * jb.N - 5, nth = 2 * jb.N + 2 * jb.R;
  // the constants and parameters are requested first; they are only needed once the records are summed
  static_assert(kMaxConsts <= kFinishThreads && kMaxTheta <= kFinishThreads, "one word per thread");
  static_assert(kFinishThreads >= 256 && kMaxKnots <= 130 && kMaxRes <= 64,
                "the finish takes the knots on waves 0-1 (128 interior rows at most), resonances on wave 2, "
                "the log on wave 3");
  const double* th = jb.tab64 ? jb.tab64 : (const double*)((const char*)targ.w + jb.theta_off);
  const double kcv = threadIdx.x < nkc ? jb.consts[threadIdx.x] : 0.0;
  const double thv = threadIdx.x < nth ? th[threadIdx.x] : 0.0;
  // field f < rs of the data groups, then of the normalisation groups.  Each thread takes up to FPT
  // fields at once and issues the loads of eight groups of all of them before adding, so the sums
  // wait on about one memory round trip; each field's groups are added in group order.
  constexpr int FPT = 2;
  const int gmax = max(jb.G_d, jb.G_n);
  for (int f0 = threadIdx.x; f0 < nf; f0 += FPT * blockDim.x) {
    // Loads are issued without branches: the field and the group index are clamped to valid records
    // (every job has at least one group of each kind), and what lies past the end is dropped.
    const double* p[FPT];
    int G[FPT], Gl[FPT];
    double sum[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = f0 + j * blockDim.x;
      const int fc = min(f, nf - 1);
      const bool nrm = fc >= rs;
      G[j] = f < nf ? (nrm ? jb.G_n : jb.G_d) : 0;
      Gl[j] = (nrm ? jb.G_n : jb.G_d) - 1;
      p[j] = jb.grec + (long long)(nrm ? jb.G_d : 0) * rs + (nrm ? fc - rs : fc);
      sum[j] = 0.0;
    }
    for (int k0 = 0; k0 < gmax; k0 += 8) {
      double v[FPT][8];
#pragma unroll
      for (int j = 0; j < FPT; ++j)
#pragma unroll
        for (int k = 0; k < 8; ++k) v[j][k] = p[j][(long long)min(k0 + k, Gl[j]) * rs];
#pragma unroll
      for (int j = 0; j < FPT; ++j)
#pragma unroll
        for (int k = 0; k < 8; ++k) sum[j] += k0 + k < G[j] ? v[j][k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < FPT; ++j)
      if (f0 + j * blockDim.x < nf) fin[f0 + j * blockDim.x] = sum[j];
  }
  if (threadIdx.x < nkc) kc[threadIdx.x] = kcv;
  if (threadIdx.x < nth) thl[threadIdx.x] = thv;
  __syncthreads();
  finish_job(jb, fin, kc, thl, seq, out_override ? out_override : jb.out);
}

// ---------------------------------------------------------------------------------------------
// Component integrals I_jk = sum_p w_p A_j A_k^* over the normalisation points (Eq. 1 components).

template <typename Real, int R>
__global__ __launch_bounds__(256) void k_integrals(Segment sg, const Real* __restrict__ wsel,
                                                   double* __restrict__ records) {
  using V2 = typename Ops<Real>::V2;
  constexpr int K = R + 1;
  __shared__ double part[4][2 * K * K];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const Real* __restrict__ tab = (const Real*)sg.table;
  const V2* __restrict__ tt = (const V2*)sg.tt;
  const V2* __restrict__ cache = (const V2*)sg.cache;
  double acc[2 * K * K];
#pragma unroll
  for (int i = 0; i < 2 * K * K; ++i) acc[i] = 0.0;
  for (int ti = blockIdx.x * 4 + wave; ti < sg.n_tiles; ti += gridDim.x * 4) {
    const Tile td = sg.tiles[ti];
    const Real* p12 = tab + 8 * td.j12;
    const Real* p13 = tab + 8 * td.j13;
    for (int i = lane; i < td.count; i += 64) {
      const long long p = (long long)td.start + i;
      const Real x12 = tt[p].x, x13 = tt[p].y;
      double cr[K], ci[K];
      cr[0] = (double)(p12[0] + x12 * (p12[2] + x12 * (p12[4] + x12 * p12[6]))) +
              (double)(p13[0] + x13 * (p13[2] + x13 * (p13[4] + x13 * p13[6])));
      ci[0] = (double)(p12[1] + x12 * (p12[3] + x12 * (p12[5] + x12 * p12[7]))) +
              (double)(p13[1] + x13 * (p13[3] + x13 * (p13[5] + x13 * p13[7])));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const V2 v = cache[(long long)r * sg.n + p];
        cr[r + 1] = v.x;
        ci[r + 1] = v.y;
      }
      const double w = wsel[p];
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          acc[2 * (j * K + k)] += w * (cr[j] * cr[k] + ci[j] * ci[k]);
          acc[2 * (j * K + k) + 1] += w * (ci[j] * cr[k] - cr[j] * ci[k]);
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 2 * K * K; ++i) {
    const double v = wave_sum(acc[i]);
    if (lane == 0) part[wave][i] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * K * K; i += blockDim.x)
    records[(long long)blockIdx.x * 2 * K * K + i] = ((part[0][i] + part[1][i]) + part[2][i]) + part[3][i];
}

__global__ __launch_bounds__(256) void k_sum_records(const double* __restrict__ rec, int nrec, int rs,
                                                     double* __restrict__ out) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, prt = threadIdx.x >> 6;
  const int f = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (f < rs)
    for (int b = prt; b < nrec; b += 4) acc += rec[(long long)b * rs + f];
  part[prt][lane] = acc;
  __syncthreads();
  if (prt == 0 && f < rs) out[f] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// ---------------------------------------------------------------------------------------------
// Efficiency table lookup: bilinear between bin centres, constant beyond the outermost centres; the
// bin index is decided in FP64.

__device__ __forceinline__ double eff_lookup(const float* __restrict__ tab, int nx, int ny, double lo, double hi,
                                             double s12, double s13) {
  const double dx = (hi - lo) / nx, dy = (hi - lo) / ny;
  double ux = (s12 - lo) / dx - 0.5, uy = (s13 - lo) / dy - 0.5;
  double fx = floor(ux), fy = floor(uy);
  fx = fx < 0.0 ? 0.0 : (fx > nx - 2 ? nx - 2 : fx);
  fy = fy < 0.0 ? 0.0 : (fy > ny - 2 ? ny - 2 : fy);
  const int i = (int)fx, j = (int)fy;
  double tx = ux - i, ty = uy - j;
  tx = tx < 0.0 ? 0.0 : (tx > 1.0 ? 1.0 : tx);
  ty = ty < 0.0 ? 0.0 : (ty > 1.0 ? 1.0 : ty);
  const double a = tab[i * ny + j], b = tab[(i + 1) * ny + j], c = tab[i * ny + j + 1], d = tab[(i + 1) * ny + j + 1];
  return (1.0 - tx) * (1.0 - ty) * a + tx * (1.0 - ty) * b + (1.0 - tx) * ty * c + tx * ty * d;
}

__global__ __launch_bounds__(256) void k_eff(const double* __restrict__ s12, const double* __restrict__ s13, long long n,
                                             const float* __restrict__ tab, int nx, int ny, double lo, double hi,
                                             double* __restrict__ eps) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x)
    eps[p] = eff_lookup(tab, nx, ny, lo, hi, s12[p], s13[p]);
}

// ---------------------------------------------------------------------------------------------
// Toy generation (FP64): Philox4x32-10 candidates, region test, accept-reject on |A|^2 eff.

struct U4 {
  unsigned x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
    const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
    const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__device__ __forceinline__ double unit53(unsigned a, unsigned b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ double map_box(double lo, double span, double u) {
#pragma clang fp contract(off)
  const double t = span * u;
  return lo + t;
}

__device__ __forceinline__ bool inside_dalitz(const GenArgs& g, double s12, double s13) {
  const double lo = (g.m1 + g.m2) * (g.m1 + g.m2), hi = (g.M - g.m3) * (g.M - g.m3);
  if (!(s12 >= lo && s12 <= hi)) return false;
  const double rs = sqrt(s12);
  const double e1 = (s12 - g.m2 * g.m2 + g.m1 * g.m1) / (2.0 * rs);
  const double e3 = (g.M * g.M - s12 - g.m3 * g.m3) / (2.0 * rs);
  const double p1 = sqrt(fmax(e1 * e1 - g.m1 * g.m1, 0.0));
  const double p3 = sqrt(fmax(e3 * e3 - g.m3 * g.m3, 0.0));
  const double es = (e1 + e3) * (e1 + e3);
  return s13 >= es - (p1 + p3) * (p1 + p3) && s13 <= es - (p1 - p3) * (p1 - p3);
}

__device__ __forceinline__ void spline_at(const GenArgs& g, double s, double& re, double& im) {
  int lo = 0, hi = g.N;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (g.knots[mid] <= s)
      lo = mid + 1;
    else
      hi = mid;
  }
  int j = lo - 1;
  j = j < 0 ? 0 : (j > g.N - 2 ? g.N - 2 : j);
  const double t = (s - g.knots[j]) / (g.knots[j + 1] - g.knots[j]);
  const double* p = g.poly + 8 * j;
  re += p[0] + t * (p[2] + t * (p[4] + t * p[6]));
  im += p[1] + t * (p[3] + t * (p[5] + t * p[7]));
}

template <int R>
__global__ __launch_bounds__(kGenBlock) void k_generate(GenArgs g, Kin<double> kin, long long first, int count,
                                                        double* __restrict__ o12, double* __restrict__ o13,
                                                        double* __restrict__ of, unsigned char* __restrict__ oflag,
                                                        int* __restrict__ block_counts, int* __restrict__ exceeded) {
  constexpr int R1 = R > 0 ? R : 1;
  const int i = blockIdx.x * kGenBlock + threadIdx.x;
  int flag = 0;
  if (i < count) {
    const unsigned long long idx = (unsigned long long)(first + i);
    const unsigned k0 = (unsigned)g.seed, k1 = (unsigned)(g.seed >> 32);
    const U4 a = philox4x32_10(U4{(unsigned)idx, (unsigned)(idx >> 32), 0u, 0u}, k0, k1);
    const U4 b = philox4x32_10(U4{(unsigned)idx, (unsigned)(idx >> 32), 1u, 0u}, k0, k1);
    const double s12 = map_box(g.smin, g.span, unit53(a.x, a.y));
    const double s13 = map_box(g.smin, g.span, unit53(a.z, a.w));
    const double v = unit53(b.x, b.y);
    const bool in = inside_dalitz(g, s12, s13);
    double f = 0.0;
    if (in) {
      double ar = 0.0, ai = 0.0;
      spline_at(g, s12, ar, ai);
      spline_at(g, s13, ar, ai);
      double br[R1] = {}, bi[R1] = {};
      bw_pairing<double, R, false>(kin, g.res, s12, s13, br, bi, nullptr, nullptr, nullptr, nullptr);
      bw_pairing<double, R, false>(kin, g.res, s13, s12, br, bi, nullptr, nullptr, nullptr, nullptr);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        ar += g.c[2 * r] * br[r] - g.c[2 * r + 1] * bi[r];
        ai += g.c[2 * r] * bi[r] + g.c[2 * r + 1] * br[r];
      }
      f = ar * ar + ai * ai;
      if (g.eff) f *= eff_lookup(g.eff, g.nx, g.ny, g.eff_lo, g.eff_hi, s12, s13);
      if (f > g.fmax) atomicOr(exceeded, 1);
    }
    flag = g.mode == 0 ? (in && f > v * g.fmax) : in;
    o12[i] = s12;
    o13[i] = s13;
    of[i] = f;
    oflag[i] = (unsigned char)flag;
  }
  const int cnt = __syncthreads_count(flag);
  if (threadIdx.x == 0) block_counts[blockIdx.x] = cnt;
}

__global__ void k_scan(const int* __restrict__ counts, int nb, int* __restrict__ offsets, int* __restrict__ total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int s = 0;
    for (int b = 0; b < nb; ++b) {
      offsets[b] = s;
      s += counts[b];
    }
    *total = s;
  }
}

__global__ __launch_bounds__(kGenBlock) void k_scatter(const unsigned char* __restrict__ flag, int count,
                                                       const int* __restrict__ offsets, const double* __restrict__ a,
                                                       const double* __restrict__ b, const double* __restrict__ c,
                                                       double* __restrict__ oa, double* __restrict__ ob,
                                                       double* __restrict__ oc) {
  __shared__ int wsum[kGenBlock / 64];
  const int i = blockIdx.x * kGenBlock + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool fl = i < count && flag[i];
  const unsigned long long bal = __ballot(fl);
  const int lp = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wsum[wave] = __popcll(bal);
  __syncthreads();
  int woff = 0;
  for (int w = 0; w < wave; ++w) woff += wsum[w];
  if (fl) {
    const int o = offsets[blockIdx.x] + woff + lp;
    if (oa) oa[o] = a[i];
    if (ob) ob[o] = b[i];
    if (oc) oc[o] = c[i];
  }
}

// ---------------------------------------------------------------------------------------------
// launchers

namespace {
template <typename Real>
hipError_t cache_impl(int R, const Segment* s, const double* res, const Kin<double>& k, hipStream_t st) {
  const long long want = (s->n + 255) / 256;
  const int grid = (int)(want < 8192 ? (want > 0 ? want : 1) : 8192);
  switch (R) {
    case 0: return hipSuccess;
    case 1: k_cache<Real, 1><<<grid, 256, 0, st>>>(*s, res, k); break;
    case 2: k_cache<Real, 2><<<grid, 256, 0, st>>>(*s, res, k); break;
    case 3: k_cache<Real, 3><<<grid, 256, 0, st>>>(*s, res, k); break;
    case 4: k_cache<Real, 4><<<grid, 256, 0, st>>>(*s, res, k); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real, bool OTF>
hipError_t eval_impl2(int R, const Segment* segs, const int2* bs, const Job* jobs, int nb, int waves, int max_nint,
                      const void* kin, const ArgTable* targ, int parts, int order, hipStream_t st, hipEvent_t e0,
                      hipEvent_t e1) {
  Kin<Real> k = *(const Kin<Real>*)kin;
  const int nsc = 1 + 2 * R + (OTF ? 4 * R : 0);
  const int tw = (table_real_words(max_nint, R, sizeof(Real) == sizeof(double)) * (int)sizeof(Real) + 7) / 8;
  // as many parts as asked for whose histograms fit the 64 KiB a workgroup may take; one with shapes
  // floated (that sweep is bound by the vector ALU, not by reads the Infinity Cache could serve)
  if (OTF) parts = 1;
  size_t lds = 0;
  for (;; parts /= 2) {
    lds = ((size_t)tw + (size_t)parts * waves * (8 * max_nint + nsc)) * sizeof(double);
    if (lds <= 65536 || parts == 1) break;
  }
  static const ArgTable empty{};
  const ArgTable* ta = targ ? targ : &empty;
  const dim3 grid(nb), block(64 * waves);
  const void* fn = nullptr;
  switch (R) {
    case 0: fn = (const void*)k_eval<Real, 0, OTF>; break;
    case 1: fn = (const void*)k_eval<Real, 1, OTF>; break;
    case 2: fn = (const void*)k_eval<Real, 2, OTF>; break;
    case 3: fn = (const void*)k_eval<Real, 3, OTF>; break;
    case 4: fn = (const void*)k_eval<Real, 4, OTF>; break;
    default: return hipErrorInvalidValue;
  }
  void* args[] = {(void*)&segs, (void*)&bs, (void*)&jobs, (void*)&k, (void*)&max_nint, (void*)ta, (void*)&parts,
                  (void*)&order};
  // start/stop events (when given) are recorded on the stream right before and after the dispatch
  // (events attached to the dispatch itself cost ~15 us of host time per launch on this runtime)
  if (e0) {
    const hipError_t e = hipEventRecord(e0, st);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipLaunchKernel(fn, grid, block, args, lds, st);
  if (e == hipSuccess && e1) e = hipEventRecord(e1, st);
  return e;
}

template <typename Real>
hipError_t integrals_impl(int R, const Segment* s, const void* w, double* rec, int nb, double* out, hipStream_t st) {
  const Real* ws = (const Real*)w;
  switch (R) {
    case 0: k_integrals<Real, 0><<<nb, 256, 0, st>>>(*s, ws, rec); break;
    case 1: k_integrals<Real, 1><<<nb, 256, 0, st>>>(*s, ws, rec); break;
    case 2: k_integrals<Real, 2><<<nb, 256, 0, st>>>(*s, ws, rec); break;
    case 3: k_integrals<Real, 3><<<nb, 256, 0, st>>>(*s, ws, rec); break;
    case 4: k_integrals<Real, 4><<<nb, 256, 0, st>>>(*s, ws, rec); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int rs = 2 * (R + 1) * (R + 1);
  k_sum_records<<<(rs + 63) / 64, 256, 0, st>>>(rec, nb, rs, out);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_cache(bool fp64, int R, const Segment* s, const double* res64, const Kin<double>& kin64,
                        hipStream_t st) {
  (void)hipGetLastError();
  return fp64 ? cache_impl<double>(R, s, res64, kin64, st) : cache_impl<float>(R, s, res64, kin64, st);
}

hipError_t launch_eval(bool fp64, int R, bool otf, const Segment* segs, const int2* bs, const Job* jobs, int nb,
                       int waves, int max_nint, const void* kin, const ArgTable* targ, int parts, int order,
                       hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  (void)hipGetLastError();
  if (parts != 1 && parts != 2 && parts != 4) return hipErrorInvalidValue;
  order &= 1;
  if (fp64)
    return otf ? eval_impl2<double, true>(R, segs, bs, jobs, nb, waves, max_nint, kin, targ, parts, order, st, e0, e1)
               : eval_impl2<double, false>(R, segs, bs, jobs, nb, waves, max_nint, kin, targ, parts, order, st, e0, e1);
  return otf ? eval_impl2<float, true>(R, segs, bs, jobs, nb, waves, max_nint, kin, targ, parts, order, st, e0, e1)
             : eval_impl2<float, false>(R, segs, bs, jobs, nb, waves, max_nint, kin, targ, parts, order, st, e0, e1);
}

hipError_t launch_reduce(const Segment* segs, const Job* jobs, const int2* tasks, int n_tasks, int n_jobs,
                         const ArgTable* targ, hipStream_t st,
                         unsigned long long seq, double* out_override, const Job* single, const GroupPlan* plan) {
  (void)hipGetLastError();
  static const ArgTable empty{};
  if (plan) {
    if (n_jobs != 1 || plan->G_d < 1 || plan->G_n < 1) return hipErrorInvalidValue;
    k_group_sum<<<plan->G_d + plan->G_n, 512, 0, st>>>(segs, jobs, nullptr, *plan);
  } else {
    k_group_sum<<<n_tasks, 512, 0, st>>>(segs, jobs, tasks, GroupPlan{});
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  static const Job none{};
  if (single && n_jobs != 1) return hipErrorInvalidValue;
  k_job_finish<<<n_jobs, kFinishThreads, 0, st>>>(single ? nullptr : jobs, single ? *single : none,
                                                  targ ? *targ : empty, seq, out_override);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_upload(const uint4* __restrict__ src, uint4* __restrict__ dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t launch_upload(void* d_dst, const void* h_src_dev, size_t bytes, hipStream_t st) {
  (void)hipGetLastError();
  if (bytes % 16 || (reinterpret_cast<uintptr_t>(d_dst) | reinterpret_cast<uintptr_t>(h_src_dev)) % 16)
    return hipErrorInvalidValue;
  const long long n = (long long)(bytes / 16);
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<long long>((n + 255) / 256, 64);
  k_upload<<<blocks, 256, 0, st>>>(static_cast<const uint4*>(h_src_dev), static_cast<uint4*>(d_dst), n);
  return hipGetLastError();
}

template <typename Real>
hipError_t moments_impl(int R, const Segment* s, const Tile* cells, int n_cells, double* mom, hipStream_t st) {
  switch (R) {
    case 0: k_moments<Real, 0><<<n_cells, kMomChunk, 0, st>>>(*s, cells, mom); break;
    case 1: k_moments<Real, 1><<<n_cells, kMomChunk, 0, st>>>(*s, cells, mom); break;
    case 2: k_moments<Real, 2><<<n_cells, kMomChunk, 0, st>>>(*s, cells, mom); break;
    case 3: k_moments<Real, 3><<<n_cells, kMomChunk, 0, st>>>(*s, cells, mom); break;
    case 4: k_moments<Real, 4><<<n_cells, kMomChunk, 0, st>>>(*s, cells, mom); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_moments(bool fp64, int R, const Segment* s, const Tile* cells, int n_cells, double* mom,
                          hipStream_t st) {
  (void)hipGetLastError();
  if (n_cells <= 0) return hipSuccess;
  return fp64 ? moments_impl<double>(R, s, cells, n_cells, mom, st) : moments_impl<float>(R, s, cells, n_cells, mom, st);
}

hipError_t launch_integrals(bool fp64, int R, const Segment* s, const void* w, double* rec, int nb, double* out,
                            hipStream_t st) {
  (void)hipGetLastError();
  return fp64 ? integrals_impl<double>(R, s, w, rec, nb, out, st) : integrals_impl<float>(R, s, w, rec, nb, out, st);
}

hipError_t launch_eff_lookup(const double* s12, const double* s13, long long n, const float* tab, int nx, int ny,
                             double lo, double hi, double* eps, hipStream_t st) {
  (void)hipGetLastError();
  const long long want = (n + 255) / 256;
  const int grid = (int)(want < 8192 ? (want > 0 ? want : 1) : 8192);
  k_eff<<<grid, 256, 0, st>>>(s12, s13, n, tab, nx, ny, lo, hi, eps);
  return hipGetLastError();
}

hipError_t launch_generate_chunk(const GenArgs& g, const void* kin, long long first, int count, double* o12,
                                 double* o13, double* of, unsigned char* oflag, int* bc, int* exc, hipStream_t st) {
  (void)hipGetLastError();
  const Kin<double>& k = *(const Kin<double>*)kin;
  const int nb = (count + kGenBlock - 1) / kGenBlock;
  switch (g.R) {
    case 0: k_generate<0><<<nb, kGenBlock, 0, st>>>(g, k, first, count, o12, o13, of, oflag, bc, exc); break;
    case 1: k_generate<1><<<nb, kGenBlock, 0, st>>>(g, k, first, count, o12, o13, of, oflag, bc, exc); break;
    case 2: k_generate<2><<<nb, kGenBlock, 0, st>>>(g, k, first, count, o12, o13, of, oflag, bc, exc); break;
    case 3: k_generate<3><<<nb, kGenBlock, 0, st>>>(g, k, first, count, o12, o13, of, oflag, bc, exc); break;
    case 4: k_generate<4><<<nb, kGenBlock, 0, st>>>(g, k, first, count, o12, o13, of, oflag, bc, exc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_compact(const unsigned char* flag, int count, const int* counts, int* offsets, int* total,
                          const double* a, const double* b, const double* c, double* oa, double* ob, double* oc,
                          hipStream_t st) {
  (void)hipGetLastError();
  const int nb = (count + kGenBlock - 1) / kGenBlock;
  k_scan<<<1, 64, 0, st>>>(counts, nb, offsets, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scatter<<<nb, kGenBlock, 0, st>>>(flag, count, offsets, a, b, c, oa, ob, oc);
  return hipGetLastError();
}

}  // namespace mipwa
