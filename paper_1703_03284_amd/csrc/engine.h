// Internal interface between the host library (mipwa.cpp) and the gfx950 kernels (kernels.hip).
// Not installed; the public boundary is include/mipwa.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mipwa {

// Points per tile (a multiple of 64).  A tile holds points of a single spline cell (j12, j13), so
// inside a tile both interval indices are wave-uniform; each lane streams kTile/64 points of a tile
// with all their loads issued together.
#ifndef MIPWA_TILE
#define MIPWA_TILE 256
#endif
constexpr int kTile = MIPWA_TILE;
static_assert(kTile % 64 == 0, "tiles hold whole wavefronts");
constexpr int kMaxWaves = 16;
constexpr int kMaxRes = 4;
// S-wave parameter forms (mipwa_set_swave_form).  Inside the library theta is always the polar
// spline form; these select how the finish writes the gradient.
constexpr int kSwavePolar = 0, kSwaveCartesian = 1, kSwaveIsobar = 2;
constexpr int kMaxKnots = 128;
// Doubles of the per-model constants: Thomas factors and interval widths.
__host__ __device__ constexpr int consts_words(int N) { return 3 * N - 5; }
// Words per resonance in the evaluation table:
// m^2, kappa, delta, rho^2, L, m, dln(kappa)/dm, d(delta)/dm, d(delta)/dGamma, unused.
constexpr int kResWords = 10;

struct Tile {
  int j12, j13, start, count;
};

// Decay kinematics, precomputed on the host in FP64 and passed by value in working precision.
template <typename Real>
struct Kin {
  Real sum;             // M^2 + m1^2 + m2^2 + m3^2 (so s23 = sum - s12 - s13)
  Real thr_hi, thr_lo;  // (m1+m2)^2, (m1-m2)^2:  q^2 = (x - thr_hi)(x - thr_lo) / (4x)
  Real pb_hi, pb_lo;    // (M+m3)^2, (M-m3)^2:    p^2 = (x - pb_hi)(x - pb_lo) / (4x)
  Real t1corr;          // (M^2 - m3^2)(m1^2 - m2^2)
  Real t2a, t2b;        // 2M^2 + 2m3^2, (M^2 - m3^2)^2
  Real t2c, t2d;        // 2m1^2 + 2m2^2, (m1^2 - m2^2)^2
  Real rD2;             // D barrier radius squared
};

// Blocks of one segment are reduced in groups of kGroup consecutive blocks (k_group_sum), then the
// group records of a job are summed and the FP64 finish runs (k_job_finish).  Each stage is its own
// kernel, so no block ever reads another block's output within a launch.
constexpr int kGroup = 32;

// One stream of points (data events or normalisation points of one job) and where its per-block
// partial records go.  Lives in device memory; read with uniform (scalar) loads.
struct Segment {
  const void* tt;     // Real2[n]: (t12, t13), local spline coordinates of the two h+h- invariants
  const void* ss;     // double2[n]: (s12, s13), canonical order s12 <= s13 (FP64 in both precisions)
  const void* w;      // Real[n]: weight x efficiency (normalisation points), nullptr for data
  const void* cache;  // Real2[R][n]: symmetrised resonance amplitudes R_r at each point
  const Tile* tiles;
  const void* table;  // evaluation table in working precision (spline polynomials, c, resonances)
  double* records;    // n_blocks x rs
  long long n;        // number of points
  int n_tiles;
  int kind;           // 0 = data, 1 = normalisation points, 2 = normalisation as a quadratic form
                      // (kind 2: tiles = the cells, n_tiles = their number, cache = their moments)
  int nint;           // N - 1 spline intervals
  int rs;             // record size in doubles
  int n_blocks;       // blocks assigned to this segment
  int job;            // index of the segment's job in the job array
  int g0;             // first reduction group of this segment within its job
  int pad;
};

// One likelihood evaluation to finish (its data and normalisation segments).
struct Job {
  const double* tab64;   // theta[P]
  const double* consts;  // Thomas c'[N-2], 1/pivot[N-2], h[N-1] of the job's knots
  double* out;           // 1 + P results: -2 ln L, gradient (device or mapped host memory)
  unsigned long long* seq_out;  // when set: the evaluation's sequence number, stored after the results
  double* grec;          // (G_d + G_n) x rs group records
  double n_ev;
  double c_eps;          // -2 sum ln eff over the events
  int G_d, G_n;
  int N, R, rs, otf;
  int theta_off;         // byte offset of theta in the launch's ArgTable when tab64 == nullptr
  int swave;             // parameter form of the S-wave (kSwave*): the layout of the gradient written
};

__host__ __device__ constexpr int n_groups(int n_blocks) { return (n_blocks + kGroup - 1) / kGroup; }

// Small per-evaluation tables travel in the launch's kernel arguments: [table in working precision |
// theta (FP64) at theta_off bytes].  A segment with table == nullptr and a job with tab64 == nullptr
// read them from here.
constexpr int kArgBytes = 3840;
struct ArgTable {
  double w[kArgBytes / 8];
};

// Record layout (doubles): [8 * nint spline-polynomial partials (interval j, power m, re/im)]
// [sum] [2R: sum g conj(R_r)] [OTF: 2R sum g conj(dR_r/dm), 2R sum g conj(dR_r/dGamma)].
__host__ __device__ constexpr int record_size(int nint, int R, bool otf) { return 8 * nint + 1 + 2 * R + (otf ? 4 * R : 0); }
__host__ __device__ constexpr int table_words(int nint, int R) { return 8 * nint + 2 * R + kResWords * R; }
// An FP32 table is followed by the rounding residues of the coefficients that set the amplitude's size,
// [P_0 re, P_0 im, P_1 re, P_1 im of each interval | c_r re, im]: a coefficient is its FP32 word plus
// its residue, which carries the FP64 value to about 2^-48 (a rounding of the coefficients alone would
// act like a shift of theta by one FP32 ulp, coherent over every point).
__host__ __device__ constexpr int table_lo_words(int nint, int R) { return 4 * nint + 2 * R; }
// words of the table in the working precision
__host__ __device__ constexpr int table_real_words(int nint, int R, bool fp64) {
  return table_words(nint, R) + (fp64 ? 0 : table_lo_words(nint, R));
}

// ---- launchers (kernels.hip); all asynchronous on `stream` ----
// resonance cache of a segment, computed in FP64 from res64 (device, kResWords x R FP64 constants) and
// stored in working precision
hipError_t launch_cache(bool fp64, int R, const Segment* h_seg, const double* res64, const Kin<double>& kin64,
                        hipStream_t stream);
// e0/e1 (nullable): HIP events recorded by the dispatch at the kernel's start and end
// d_block_map[b] = (segment, block index within that segment) for every block b of the grid; each
// block writes its FP64 record.  e0/e1 (nullable): HIP events recorded by the dispatch at the kernel's
// start and end.
// parts (1, 2 or 4): each wave sweeps its tiles in that many consecutive parts, in ascending (order 0)
// or descending (order 1) part order; consecutive evaluations alternate the order so that each starts
// on what the previous one read last (the result is bitwise the same; sweep_parts chooses the count).
hipError_t launch_eval(bool fp64, int R, bool otf, const Segment* d_segs, const int2* d_block_map,
                       const Job* d_jobs, int n_blocks, int waves, int max_nint, const void* kin,
                       const ArgTable* args, int parts, int order, hipStream_t stream, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
// Parts for a sweep that reads `bytes` per evaluation: the alternation pays where the part read last
// is still in the 256 MB Infinity Cache of an MI355X when the next evaluation starts, and costs the
// extra flushes where the stream fits the cache (one pass in the same order each time is then served
// from it) or is several times its size.  Measured (mixed k_eval, us, one part / two parts): 260 MB
// 54.4 / 55.7, 312 MB 62.1 / 64.2, 416 MB 86.2 / 81.7, 520 MB 103.9 / 98.3, 624 MB 121.6 / 116.8,
// 832 MB 157.0 / 153.9; 1 GB (FP64) +2.7 % with two; four parts measured no gain at 520 MB.
constexpr double kInfinityCacheBytes = 256.0 * (1 << 20);
inline int sweep_parts(double bytes) {
  return bytes <= 1.4 * kInfinityCacheBytes ? 1 : bytes <= 3.5 * kInfinityCacheBytes ? 2 : 1;
}
// The group sums of a single job's two segments, passed by value (no task, segment or job descriptor
// to load first): block b < G_d sums data group b, block G_d + g normalisation group g.
struct GroupPlan {
  const double* records[2];  // the segments' block records (device)
  double* grec;              // (G_d + G_n) x rs group records (device)
  int n_blocks[2];
  int G_d, G_n, rs, pad;
};
// group sums (one block per task (segment, group), or per group of `plan` when given: then d_tasks
// and n_tasks are unused and n_jobs is 1) then one finishing block per job
hipError_t launch_reduce(const Segment* d_segs, const Job* d_jobs, const int2* d_tasks, int n_tasks, int n_jobs,
                         const ArgTable* args, hipStream_t stream, unsigned long long seq = 0,
                         double* out_override = nullptr, const Job* single = nullptr,
                         const GroupPlan* plan = nullptr);
// Copy `bytes` (a multiple of 16, both addresses 16-byte aligned) from mapped host memory to device
// memory with a kernel on `stream`.  Per-evaluation tables go up this way, ordered with the kernels
// that read them like any other kernel on the stream.
hipError_t launch_upload(void* d_dst, const void* h_src_dev, size_t bytes, hipStream_t stream);
hipError_t launch_integrals(bool fp64, int R, const Segment* h_seg, const void* w_override,
                            double* d_records, int n_blocks, double* d_out, hipStream_t stream);
// Moments of the normalisation points per spline cell for the quadratic form of I (fixed shapes):
// M_c[i][j] = sum_p w_p phi_i(p) conj(phi_j(p)) over the points of cell c, with
// phi = (t12^0..3, t13^0..3, R_1..R_R), stored as complex FP64, K = 8 + R, row-major [c][i][j].
inline int qform_dim(int R) { return 8 + R; }
hipError_t launch_moments(bool fp64, int R, const Segment* h_norm, const Tile* d_cells, int n_cells, double* d_mom,
                          hipStream_t stream);
hipError_t launch_eff_lookup(const double* d_s12, const double* d_s13, long long n, const float* d_table,
                             int nx, int ny, double lo, double hi, double* d_eps, hipStream_t stream);

// Toy generation: candidate evaluation + order-preserving compaction (FP64).
struct GenArgs {
  const double* poly;   // 8 * (N - 1) spline polynomial coefficients
  const double* knots;  // N
  const double* c;      // 2R
  const double* res;    // kResWords * R
  const float* eff;     // nx * ny or nullptr
  int N, R, nx, ny;
  double eff_lo, eff_hi;
  double M, m1, m2, m3; // kinematics for the region test
  double smin, span;    // candidate box
  unsigned long long seed;
  double fmax;
  int mode;             // 0: keep inside && f > v fmax; 1: keep inside (for the density maximum)
  int pad;
};
hipError_t launch_generate_chunk(const GenArgs& g, const void* kin, long long first, int count,
                                 double* d_s12, double* d_s13, double* d_f, unsigned char* d_flag,
                                 int* d_block_counts, int* d_exceeded, hipStream_t stream);
hipError_t launch_compact(const unsigned char* d_flag, int count, const int* d_block_counts,
                          int* d_block_offsets, int* d_total, const double* a, const double* b,
                          const double* c, double* out_a, double* out_b, double* out_c,
                          hipStream_t stream);
constexpr int kGenBlock = 1024;

}  // namespace mipwa
