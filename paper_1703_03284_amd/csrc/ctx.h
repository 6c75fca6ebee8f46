// The opaque context behind mipwa_ctx*.  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "engine.h"
#include "host.h"

struct mipwa_ctx {
  int device = 0;
  bool fp64 = true;
  mipwa::ModelHost mh;
  hipStream_t stream = nullptr;
  mipwa::PointSet ev, nm;
  mipwa::EffTable eff;

  std::vector<double> theta;       // internal: the polar spline layout (2N + 4R)
  bool have_theta = false;
  std::vector<unsigned char> fixed;  // external layout (ext_P entries)
  int swave = mipwa::kSwavePolar;    // parameter form seen through the C ABI
  // normalisation as a quadratic form over per-cell moments (fixed shapes only)
  bool qform = false;
  bool mom_valid = false;
  mipwa::DevBuf d_mom;
  bool otf = false;

  std::vector<double> cache_shape;
  bool cache_valid = false;

  // [Real evaluation table | pad to 256 B | FP64: theta, K^T, h]; h_blob is mapped host memory that a
  // kernel copies into d_blob ahead of each evaluation that does not carry its tables in arguments
  mipwa::DevBuf d_blob;
  mipwa::HostBuf h_blob;
  size_t tab64_off = 0, upload_bytes = 0, consts_off = 0;
  // small tables go in the kernel arguments instead of an upload
  bool use_arg = false;
  int arg_theta_off = 0;
  mipwa::ArgTable h_args{};

  mipwa::DevBuf d_segs, d_block_seg, d_records, d_grec, d_out, d_job, d_res64;
  mipwa::HostBuf h_out;          // mapped, coherent: the finish writes the results here
  double* h_out_dev = nullptr;   // device view of h_out
  mipwa::Segment h_segs[2];
  mipwa::Job h_jobs[2];          // host copies: the finish takes the job descriptor by value
  mipwa::GroupPlan h_plan{};     // the group sums' layout, passed by value as well
  int blocks_cfg = 512, waves_cfg = 0, waves_eff = 4;
  int n_blocks = 0, nb_d = 0, nb_n = 0, rs = 0;
  bool launch_dirty = true;

  // Timing events: two sets [before the first launch, sweep start, sweep end, after the finish] used
  // in turn, so that an evaluation reads the previous one's times after its own launches are queued.
  // A timed evaluation records one pair only: the step pair (first and last) or the sweep pair
  // (second and third), alternately; each pair costs device time, so timing samples every
  // timing_period-th evaluation.
  hipEvent_t ev_staged = nullptr;
  // Completion of the last enqueued evaluation and the stream it went to.  The context's scratch
  // (records, group records, tables, resonance cache, moments) is shared by every stream an
  // evaluation may be queued on, so the next enqueue on another stream waits for this event, and
  // host-side replacement of those buffers first waits for it.
  hipEvent_t ev_done = nullptr;
  hipStream_t last_st = nullptr;
  // ascending or descending order of the parts each wave of the point sweep reads; alternates per
  // evaluation
  int sweep_order = 0;
  int sweep_parts_eff = 1;
  hipEvent_t ev_t[2][4] = {};
  int ev_cur = 0;                 // set the next timed evaluation records into
  int ev_last = 0;                // set of the last timed evaluation
  bool set_unread[2] = {false, false};
  int set_kind[2] = {0, 0};       // 0: the step pair was recorded in the set, 1: the sweep pair
  bool timing_pending = false;
  int timing_period = 0;          // 0: off; n: every n-th evaluation is timed
  unsigned long long timing_calls = 0;
  int timing_next_kind = 0;
  long long t_count_step = 0, t_count_sweep = 0;
  unsigned long long seq = 0;     // sequence number of the last synchronous evaluation
  double t_total = 0.0, t_stream = 0.0;


  std::string err;

  ~mipwa_ctx() {
    if (ev_staged) (void)hipEventDestroy(ev_staged);
    if (ev_done) (void)hipEventDestroy(ev_done);
    for (auto& set : ev_t)
      for (hipEvent_t e : set)
        if (e) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
  }

  int fail(int code, const std::string& msg);
  // external parameter count and the offset of the resonance coefficients in the external layout
  bool use_qform() const { return qform && !otf && nm.loaded && nm.n_cells > 0; }
  int ext_P() const { return swave == mipwa::kSwaveIsobar ? 2 + 4 * mh.R : mh.P; }
  int ext_res_off() const { return swave == mipwa::kSwaveIsobar ? 2 : 2 * mh.N; }
  // external theta -> internal (polar spline) theta
  void to_internal(const double* ext, double* internal) const;
  // grid and record layout of an evaluation: blocks of the data and normalisation streams, record size
  // and reduction groups
  struct LaunchPlan {
    int B = 0, nb_d = 0, nb_n = 0, rs = 0, G_d = 0, G_n = 0, waves = 4;
    int parts = 1;  // parts of each wave's tile range in the point sweep (launch_eval)
  };
  LaunchPlan plan_launch() const;
  // segment and job descriptors of the point-sweep evaluation with its records at `records` and its
  // group records at `grec` (device addresses)
  void make_segments(const LaunchPlan& L, double* records, mipwa::Segment sg[2]) const;
  void make_job(const LaunchPlan& L, double* grec, mipwa::Job& jb) const;
  int rebuild_launch();
  int stage_params();
  bool shapes_changed() const;
  int ensure_cache(hipStream_t st);
  int prepare_eval(hipStream_t st);
  int enqueue_kernels(hipStream_t st, bool to_host, bool timed, unsigned long long s = 0, double* out = nullptr);
  size_t upload16() const { return (upload_bytes + 15) / 16 * 16; }
  int wait_result(unsigned long long s);
  bool take_timing() { return timing_period > 0 && timing_calls++ % (unsigned long long)timing_period == 0; }
  int fold_timing(int set);
  int fold_all_timing();
  int run_sync_eval();
  // order work about to go on stream st after the last evaluation queued on any other stream
  int order_after_last(hipStream_t st);
  // block the host until every evaluation queued so far, on any stream, has completed
  int drain();
};
