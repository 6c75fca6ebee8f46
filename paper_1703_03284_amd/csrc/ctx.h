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

  std::vector<double> theta;
  bool have_theta = false;
  std::vector<unsigned char> fixed;
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

  mipwa::DevBuf d_segs, d_block_seg, d_records, d_grec, d_tasks, d_out, d_job, d_res64;
  mipwa::HostBuf h_out;          // mapped, coherent: the finish writes the results here
  double* h_out_dev = nullptr;   // device view of h_out
  mipwa::Segment h_segs[2];
  int blocks_cfg = 512, waves_cfg = 0, waves_eff = 4;
  int n_blocks = 0, nb_d = 0, nb_n = 0, rs = 0, n_tasks = 0;
  bool launch_dirty = true;

  hipEvent_t ev_staged = nullptr, ev_t0 = nullptr, ev_t1 = nullptr, ev_t2 = nullptr, ev_t3 = nullptr;
  bool timing_pending = false;
  bool timing_on = false;
  bool timing_unread = false;     // the last timed synchronous evaluation is not yet in the totals
  unsigned long long seq = 0;     // sequence number of the last synchronous evaluation
  long long t_count = 0;
  double t_total = 0.0, t_stream = 0.0;


  std::string err;

  ~mipwa_ctx() {
    for (hipEvent_t e : {ev_staged, ev_t0, ev_t1, ev_t2, ev_t3})
      if (e) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
  }

  int fail(int code, const std::string& msg);
  int rebuild_launch();
  int stage_params();
  bool shapes_changed() const;
  int ensure_cache(hipStream_t st);
  int prepare_eval(hipStream_t st);
  int enqueue_kernels(hipStream_t st, bool to_host, bool timed, unsigned long long s = 0, double* out = nullptr);
  size_t upload16() const { return (upload_bytes + 15) / 16 * 16; }
  int wait_result(unsigned long long s);
  int fold_timing();
  int run_sync_eval();
};
