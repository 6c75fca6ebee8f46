// C ABI of libmipwa: contexts, evaluation, integrals, toy generation.  The fit lives in fit.cpp and
// the serving loop in serve.cpp.
#include "mipwa.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <immintrin.h>
#include <string>
#include <vector>

#include "ctx.h"

using namespace mipwa;

#define HIPCHK(expr, what)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return ctx->fail(MIPWA_E_HIP, std::string(what) + ": " + \
                                                             hipGetErrorString(e_)); \
  } while (0)

int mipwa_ctx::fail(int code, const std::string& msg) {
  err = msg;
  return code;
}

namespace {

int default_blocks(int device) {
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  return 2 * cus;
}

}  // namespace

void mipwa_ctx::to_internal(const double* ext, double* in) const {
  const int N = mh.N, R = mh.R;
  if (swave == kSwaveCartesian) {
    for (int k = 0; k < N; ++k) {
      in[2 * k] = std::hypot(ext[2 * k], ext[2 * k + 1]);
      in[2 * k + 1] = std::atan2(ext[2 * k + 1], ext[2 * k]);
    }
    std::copy(ext + 2 * N, ext + mh.P, in + 2 * N);
  } else if (swave == kSwaveIsobar) {
    // c_NR carried by both knots of a two-knot spline at c_NR / 2
    in[0] = in[2] = 0.5 * ext[0];
    in[1] = in[3] = ext[1];
    std::copy(ext + 2, ext + 2 + 4 * R, in + 4);
  } else {
    std::copy(ext, ext + mh.P, in);
  }
}

// Sequence numbers of synchronous evaluations, unique in the process.
static std::atomic<unsigned long long> g_eval_seq{0};

// ---- device descriptors and tables -----------------------------------------------------------

mipwa_ctx::LaunchPlan mipwa_ctx::plan_launch() const {
  LaunchPlan L;
  L.waves = waves_cfg ? waves_cfg : 4;
  if (use_qform()) {
    // the data stream gets the blocks; the cells of the quadratic form a few blocks of ~4 cells per wave
    L.nb_d = std::max(1, std::min(blocks_cfg, std::max(1, ev.n_tiles / (2 * L.waves))));
    L.nb_n = std::min(64, std::max(1, (nm.n_cells + 4 * L.waves - 1) / (4 * L.waves)));
    L.B = L.nb_d + L.nb_n;
  } else {
    const int total_tiles = ev.n_tiles + nm.n_tiles;
    // up to the configured grid, at least one tile per wave: small point sets spread over as many
    // CUs as they have tiles (one tile per wave measured faster than two for 10 k + 100 k points)
    L.B = std::max(2, std::min(blocks_cfg, std::max(2, total_tiles / L.waves)));
    L.nb_d = (int)std::llround((double)L.B * ev.n_tiles / std::max(total_tiles, 1));
    L.nb_d = std::min(std::max(L.nb_d, 1), L.B - 1);
    L.nb_n = L.B - L.nb_d;
  }
  L.rs = record_size(mh.N - 1, mh.R, otf);
  L.G_d = n_groups(L.nb_d);
  L.G_n = n_groups(L.nb_n);
  // bytes the sweep reads per evaluation (coordinates, cached amplitudes, normalisation weights)
  const double real = fp64 ? 8.0 : 4.0;
  double bytes = (double)ev.n * (2 + 2 * mh.R) * real;
  if (!use_qform()) bytes += (double)nm.n * (3 + 2 * mh.R) * real;
  L.parts = otf ? 1 : sweep_parts(bytes);
  return L;
}

void mipwa_ctx::make_segments(const LaunchPlan& L, double* records, Segment sg[2]) const {
  std::memset(sg, 0, 2 * sizeof(Segment));
  const PointSet* ps[2] = {&ev, &nm};
  for (int k = 0; k < 2; ++k) {
    sg[k].tt = ps[k]->tt.p;
    sg[k].ss = ps[k]->ss.p;
    sg[k].w = k ? ps[k]->w.p : nullptr;
    sg[k].cache = ps[k]->cache.p;
    sg[k].tiles = ps[k]->tiles.as<Tile>();
    sg[k].table = use_arg ? nullptr : d_blob.p;
    sg[k].records = records + (size_t)(k ? L.nb_d : 0) * L.rs;
    sg[k].n = ps[k]->n;
    sg[k].n_tiles = ps[k]->n_tiles;
    sg[k].kind = k;
    sg[k].nint = mh.N - 1;
    sg[k].rs = L.rs;
    sg[k].n_blocks = k ? L.nb_n : L.nb_d;
    sg[k].job = 0;
    sg[k].g0 = k ? L.G_d : 0;
  }
}

void mipwa_ctx::make_job(const LaunchPlan& L, double* grec, Job& jb) const {
  std::memset(&jb, 0, sizeof(jb));
  jb.tab64 = use_arg ? nullptr : d_blob.as<double>() + tab64_off / sizeof(double);
  jb.theta_off = arg_theta_off;
  jb.consts = d_blob.as<double>() + consts_off / sizeof(double);
  jb.grec = grec;
  jb.n_ev = (double)ev.n;
  jb.c_eps = ev.c_eps;
  jb.G_d = L.G_d;
  jb.G_n = L.G_n;
  jb.N = mh.N;
  jb.R = mh.R;
  jb.rs = L.rs;
  jb.otf = otf ? 1 : 0;
  jb.swave = swave;
}

int mipwa_ctx::rebuild_launch() {
  mipwa_ctx* ctx = this;
  // the buffers below are replaced: nothing queued, on any stream, may still use them
  if (int rc = drain()) return rc;
  const LaunchPlan L = plan_launch();
  waves_eff = L.waves;
  nb_d = L.nb_d;
  nb_n = L.nb_n;
  n_blocks = L.B;
  rs = L.rs;
  sweep_parts_eff = L.parts;
  const bool qf = use_qform();
  HIPCHK(d_records.alloc((size_t)L.B * L.rs * sizeof(double)), "records allocation");
  HIPCHK(d_grec.alloc((size_t)(L.G_d + L.G_n) * L.rs * sizeof(double)), "group records allocation");
  std::vector<int2> bs(L.B);
  for (int b = 0; b < L.B; ++b) bs[b] = b < L.nb_d ? int2{0, b} : int2{1, b - L.nb_d};
  HIPCHK(d_block_seg.alloc(L.B * sizeof(int2)), "block map allocation");
  HIPCHK(hipMemcpy(d_block_seg.p, bs.data(), L.B * sizeof(int2), hipMemcpyHostToDevice), "block map upload");
  Segment sg[2];
  make_segments(L, d_records.as<double>(), sg);
  std::memcpy(h_segs, sg, sizeof(sg));  // the point streams: cache builds and the moment pass use them
  if (qf) {
    const int K = qform_dim(mh.R);
    HIPCHK(d_mom.alloc((size_t)nm.n_cells * K * K * 2 * sizeof(double)), "moment allocation");
    sg[1].kind = 2;
    sg[1].tiles = nm.cells.as<Tile>();
    sg[1].n_tiles = nm.n_cells;
    sg[1].cache = d_mom.p;
    mom_valid = false;
  }
  HIPCHK(d_segs.alloc(sizeof(sg)), "segment allocation");
  HIPCHK(hipMemcpy(d_segs.p, sg, sizeof(sg), hipMemcpyHostToDevice), "segment upload");
  // job 0 writes the results into mapped pinned host memory (synchronous evaluations), job 1 into
  // device memory (asynchronous evaluations, copied to the caller's buffer on its stream)
  Job jb[2];
  for (int k = 0; k < 2; ++k) make_job(L, d_grec.as<double>(), jb[k]);
  jb[0].out = h_out_dev;
  jb[0].seq_out = reinterpret_cast<unsigned long long*>(h_out_dev + 1 + mh.P);
  jb[1].out = d_out.as<double>();
  jb[1].seq_out = nullptr;
  HIPCHK(hipMemcpy(d_job.p, jb, sizeof(jb), hipMemcpyHostToDevice), "job upload");
  h_jobs[0] = jb[0];
  h_jobs[1] = jb[1];
  h_plan = GroupPlan{};
  for (int k = 0; k < 2; ++k) {
    h_plan.records[k] = sg[k].records;
    h_plan.n_blocks[k] = sg[k].n_blocks;
  }
  h_plan.grec = d_grec.as<double>();
  h_plan.G_d = L.G_d;
  h_plan.G_n = L.G_n;
  h_plan.rs = L.rs;
  launch_dirty = false;
  return MIPWA_OK;
}

int mipwa_ctx::stage_params() {
  mipwa_ctx* ctx = this;
  // wait until the previous upload has left the staging buffer (evaluations whose tables travel in
  // the kernel arguments upload nothing; mipwa_integrals waits for its own upload before returning)
  if (!use_arg) HIPCHK(hipEventSynchronize(ev_staged), "staging wait");
  const size_t tbytes = (size_t)table_real_words(mh.N - 1, mh.R, fp64) * (fp64 ? 8 : 4);
  char* hb = h_blob.as<char>();
  // residues only where the data and the normalisation are both FP32 point sweeps (they keep the same
  // part of them); the quadratic form's FP64 arithmetic would keep all of them, and a normalisation
  // that sees the coefficients otherwise than the data term shifts the fit's minimum
  mh.eval_table(theta.data(), fp64, hb, !use_qform());
  std::memcpy(hb + tab64_off, theta.data(), mh.P * sizeof(double));
  if (use_arg) {
    char* a = reinterpret_cast<char*>(h_args.w);
    std::memcpy(a, hb, tbytes);
    std::memcpy(a + arg_theta_off, theta.data(), mh.P * sizeof(double));
  }
  return MIPWA_OK;
}

bool mipwa_ctx::shapes_changed() const {
  if (!cache_valid) return true;
  for (int p = 2 * mh.N + 2 * mh.R; p < mh.P; ++p)
    if (theta[p] != cache_shape[p - 2 * mh.N - 2 * mh.R]) return true;
  return false;
}

int mipwa_ctx::ensure_cache(hipStream_t st) {
  mipwa_ctx* ctx = this;
  if (!shapes_changed()) return MIPWA_OK;
  // the resonance constants are replaced from the host and the cache rewritten: every evaluation
  // still reading them, on any stream, must have finished
  if (int rc = drain()) return rc;
  HIPCHK(hipStreamSynchronize(st), "stream sync");
  if (int rc = mh.upload_res64(theta.data(), d_res64)) return fail(rc, "resonance constants upload failed");
  PointSet* ps[2] = {&ev, &nm};
  for (int k = 0; k < 2; ++k) {
    if (!ps[k]->loaded) continue;
    HIPCHK(launch_cache(fp64, mh.R, &h_segs[k], d_res64.as<double>(), mh.kin64, st), "resonance cache kernel");
  }
  cache_shape.assign(theta.begin() + 2 * mh.N + 2 * mh.R, theta.end());
  cache_valid = ev.loaded && nm.loaded;
  mom_valid = false;  // the moments hold the normalisation points' resonance amplitudes
  return MIPWA_OK;
}

int mipwa_ctx::order_after_last(hipStream_t st) {
  mipwa_ctx* ctx = this;
  if (last_st != nullptr && last_st != st) HIPCHK(hipStreamWaitEvent(st, ev_done, 0), "stream wait");
  return MIPWA_OK;
}

int mipwa_ctx::drain() {
  mipwa_ctx* ctx = this;
  if (last_st != nullptr) HIPCHK(hipEventSynchronize(ev_done), "event sync");
  HIPCHK(hipStreamSynchronize(stream), "stream sync");
  return MIPWA_OK;
}

int mipwa_ctx::enqueue_kernels(hipStream_t st, bool to_host, bool timed, unsigned long long s, double* out) {
  mipwa_ctx* ctx = this;
  const int cs = ev_cur;
  const int kind = timed ? timing_next_kind : -1;  // 0: step pair, 1: sweep pair
  if (kind == 0) HIPCHK(hipEventRecord(ev_t[cs][0], st), "event");
  if (!use_arg) {
    HIPCHK(launch_upload(d_blob.p, h_blob.dev, upload16(), st), "parameter upload");
    HIPCHK(hipEventRecord(ev_staged, st), "event");
  }
  // with use_arg the table and theta travel in the kernel arguments (copied at the launch)
  HIPCHK(launch_eval(fp64, mh.R, otf, d_segs.as<Segment>(), d_block_seg.as<int2>(), d_job.as<Job>() + (to_host ? 0 : 1),
                     n_blocks, waves_eff, mh.N - 1, fp64 ? (const void*)&mh.kin64 : (const void*)&mh.kin32,
                     use_arg ? &h_args : nullptr, sweep_parts_eff, sweep_order, st, kind == 1 ? ev_t[cs][1] : nullptr,
                     kind == 1 ? ev_t[cs][2] : nullptr),
         "likelihood kernel");
  // the group sums take their layout from h_plan: no task list
  HIPCHK(launch_reduce(d_segs.as<Segment>(), d_job.as<Job>() + (to_host ? 0 : 1), nullptr, 0, 1,
                       use_arg ? &h_args : nullptr, st, s, out, &h_jobs[to_host ? 0 : 1], &h_plan),
         "reduction kernels");
  HIPCHK(hipEventRecord(ev_done, st), "event");
  last_st = st;
  sweep_order ^= 1;
  if (timed) {
    if (kind == 0) HIPCHK(hipEventRecord(ev_t[cs][3], st), "event");
    set_kind[cs] = kind;
    timing_next_kind ^= 1;
    set_unread[cs] = true;
    timing_pending = true;
    ev_last = cs;
    ev_cur = cs ^ 1;
    // the other set holds the previous timed evaluation: take its times now that this one is queued
    int rc = fold_timing(cs ^ 1);
    if (rc) return rc;
  }
  return MIPWA_OK;
}

int mipwa_ctx::prepare_eval(hipStream_t st) {
  if (!ev.loaded || !nm.loaded) return fail(MIPWA_E_STATE, "load events and normalisation points first");
  if (!have_theta) return fail(MIPWA_E_STATE, "set parameters first");
  if (launch_dirty) {
    int rc = rebuild_launch();
    if (rc) return rc;
  }
  int rc = order_after_last(st);
  if (rc) return rc;
  rc = stage_params();
  if (rc) return rc;
  if (!otf && shapes_changed()) {
    rc = ensure_cache(st);
    if (rc) return rc;
  }
  if (use_qform() && !mom_valid) {
    mipwa_ctx* ctx = this;
    HIPCHK(launch_moments(fp64, mh.R, &h_segs[1], nm.cells.as<Tile>(), nm.n_cells, d_mom.as<double>(), st),
           "moment pass");
    mom_valid = true;
  }
  return MIPWA_OK;
}

// Wait for the finish kernel to publish sequence number s after the results in mapped host memory.
// Spinning on that word returns as soon as the results land, without waiting for the stream's
// completion signal; the stream is queried now and then so that a failed launch is still reported.
int mipwa_ctx::wait_result(unsigned long long s) {
  const unsigned long long* word = reinterpret_cast<const unsigned long long*>(h_out.as<double>() + 1 + mh.P);
  for (unsigned long long it = 1;; ++it) {
    if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == s) return MIPWA_OK;
    if ((it & 1023) == 0) {
      const hipError_t q = hipStreamQuery(stream);
      if (q == hipSuccess) {
        if (__atomic_load_n(word, __ATOMIC_ACQUIRE) == s) return MIPWA_OK;
        return fail(MIPWA_E_HIP, "the evaluation ended without publishing its result");
      }
      if (q != hipErrorNotReady) return fail(MIPWA_E_HIP, std::string("evaluation failed: ") + hipGetErrorString(q));
    }
    _mm_pause();
  }
}

int mipwa_ctx::fold_timing(int set) {
  mipwa_ctx* ctx = this;
  if (!set_unread[set]) return MIPWA_OK;
  set_unread[set] = false;
  const bool step = set_kind[set] == 0;
  hipEvent_t e0 = step ? ev_t[set][0] : ev_t[set][1], e1 = step ? ev_t[set][3] : ev_t[set][2];
  HIPCHK(hipEventSynchronize(e1), "event sync");
  float a = 0;
  if (hipEventElapsedTime(&a, e0, e1) == hipSuccess) {
    if (step) {
      t_count_step += 1;
      t_total += a;
    } else {
      t_count_sweep += 1;
      t_stream += a;
    }
  }
  (void)hipGetLastError();
  return MIPWA_OK;
}

int mipwa_ctx::fold_all_timing() {
  for (int k = 0; k < 2; ++k)
    if (int rc = fold_timing(ev_cur ^ 1 ^ k)) return rc;
  return MIPWA_OK;
}

int mipwa_ctx::run_sync_eval() {
  int rc = prepare_eval(stream);
  if (rc) return rc;
  // numbers are unique in the process: pinned memory handed back by a destroyed context may still
  // hold one of its sequence numbers
  const unsigned long long s = seq = g_eval_seq.fetch_add(1, std::memory_order_relaxed) + 1;
  rc = enqueue_kernels(stream, true, take_timing(), s);
  if (rc) return rc;
  return wait_result(s);
}

// ---- C ABI -----------------------------------------------------------------------------------

extern "C" {

const char* mipwa_strerror(int s) {
  switch (s) {
    case MIPWA_OK: return "ok";
    case MIPWA_E_INVAL: return "invalid argument";
    case MIPWA_E_NOMEM: return "out of memory or over budget";
    case MIPWA_E_HIP: return "HIP runtime error";
    case MIPWA_E_STATE: return "call out of order";
    case MIPWA_E_DOMAIN: return "non-finite likelihood";
    case MIPWA_E_NOCONV: return "fit did not converge";
    case MIPWA_E_CANCELLED: return "cancelled";
    case MIPWA_E_BUSY: return "no result yet";
    default: return "unknown status";
  }
}

int mipwa_create(const mipwa_model* model, int precision, int device, mipwa_ctx** out) {
  if (!out) return MIPWA_E_INVAL;
  *out = nullptr;
  if (precision != MIPWA_FP64 && precision != MIPWA_MIXED) return MIPWA_E_INVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MIPWA_E_HIP;
  if (device < 0 || device >= ndev) return MIPWA_E_INVAL;
  mipwa_ctx* ctx = new (std::nothrow) mipwa_ctx();
  if (!ctx) return MIPWA_E_NOMEM;
  ctx->device = device;
  ctx->fp64 = precision == MIPWA_FP64;
  std::string err;
  int rc = ctx->mh.init(model, err);
  if (rc) {
    delete ctx;
    return rc;
  }
  if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
    delete ctx;
    return MIPWA_E_HIP;
  }
  bool events_ok = hipEventCreate(&ctx->ev_staged) == hipSuccess &&
                   hipEventCreateWithFlags(&ctx->ev_done, hipEventDisableTiming) == hipSuccess;
  for (auto& set : ctx->ev_t)
    for (hipEvent_t& e : set) events_ok = events_ok && hipEventCreate(&e) == hipSuccess;
  if (!events_ok) {
    delete ctx;
    return MIPWA_E_HIP;
  }
  const mipwa::ModelHost& mh = ctx->mh;
  const size_t real = ctx->fp64 ? 8 : 4;
  const size_t tbytes = table_real_words(mh.N - 1, mh.R, ctx->fp64) * real;
  ctx->tab64_off = (tbytes + 255) / 256 * 256;
  ctx->upload_bytes = ctx->tab64_off + mh.P * sizeof(double);
  ctx->consts_off = ctx->upload16();  // the per-evaluation upload never reaches the constants
  ctx->arg_theta_off = (int)((tbytes + 7) / 8 * 8);
  ctx->use_arg = ctx->arg_theta_off + mh.P * sizeof(double) <= (size_t)kArgBytes;
  const size_t blob = ctx->consts_off + (size_t)consts_words(mh.N) * sizeof(double);
  if (ctx->d_blob.alloc(blob) != hipSuccess || ctx->h_blob.alloc(ctx->upload16(), true) != hipSuccess ||
      ctx->d_out.alloc((1 + mh.P) * sizeof(double)) != hipSuccess ||
      ctx->h_out.alloc((2 + mh.P) * sizeof(double), true) != hipSuccess ||
      hipHostGetDevicePointer((void**)&ctx->h_out_dev, ctx->h_out.p, 0) != hipSuccess ||
      ctx->d_job.alloc(2 * sizeof(Job)) != hipSuccess) {
    delete ctx;
    return MIPWA_E_NOMEM;
  }
  std::memset(ctx->h_out.p, 0, (2 + mh.P) * sizeof(double));
  // constant part of the FP64 table (at consts_off): Thomas factors of the interior spline system, h
  const int ni = mh.N - 2;
  std::vector<double> cst(consts_words(mh.N));
  for (int i = 0; i < ni; ++i) {
    cst[i] = mh.th_c[i];
    cst[ni + i] = 1.0 / mh.th_d[i];
  }
  std::copy(mh.h.begin(), mh.h.end(), cst.begin() + 2 * ni);
  if (hipMemcpy(ctx->d_blob.as<char>() + ctx->consts_off, cst.data(),
                cst.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    delete ctx;
    return MIPWA_E_HIP;
  }
  ctx->fixed.assign(mh.P, 0);
  for (int p = 2 * mh.N + 2 * mh.R; p < mh.P; ++p) ctx->fixed[p] = 1;
  ctx->blocks_cfg = default_blocks(device);
  ctx->waves_cfg = 0;
  *out = ctx;
  return MIPWA_OK;
}

void mipwa_destroy(mipwa_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)ctx->drain();
  delete ctx;
}

const char* mipwa_last_error(const mipwa_ctx* ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

int mipwa_n_params(const mipwa_ctx* ctx) { return ctx ? ctx->ext_P() : MIPWA_E_INVAL; }

int mipwa_set_norm_mode(mipwa_ctx* ctx, int mode) {
  if (!ctx) return MIPWA_E_INVAL;
  if (mode != MIPWA_NORM_POINTS && mode != MIPWA_NORM_QFORM) return ctx->fail(MIPWA_E_INVAL, "unknown mode");
  ctx->qform = mode == MIPWA_NORM_QFORM;
  ctx->launch_dirty = true;
  ctx->mom_valid = false;
  return MIPWA_OK;
}

int mipwa_set_swave_form(mipwa_ctx* ctx, int form) {
  if (!ctx) return MIPWA_E_INVAL;
  if (form != MIPWA_SWAVE_POLAR && form != MIPWA_SWAVE_CARTESIAN && form != MIPWA_SWAVE_ISOBAR)
    return ctx->fail(MIPWA_E_INVAL, "unknown S-wave form");
  if (form == MIPWA_SWAVE_ISOBAR && ctx->mh.N != 2)
    return ctx->fail(MIPWA_E_INVAL, "the isobar form needs a model with exactly two knots");
  ctx->swave = form;
  ctx->have_theta = false;
  const int P = ctx->ext_P(), o = ctx->ext_res_off() + 2 * ctx->mh.R;
  ctx->fixed.assign(P, 0);
  for (int p = o; p < P; ++p) ctx->fixed[p] = 1;
  ctx->otf = false;
  ctx->launch_dirty = true;
  return MIPWA_OK;
}

int mipwa_set_launch(mipwa_ctx* ctx, int blocks, int waves) {
  if (!ctx) return MIPWA_E_INVAL;
  if (blocks < 0 || waves < 0 || waves > 8) return ctx->fail(MIPWA_E_INVAL, "waves per block must be 1..8");
  ctx->blocks_cfg = blocks ? blocks : default_blocks(ctx->device);
  ctx->waves_cfg = waves;  // 0: 4 waves per block
  ctx->launch_dirty = true;
  return MIPWA_OK;
}

int mipwa_set_eff_table(mipwa_ctx* ctx, const float* table, int nx, int ny, double lo, double hi) {
  if (!ctx) return MIPWA_E_INVAL;
  if (!table || nx < 2 || ny < 2 || !(hi > lo)) return ctx->fail(MIPWA_E_INVAL, "efficiency table needs nx, ny >= 2, hi > lo");
  for (long i = 0; i < (long)nx * ny; ++i)
    if (!(table[i] > 0) || !std::isfinite(table[i]))
      return ctx->fail(MIPWA_E_INVAL, "efficiency table values must be positive");
  (void)hipSetDevice(ctx->device);
  // the device copy is made first and the table replaced only once it is complete: a failed call
  // leaves the previous table (or none) in force, never sizes that do not match the device buffer
  DevBuf d;
  HIPCHK(d.alloc((size_t)nx * ny * sizeof(float)), "efficiency table allocation");
  HIPCHK(hipMemcpy(d.p, table, (size_t)nx * ny * sizeof(float), hipMemcpyHostToDevice), "efficiency table upload");
  ctx->eff.tab.assign(table, table + (size_t)nx * ny);
  ctx->eff.nx = nx;
  ctx->eff.ny = ny;
  ctx->eff.lo = lo;
  ctx->eff.hi = hi;
  ctx->eff.d = std::move(d);
  return MIPWA_OK;
}

int mipwa_load_events(mipwa_ctx* ctx, const double* s12, const double* s13, const double* eff, int64_t n) {
  if (!ctx) return MIPWA_E_INVAL;
  (void)hipSetDevice(ctx->device);
  if (int rc = ctx->drain()) return rc;
  int rc = load_points(ctx->mh, ctx->fp64, 0, s12, s13, nullptr, eff, n, ctx->eff, ctx->stream, ctx->ev, ctx->err);
  ctx->cache_valid = false;
  ctx->launch_dirty = true;
  return rc;
}

int mipwa_load_norm(mipwa_ctx* ctx, const double* s12, const double* s13, const double* w, const double* eff,
                    int64_t n) {
  if (!ctx) return MIPWA_E_INVAL;
  (void)hipSetDevice(ctx->device);
  if (int rc = ctx->drain()) return rc;
  int rc = load_points(ctx->mh, ctx->fp64, 1, s12, s13, w, eff, n, ctx->eff, ctx->stream, ctx->nm, ctx->err);
  ctx->cache_valid = false;
  ctx->launch_dirty = true;
  return rc;
}

int mipwa_set_fixed(mipwa_ctx* ctx, const unsigned char* fixed, int n) {
  if (!ctx) return MIPWA_E_INVAL;
  if (!fixed || n != ctx->ext_P()) return ctx->fail(MIPWA_E_INVAL, "fixed mask must have P entries");
  ctx->fixed.assign(fixed, fixed + n);
  bool otf = false;
  for (int p = ctx->ext_res_off() + 2 * ctx->mh.R; p < n; ++p) otf |= fixed[p] == 0;
  if (otf != ctx->otf) {
    ctx->otf = otf;
    ctx->launch_dirty = true;
  }
  return MIPWA_OK;
}

int mipwa_set_params(mipwa_ctx* ctx, const double* theta, int n) {
  if (!ctx) return MIPWA_E_INVAL;
  if (!theta || n != ctx->ext_P()) return ctx->fail(MIPWA_E_INVAL, "theta must have P entries");
  for (int p = 0; p < n; ++p)
    if (!std::isfinite(theta[p])) return ctx->fail(MIPWA_E_INVAL, "theta has a non-finite entry");
  std::vector<double> in(ctx->mh.P);
  ctx->to_internal(theta, in.data());
  int rc = ctx->mh.check_theta(in.data(), ctx->err);
  if (rc) return rc;
  ctx->theta.swap(in);
  ctx->have_theta = true;
  return MIPWA_OK;
}

int mipwa_eval(mipwa_ctx* ctx, double* nll, double* grad) {
  if (!ctx) return MIPWA_E_INVAL;
  (void)hipSetDevice(ctx->device);
  int rc = ctx->run_sync_eval();
  if (rc) return rc;
  const double* o = ctx->h_out.as<double>();
  if (nll) *nll = o[0];
  if (grad) std::memcpy(grad, o + 1, ctx->ext_P() * sizeof(double));
  if (!std::isfinite(o[0])) {
    if (nll) *nll = INFINITY;
    return ctx->fail(MIPWA_E_DOMAIN, "-2 ln L is not finite (|A|^2 = 0 at an event?)");
  }
  return MIPWA_OK;
}

int mipwa_eval_async(mipwa_ctx* ctx, void* stream, double* d_out) {
  if (!ctx) return MIPWA_E_INVAL;
  if (!d_out) return ctx->fail(MIPWA_E_INVAL, "d_out is NULL");
  (void)hipSetDevice(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = ctx->prepare_eval(st);
  if (rc) return rc;
  return ctx->enqueue_kernels(st, false, ctx->take_timing(), 0, d_out);
}

int mipwa_last_timing(const mipwa_ctx* cctx, double* total_ms, double* stream_ms) {
  mipwa_ctx* ctx = const_cast<mipwa_ctx*>(cctx);
  if (!ctx) return MIPWA_E_INVAL;
  if (!ctx->timing_pending) return ctx->fail(MIPWA_E_STATE, "no evaluation timed yet");
  // the two sets hold the last two timed evaluations, one of each pair when both exist
  double v[2] = {NAN, NAN};
  for (int k = 0; k < 2; ++k) {
    const int set = ctx->ev_last ^ k;
    if (k == 1 && ctx->set_kind[set] == ctx->set_kind[ctx->ev_last]) break;
    const bool step = ctx->set_kind[set] == 0;
    hipEvent_t e0 = step ? ctx->ev_t[set][0] : ctx->ev_t[set][1], e1 = step ? ctx->ev_t[set][3] : ctx->ev_t[set][2];
    float a = 0;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&a, e0, e1) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    v[step ? 0 : 1] = a;
  }
  if (total_ms) *total_ms = v[0];
  if (stream_ms) *stream_ms = v[1];
  return MIPWA_OK;
}

int mipwa_set_timing(mipwa_ctx* ctx, int period) {
  if (!ctx) return MIPWA_E_INVAL;
  if (period < 0) return ctx->fail(MIPWA_E_INVAL, "the timing period must be >= 0");
  if (int rc = ctx->fold_all_timing()) return rc;  // finish with the events still in use
  ctx->timing_period = period;
  ctx->timing_calls = 0;
  ctx->timing_next_kind = 0;
  ctx->set_unread[0] = ctx->set_unread[1] = false;
  ctx->t_count_step = ctx->t_count_sweep = 0;
  ctx->t_total = ctx->t_stream = 0.0;
  return MIPWA_OK;
}

int mipwa_timing_stats(const mipwa_ctx* ctx, int64_t* count, double* mean_total_ms, double* mean_stream_ms) {
  if (!ctx) return MIPWA_E_INVAL;
  if (int rc = const_cast<mipwa_ctx*>(ctx)->fold_all_timing()) return rc;
  if (count) *count = ctx->t_count_step + ctx->t_count_sweep;
  if (mean_total_ms) *mean_total_ms = ctx->t_count_step ? ctx->t_total / ctx->t_count_step : NAN;
  if (mean_stream_ms) *mean_stream_ms = ctx->t_count_sweep ? ctx->t_stream / ctx->t_count_sweep : NAN;
  return MIPWA_OK;
}

int mipwa_integrals(mipwa_ctx* ctx, int with_eff, double* Ijk) {
  if (!ctx) return MIPWA_E_INVAL;
  if (!Ijk) return ctx->fail(MIPWA_E_INVAL, "Ijk is NULL");
  if (!ctx->nm.loaded) return ctx->fail(MIPWA_E_STATE, "load normalisation points first");
  if (!ctx->have_theta) return ctx->fail(MIPWA_E_STATE, "set parameters first");
  (void)hipSetDevice(ctx->device);
  hipStream_t st = ctx->stream;
  // the normalisation cache is rewritten below: evaluations still reading it must finish first
  if (int rc = ctx->drain()) return rc;
  if (ctx->launch_dirty && ctx->ev.loaded) {
    int rc = ctx->rebuild_launch();
    if (rc) return rc;
  }
  int rc = ctx->stage_params();
  if (rc) return rc;
  HIPCHK(launch_upload(ctx->d_blob.p, ctx->h_blob.dev, ctx->upload16(), st), "upload");
  HIPCHK(hipEventRecord(ctx->ev_staged, st), "event");
  // the normalisation segment with its cache valid at the current shapes
  Segment sg;
  std::memset(&sg, 0, sizeof(sg));
  sg.tt = ctx->nm.tt.p;
  sg.ss = ctx->nm.ss.p;
  sg.w = ctx->nm.w.p;
  sg.cache = ctx->nm.cache.p;
  sg.tiles = ctx->nm.tiles.as<Tile>();
  sg.table = ctx->d_blob.p;
  sg.n = ctx->nm.n;
  sg.n_tiles = ctx->nm.n_tiles;
  sg.kind = 1;
  sg.nint = ctx->mh.N - 1;
  if (int rc2 = ctx->mh.upload_res64(ctx->theta.data(), ctx->d_res64)) return ctx->fail(rc2, "resonance constants upload");
  HIPCHK(launch_cache(ctx->fp64, ctx->mh.R, &sg, ctx->d_res64.as<double>(), ctx->mh.kin64, st), "resonance cache kernel");
  ctx->cache_valid = false;  // the event cache was not rebuilt for these shapes
  const int K = ctx->mh.R + 1;
  const int nb = std::max(1, std::min(1024, (ctx->nm.n_tiles + 3) / 4));
  DevBuf rec, out;
  HIPCHK(rec.alloc((size_t)nb * 2 * K * K * sizeof(double)), "integral records");
  HIPCHK(out.alloc(2 * K * K * sizeof(double)), "integral output");
  HIPCHK(launch_integrals(ctx->fp64, ctx->mh.R, &sg, with_eff ? ctx->nm.w.p : ctx->nm.wplain.p, rec.as<double>(), nb,
                          out.as<double>(), st),
         "integral kernel");
  HIPCHK(hipStreamSynchronize(st), "stream sync");
  HIPCHK(hipMemcpy(Ijk, out.p, 2 * K * K * sizeof(double), hipMemcpyDeviceToHost), "integral copy");
  return MIPWA_OK;
}

int mipwa_fit_fractions(mipwa_ctx* ctx, double* ff) {
  if (!ctx) return MIPWA_E_INVAL;
  if (!ff) return ctx->fail(MIPWA_E_INVAL, "ff is NULL");
  const int K = ctx->mh.R + 1, N = ctx->mh.N;
  std::vector<double> I(2 * K * K);
  int rc = mipwa_integrals(ctx, 0, I.data());
  if (rc) return rc;
  std::vector<double> cr(K), ci(K);
  cr[0] = 1.0;
  ci[0] = 0.0;
  for (int r = 0; r < ctx->mh.R; ++r) {
    const double m = ctx->theta[2 * N + 2 * r], a = ctx->theta[2 * N + 2 * r + 1];
    cr[r + 1] = m * std::cos(a);
    ci[r + 1] = m * std::sin(a);
  }
  double tot = 0.0;
  for (int j = 0; j < K; ++j)
    for (int k = 0; k < K; ++k) {
      // Re(c_j conj(c_k) I_jk)
      const double pr = cr[j] * cr[k] + ci[j] * ci[k], pi = ci[j] * cr[k] - cr[j] * ci[k];
      const double v = pr * I[2 * (j * K + k)] - pi * I[2 * (j * K + k) + 1];
      ff[j * K + k] = v;
      tot += v;
    }
  for (int i = 0; i < K * K; ++i) ff[i] /= tot;
  return MIPWA_OK;
}

}  // extern "C"
