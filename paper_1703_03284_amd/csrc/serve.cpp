// Toy-fit serving with continuous batching.
//
// Each submitted job is a maximum-likelihood fit (the fit of Sec. 2 / Sec. 4 on a toy sample) of its
// own events against a normalisation sample shared by the server.  Jobs wait in a queue until their
// device footprint fits the HBM budget; an admitted job's thread loads its events (cell sort,
// resonance cache) on one of a few loader streams, taken first come first served, then runs the BFGS
// fit.  The normalisation points are cell-sorted once per knot grid and shared, and so are their
// per-cell moments at each set of resonance shapes (formed by the first job that needs them); with the
// shapes fixed, each evaluation takes the normalisation integral as a quadratic form over those
// moments instead of a sweep over the points.  Device memory comes from a pool owned by the server
// and goes back to it in stream order, without waiting for the device.  Every evaluation a job asks
// for is posted to the scheduler, which gathers the pending evaluations of active jobs into one launch
// of the streaming kernel (one data segment and one cell segment per job).  Up to two such steps are
// in flight on the server's stream, so that one group of jobs computes its next points while the
// other's step runs.  A job's block count depends only on its own sizes and every job is swept in one
// part, so its reduction order, and therefore its result, is bitwise the same alone or in any mix.
#include <hip/hip_runtime.h>
#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.h"
#include "host.h"
#include "minimizer.h"
#include "mipwa.h"

using namespace mipwa;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int kServeWaves = 4;
constexpr int kServeTilesPerWave = 8;
constexpr int kMaxSegBlocks = 512;
constexpr int kBatchWindowUs = 50;
// odd: consecutive steps alternate between two groups of jobs, so an even period would time one group only
constexpr int kStepTimingPeriod = 17;
constexpr size_t kBatchBytes0 = (size_t)4 << 20;   // initial step descriptor buffer (host and device)
constexpr size_t kResultBytes0 = (size_t)1 << 20;  // initial result buffer (mapped host memory)
constexpr size_t kSeqBytes0 = (size_t)64 << 10;    // initial sequence words: 8192 jobs per step
constexpr int kLoadStreams = 4;                    // streams the jobs' loads are spread over

// Sequence numbers of serving steps, unique in the process: pinned memory handed back by a destroyed
// server may still hold one of its numbers.
std::atomic<unsigned long long> g_step_seq{0};

// The server's own copy of a job's events (the caller may free its arrays once submit returns), s12
// then s13 in one block, left uninitialised until the copy.  Copying into freshly allocated memory
// is bound by first-touch page faults, which proceed in parallel: large submissions are copied by
// several threads.  (Huge pages made these copies faster but the loads' uploads from them slower.)
double* alloc_events(long long n) { return new (std::nothrow) double[(size_t)2 * n]; }

void copy_events(double* d12, double* d13, const double* s12, const double* s13, long long n) {
  constexpr long long kPerThread = 1 << 20;  // events (16 MB of both coordinates)
  const int T = (int)std::min<long long>(8, std::max<long long>(1, n / kPerThread));
  auto part = [&](int t) {
    const long long a = n * t / T, b = n * (t + 1) / T;
    std::memcpy(d12 + a, s12 + a, (size_t)(b - a) * sizeof(double));
    std::memcpy(d13 + a, s13 + a, (size_t)(b - a) * sizeof(double));
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) {
    try {
      th.emplace_back(part, t);
    } catch (...) {
      part(t);  // no thread to spare: this part on the caller's thread
    }
  }
  part(0);
  for (auto& x : th) x.join();
}

// blocks of a job's event segment: about kServeTilesPerWave tiles per wave
int seg_blocks(int n_tiles) {
  const int per_block = kServeTilesPerWave * kServeWaves;
  const int b = (n_tiles + per_block - 1) / per_block;
  return std::min(std::max(b, 1), kMaxSegBlocks);
}

// Per-cell moments of a normalisation set's points at one set of resonance shapes: the normalisation
// integral as a quadratic form.  The first job that needs them forms them; every job with the same
// knots and shapes then uses the same buffer (the moments are the same numbers whichever job forms
// them, so a job's results do not depend on which one did).
struct Moments {
  std::mutex m;  // held while the moments are formed
  bool ready = false;
  DevBuf d;
};

// The shared normalisation sample sorted for one knot grid: local spline coordinates, weights and
// tiles, and its moments for each set of resonance shapes the jobs have asked for.
struct NormSet {
  std::vector<double> key;  // kinematics and knots
  PointSet ps;              // no resonance cache of its own
  int nb = 0;
  size_t bytes = 0;
  std::mutex mom_mu;        // the map below
  std::map<std::vector<double>, std::unique_ptr<Moments>> moments;  // by resonance constants
};

enum JobState { QUEUED, LOADING, ACTIVE, FINISHED };

struct SJob {
  int64_t id = 0;
  ModelHost mh;
  std::unique_ptr<double[]> ev_host;  // the server's copy of the events (s12 then s13), until loaded
  const double* ev12 = nullptr;       // the events to load: the copy, or the caller's borrowed arrays
  const double* ev13 = nullptr;
  long long n = 0;
  std::vector<double> theta0;
  std::vector<unsigned char> fixed;
  double tol = 1e-4;
  int max_iter = 1000;
  bool hessian = false;
  PointSet ev;
  NormSet* norm = nullptr;
  int nb_d = 0, G_d = 0, G_n = 0, rs = 0;
  DevBuf d_rec, d_grec, d_consts, d_tab;
  const void* mom = nullptr;  // per-cell moments of the normalisation points at this job's shapes
  int nb_q = 0;     // blocks of the job's normalisation (cell) segment
  size_t bytes = 0;
  JobState state = QUEUED;
  bool retired = false;  // FINISHED and its memory returned: the worker thread is about to end
  int status = MIPWA_OK;
  std::atomic<bool> cancel{false};
  std::string err;
  Clock::time_point t_submit, t_done;
  std::thread worker;
  // One outstanding evaluation request.  req and inflight are guarded by the server's mutex (the
  // scheduler forms batches under it); done, and the hand-over of staged and of the results, by the
  // job's own mutex m, so that returning the results of a step takes no server-wide lock.
  bool req = false, inflight = false, done = false;
  std::vector<char> staged;  // [Real table | pad to 256 | theta (P doubles)]
  double f = 0;
  std::vector<double> g;
  int step_rc = 0;        // non-zero: the step that carried this job's evaluation failed
  std::string step_err;   // and why
  std::mutex m;
  std::condition_variable cv;
  FitOut result;
  int load_slot = -1;               // the loader stream handed to this job (guarded by the server's load_mu)
  std::condition_variable load_cv;  // signalled when it is handed one, or the server stops
};

std::vector<double> norm_key(const ModelHost& mh) {
  std::vector<double> k = {mh.M, mh.m1, mh.m2, mh.m3, mh.rD, (double)mh.N};
  k.insert(k.end(), mh.knots.begin(), mh.knots.end());
  return k;
}

size_t staged_bytes(const ModelHost& mh, bool fp64, size_t* theta_off) {
  const size_t t = table_real_words(mh.N - 1, mh.R, fp64) * (fp64 ? 8 : 4);
  *theta_off = (t + 255) / 256 * 256;
  return *theta_off + (size_t)mh.P * 8;
}

// evaluation table (working precision) and theta (FP64) for one job at theta
void stage(const ModelHost& mh, bool fp64, const double* theta, std::vector<char>& out) {
  size_t toff = 0;
  out.assign(staged_bytes(mh, fp64, &toff), 0);
  // no residues: the normalisation is a quadratic form in FP64, the data a sweep in FP32, and both
  // must see the same coefficients (see the context's staging)
  mh.eval_table(theta, fp64, out.data(), false);
  std::memcpy(out.data() + toff, theta, (size_t)mh.P * 8);
}

Segment cache_segment(const PointSet& ps, int nint) {
  Segment sg;
  std::memset(&sg, 0, sizeof(sg));
  sg.ss = ps.ss.p;
  sg.cache = ps.cache.p;
  sg.n = ps.n;
  sg.nint = nint;
  return sg;
}

}  // namespace

struct mipwa_server {
  int device = 0;
  bool fp64 = false;
  size_t budget = 0;
  hipStream_t stream = nullptr;
  // Device memory of the jobs and the normalisation sets: a stream-ordered pool that keeps what is
  // freed, so that loading and retiring jobs neither waits for the device (as a plain free does,
  // stalling every other job's loads and the steps' launches) nor hands memory back to the HIP runtime.
  // A job's memory is freed in the order of `stream`, after every step that may use it.
  hipMemPool_t pool = nullptr;
  // Loads run one per loader stream at a time, in about the order jobs are admitted: many loads at
  // once (each uploading its events from pageable host memory) slow every one of them down.
  hipStream_t load_st[kLoadStreams] = {};
  std::mutex load_mu;                 // the two members below and the jobs' load_slot
  bool load_busy[kLoadStreams] = {};
  std::deque<SJob*> load_wait;        // jobs waiting for a loader stream, first come first served
  // Serving sweeps every job in one part (launch_eval): the part count changes the rounding of a
  // job's sums, and a job's result must not depend on the other jobs of its steps.
  int sweep_order = 0;
  std::mutex mu;       // all job and queue state
  std::mutex norm_mu;  // creation of shared normalisation sets
  std::condition_variable cv_sched, cv_done;
  std::thread sched;
  std::atomic<bool> stop{false};
  std::vector<double> n12, n13, nw;
  std::vector<std::unique_ptr<NormSet>> norms;
  std::map<int64_t, std::unique_ptr<SJob>> jobs;
  std::deque<SJob*> queue;
  int64_t next_id = 1;
  size_t used = 0, peak = 0;
  int running = 0;  // LOADING + ACTIVE
  int n_active = 0;  // ACTIVE: jobs that ask for evaluations
  int n_req = 0;     // ACTIVE jobs with a request not yet taken into a batch
  int n_inflight = 0;  // jobs whose evaluation is in a step in flight
  long long steps = 0;
  double batch_sum = 0;
  // scheduler time (s): idle until a request, in the batching window, staging the step, on the GPU
  // and handing results back to the jobs' threads, admitting jobs and joining finished ones
  double t_idle = 0, t_window = 0, t_stage = 0, t_gpu = 0, t_wake = 0, t_admit = 0;
  long long n_overlapped = 0;  // steps launched while the previous step was still in flight
  bool any_submit = false;
  Clock::time_point t_first_submit, t_last_done, t_create = Clock::now();
  std::vector<double> latencies;
  // Buffers of a step: descriptors (pinned host memory, copied to the device by the step's first
  // kernel), results and one sequence word per job (mapped host memory: the finish stores the step's
  // sequence number after a job's results, and the scheduler polls it).  Two sets, used by
  // alternate steps, so that a step can be formed while the previous one runs.
  struct StepBufs {
    HostBuf h_batch, h_res, h_seq;
    DevBuf d_batch;
    double* h_res_dev = nullptr;
    unsigned long long* h_seq_dev = nullptr;
  } bufs[2];
  int next_buf = 0;
  // device time of every kStepTimingPeriod-th step (a pair of events around its kernels); the events
  // and the figures below are guarded by timing_mu (the scheduler records, mipwa_server_stats reads)
  std::mutex timing_mu;
  hipEvent_t ev_step[2] = {nullptr, nullptr};
  bool step_timed_unread = false;
  long long n_step_timed = 0;
  double step_dev_ms = 0.0;
  std::string err;

  // err is written by the callers' threads and by the scheduler: under its own lock
  mutable std::mutex err_mu;
  int fail(int code, const std::string& m) {
    std::lock_guard<std::mutex> g(err_mu);
    err = m;
    return code;
  }
  std::string last_error() const {
    std::lock_guard<std::mutex> g(err_mu);
    return err;
  }
};

static void serve_worker(mipwa_server* S, SJob* J);

namespace {

// Event trace on stderr when MIPWA_SERVE_TRACE is set: job admission, end of loading, completion,
// and every 256th batched step (seconds since the server was created).
bool trace_on() {
  static const bool on = std::getenv("MIPWA_SERVE_TRACE") != nullptr;
  return on;
}

void trace(const mipwa_server* S, const char* fmt, ...) {
  if (!trace_on()) return;
  char msg[256];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[serve %.4f] %s\n", std::chrono::duration<double>(Clock::now() - S->t_create).count(), msg);
}

// Wake a job's worker after setting one of the flags its wait checks (cancel, stop or done).
void wake(SJob* J) {
  { std::lock_guard<std::mutex> jl(J->m); }
  J->cv.notify_all();
}

void admit(mipwa_server* S) {
  while (!S->queue.empty()) {
    SJob* J = S->queue.front();
    if (J->cancel) {
      S->queue.pop_front();
      J->state = FINISHED;
      J->status = MIPWA_E_CANCELLED;
      S->cv_done.notify_all();
      continue;
    }
    if (S->running > 0 && S->used + J->bytes > S->budget) break;
    S->queue.pop_front();
    S->used += J->bytes;
    S->peak = std::max(S->peak, S->used);
    S->running += 1;
    J->state = LOADING;
    trace(S, "admit job %lld: %lld events, %d knots, used %.2f GB", (long long)J->id, J->n, J->mh.N, S->used / 1e9);
    J->worker = std::thread(serve_worker, S, J);
  }
}

NormSet* get_norm(mipwa_server* S, const ModelHost& mh, hipStream_t st, std::string& err, int& rc) {
  std::lock_guard<std::mutex> g(S->norm_mu);
  const std::vector<double> key = norm_key(mh);
  for (auto& ns : S->norms)
    if (ns->key == key) return ns.get();
  auto ns = std::make_unique<NormSet>();
  ns->key = key;
  EffTable none;
  rc = load_points(mh, S->fp64, 1, S->n12.data(), S->n13.data(), S->nw.data(), nullptr, (long long)S->n12.size(),
                   none, st, ns->ps, err, S->pool, S->stream);
  if (rc) return nullptr;
  ns->ps.cache.release();
  const size_t real = S->fp64 ? 8 : 4;
  ns->nb = seg_blocks(ns->ps.n_tiles);
  ns->bytes = (size_t)ns->ps.n * (4 * real + 16) + (size_t)ns->ps.n_tiles * sizeof(Tile);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->used += ns->bytes;
    S->peak = std::max(S->peak, S->used);
  }
  S->norms.push_back(std::move(ns));
  return S->norms.back().get();
}

void finish_job(mipwa_server* S, SJob* J, int status, const std::string& err) {
  // the result first: no step uses the job any more, and returning its memory (below) takes a while
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (J->state == ACTIVE) S->n_active -= 1;
    if (J->req) {
      J->req = false;
      S->n_req -= 1;
    }
    J->state = FINISHED;
    J->status = status;
    J->err = err;
    J->t_done = Clock::now();
    trace(S, "job %lld done: status %d, %d evaluations", (long long)J->id, status, J->result.n_eval);
    if (status == MIPWA_OK || status == MIPWA_E_NOCONV) {
      S->latencies.push_back(std::chrono::duration<double>(J->t_done - J->t_submit).count());
      S->t_last_done = J->t_done;
    }
    S->cv_done.notify_all();
  }
  // then its device memory, back to the pool after the steps already queued, and its share of the budget
  J->ev = PointSet();
  J->d_rec.release();
  J->d_grec.release();
  J->d_consts.release();
  std::lock_guard<std::mutex> lk(S->mu);
  S->used -= J->bytes;
  S->running -= 1;
  J->retired = true;  // the scheduler joins the worker (under the server's lock) only from here on
  S->cv_sched.notify_all();
}

}  // namespace

static void serve_worker(mipwa_server* S, SJob* J) {
  (void)hipSetDevice(S->device);
  int slot = -1;
  {
    std::unique_lock<std::mutex> g(S->load_mu);
    for (int i = 0; i < kLoadStreams && S->load_wait.empty(); ++i)
      if (!S->load_busy[i]) {
        slot = i;
        S->load_busy[i] = true;
        break;
      }
    if (slot < 0) {
      S->load_wait.push_back(J);
      J->load_cv.wait(g, [&] { return J->load_slot >= 0 || S->stop.load(); });
      slot = J->load_slot;
      if (slot < 0) S->load_wait.erase(std::find(S->load_wait.begin(), S->load_wait.end(), J));
    }
  }
  if (slot < 0) {
    finish_job(S, J, MIPWA_E_CANCELLED, "the server is shutting down");
    return;
  }
  hipStream_t st = S->load_st[slot];
  std::string err;
  EffTable none;
  int rc = load_points(J->mh, S->fp64, 0, J->ev12, J->ev13, nullptr, nullptr, J->n, none, st, J->ev, err,
                       S->pool, S->stream);
  J->ev_host.reset();
  J->ev12 = J->ev13 = nullptr;
  NormSet* ns = nullptr;
  if (!rc) ns = get_norm(S, J->mh, st, err, rc);
  if (!rc) {
    // resonance caches of the events and of the shared normalisation points at the job's (fixed)
    // shapes; per-job reduction scratch
    Segment sg = cache_segment(J->ev, J->mh.N - 1);
    Segment sgn = cache_segment(ns->ps, J->mh.N - 1);
    const size_t real = S->fp64 ? 8 : 4;
    J->norm = ns;
    J->nb_d = seg_blocks(J->ev.n_tiles);
    J->nb_q = std::min(64, std::max(1, (ns->ps.n_cells + 4 * kServeWaves - 1) / (4 * kServeWaves)));
    J->G_d = n_groups(J->nb_d);
    J->G_n = n_groups(J->nb_q);
    J->rs = record_size(J->mh.N - 1, J->mh.R, false);
    const int ni = J->mh.N - 2;
    std::vector<double> cst(consts_words(J->mh.N));
    for (int i = 0; i < ni; ++i) {
      cst[i] = J->mh.th_c[i];
      cst[ni + i] = 1.0 / J->mh.th_d[i];
    }
    std::copy(J->mh.h.begin(), J->mh.h.end(), cst.begin() + 2 * ni);
    // the job's memory is freed after the server's steps; the loading scratch after the load
    hipMemPool_t pl = S->pool;
    if (J->d_tab.alloc_from((size_t)kResWords * std::max(J->mh.R, 1) * 8, pl, st, st) ||
        J->mh.upload_res64(J->theta0.data(), J->d_tab, st) != MIPWA_OK ||
        J->d_rec.alloc_from((size_t)(J->nb_d + J->nb_q) * J->rs * 8, pl, st, S->stream) ||
        J->d_grec.alloc_from((size_t)(J->G_d + J->G_n) * J->rs * 8, pl, st, S->stream) ||
        J->d_consts.alloc_from(cst.size() * 8, pl, st, S->stream)) {
      rc = MIPWA_E_NOMEM;
      err = "device allocation for a job failed";
    } else if (hipMemcpyAsync(J->d_consts.p, cst.data(), cst.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
               launch_cache(S->fp64, J->mh.R, &sg, J->d_tab.as<double>(), J->mh.kin64, st) != hipSuccess) {
      rc = MIPWA_E_HIP;
      err = "loading a job failed";
    } else {
      // the moments at the job's shapes: found, or formed here from the normalisation points'
      // resonance amplitudes (scratch of this load)
      std::vector<double> rkey((size_t)kResWords * std::max(J->mh.R, 1) + 1, 0.0);
      rkey[0] = J->mh.R;
      J->mh.res_table(J->theta0.data(), rkey.data() + 1);
      Moments* mo = nullptr;
      {
        std::lock_guard<std::mutex> g(ns->mom_mu);
        auto& e = ns->moments[rkey];
        if (!e) e = std::make_unique<Moments>();
        mo = e.get();
      }
      std::lock_guard<std::mutex> g(mo->m);
      if (!mo->ready) {
        const size_t mom_bytes =
            (size_t)std::max(ns->ps.n_cells, 1) * qform_dim(J->mh.R) * qform_dim(J->mh.R) * 16;
        DevBuf ncache;
        if (ncache.alloc_from((size_t)std::max(J->mh.R, 1) * 2 * ns->ps.n * real, pl, st, st) ||
            mo->d.alloc_from(mom_bytes, pl, st, S->stream)) {
          rc = MIPWA_E_NOMEM;
          err = "device allocation for the normalisation moments failed";
        } else {
          sgn.cache = ncache.p;
          // the full point segment of the normalisation set for the moment pass
          Segment pts = sgn;
          pts.tt = ns->ps.tt.p;
          pts.w = ns->ps.w.p;
          pts.tiles = ns->ps.tiles.as<Tile>();
          pts.n_tiles = ns->ps.n_tiles;
          pts.kind = 1;
          if (launch_cache(S->fp64, J->mh.R, &sgn, J->d_tab.as<double>(), J->mh.kin64, st) != hipSuccess ||
              launch_moments(S->fp64, J->mh.R, &pts, ns->ps.cells.as<Tile>(), ns->ps.n_cells, mo->d.as<double>(),
                             st) != hipSuccess ||
              hipStreamSynchronize(st) != hipSuccess) {
            rc = MIPWA_E_HIP;
            err = "forming the normalisation moments failed";
          } else {
            mo->ready = true;
            std::lock_guard<std::mutex> lk(S->mu);
            S->used += mom_bytes;
            S->peak = std::max(S->peak, S->used);
          }
        }
        if (!mo->ready) mo->d.release();
      }
      if (!rc && hipStreamSynchronize(st) != hipSuccess) {
        rc = MIPWA_E_HIP;
        err = "loading a job failed";
      }
      J->mom = mo->ready ? mo->d.p : nullptr;
    }
    J->d_tab.release();
  }
  {
    // the stream goes to the longest-waiting job, else back to the free ones
    std::lock_guard<std::mutex> g(S->load_mu);
    if (!S->load_wait.empty()) {
      SJob* next = S->load_wait.front();
      S->load_wait.pop_front();
      next->load_slot = slot;
      next->load_cv.notify_one();
    } else {
      S->load_busy[slot] = false;
    }
  }
  if (rc) {
    finish_job(S, J, rc, err);
    return;
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    J->state = ACTIVE;
    S->n_active += 1;
    trace(S, "job %lld active", (long long)J->id);
    S->cv_sched.notify_all();
  }
  const ModelHost& mh = J->mh;
  FullEval fg = [S, J, &mh](const double* th, double& f, double* g) -> int {
    std::string e;
    if (mh.check_theta(th, e) != MIPWA_OK) {
      f = INFINITY;
      return MIPWA_OK;
    }
    std::vector<char> staged;
    stage(mh, S->fp64, th, staged);
    if (J->cancel || S->stop) return MIPWA_E_CANCELLED;
    {
      std::lock_guard<std::mutex> jl(J->m);
      J->staged.swap(staged);
      J->done = false;
    }
    {
      // the scheduler is woken by the first request of a step and by the one that completes it (every
      // active job outside the steps in flight has asked)
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->stop) return MIPWA_E_CANCELLED;
      J->req = true;
      S->n_req += 1;
      if (S->n_req == 1 || S->n_req >= S->n_active - S->n_inflight) S->cv_sched.notify_one();
    }
    std::unique_lock<std::mutex> jl(J->m);
    J->cv.wait(jl, [&] { return J->done || J->cancel || S->stop; });
    if (!J->done) {
      // cancelled: withdraw the request unless a step has taken it, else wait for that step
      jl.unlock();
      {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!J->inflight) {
          if (J->req) {
            J->req = false;
            S->n_req -= 1;
          }
          return MIPWA_E_CANCELLED;
        }
      }
      jl.lock();
      J->cv.wait(jl, [&] { return J->done; });
    }
    if (J->step_rc) return J->step_rc;  // a device failure ends the fit with its status
    f = std::isfinite(J->f) ? J->f : INFINITY;
    std::copy(J->g.begin(), J->g.end(), g);
    return MIPWA_OK;
  };
  FitOut out;
  std::vector<int> pairs;
  for (int k = 0; k < mh.N + mh.R; ++k) pairs.push_back(2 * k);
  rc = bfgs_fit(fg, mh.P, pairs, J->fixed, J->theta0.data(), J->tol, J->max_iter, J->hessian,
                S->fp64 ? kNoiseRelFp64 : kNoiseRelMixed, out);
  J->result = out;
  finish_job(S, J, rc ? rc : out.status, rc && !J->step_err.empty() ? J->step_err : out.err);
}

namespace {

// A batched step: the jobs it carries (every pending evaluation of one or more resonance counts, one
// launch per count), where their results and sequence words are, and the sequence number their
// finish publishes.
struct Step {
  std::vector<SJob*> batch;
  std::vector<size_t> res_off;  // per job: offset of its results in the step's result buffer
  unsigned long long seq = 0;
  int buf = 0;
  bool timed = false;
};

// Stage and launch one step on the server's stream; returns without waiting for it.  The step's buffer
// set is not in use: the step that last used it has been waited on.
int launch_step(mipwa_server* S, Step& st) {
  mipwa_server::StepBufs& B = S->bufs[st.buf];
  std::vector<SJob*>& batch = st.batch;
  std::map<int, std::vector<int>> by_r;  // resonance count -> positions in batch
  for (int i = 0; i < (int)batch.size(); ++i) by_r[batch[i]->mh.R].push_back(i);
  size_t res_total = 0;
  st.res_off.resize(batch.size());
  for (size_t i = 0; i < batch.size(); ++i) {
    st.res_off[i] = res_total;
    res_total += 1 + batch[i]->mh.P;
  }
  // (larger than the initial buffers only for steps of thousands of jobs)
  if (B.h_res.bytes < res_total * 8) {
    if (B.h_res.alloc(res_total * 8 * 2, true) != hipSuccess ||
        hipHostGetDevicePointer((void**)&B.h_res_dev, B.h_res.p, 0) != hipSuccess)
      return S->fail(MIPWA_E_NOMEM, "result buffer allocation failed");
  }
  if (B.h_seq.bytes < batch.size() * 8) {
    if (B.h_seq.alloc(batch.size() * 8 * 2, true) != hipSuccess ||
        hipHostGetDevicePointer((void**)&B.h_seq_dev, B.h_seq.p, 0) != hipSuccess)
      return S->fail(MIPWA_E_NOMEM, "sequence buffer allocation failed");
    std::memset(B.h_seq.p, 0, B.h_seq.bytes);
  }
  st.seq = g_step_seq.fetch_add(1, std::memory_order_relaxed) + 1;
  // Layout of the step's upload: per resonance count a block map, tasks, segments, jobs and the jobs'
  // tables.  All of it is laid out first, so that the buffers are grown (if at all) before any launch.
  struct Group {
    int R = 0, nj = 0, max_nint = 1;
    std::vector<int> jobs;  // positions in batch
    std::vector<int2> map, tasks;
    size_t o_map = 0, o_task = 0, o_seg = 0, o_job = 0;
    std::vector<size_t> o_tab, o_th;
  };
  std::vector<Group> groups;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) / 256 * 256;
    return o;
  };
  for (auto& kv : by_r) {
    Group g;
    g.R = kv.first;
    g.jobs = kv.second;
    g.nj = (int)g.jobs.size();
    auto J = [&](int j) { return batch[g.jobs[j]]; };
    // block map: data segments job-major, then normalisation segments interleaved by block index
    // among the jobs sharing a normalisation set
    for (int j = 0; j < g.nj; ++j)
      for (int b = 0; b < J(j)->nb_d; ++b) g.map.push_back(int2{2 * j, b});
    std::map<NormSet*, std::vector<int>> by_norm;
    for (int j = 0; j < g.nj; ++j) by_norm[J(j)->norm].push_back(j);
    for (auto& nk : by_norm)
      for (int b = 0; b < J(nk.second[0])->nb_q; ++b)
        for (int j : nk.second) g.map.push_back(int2{2 * j + 1, b});
    for (int j = 0; j < g.nj; ++j) {
      for (int q = 0; q < J(j)->G_d; ++q) g.tasks.push_back(int2{2 * j, q});
      for (int q = 0; q < J(j)->G_n; ++q) g.tasks.push_back(int2{2 * j + 1, q});
    }
    g.o_map = take(g.map.size() * sizeof(int2));
    g.o_task = take(g.tasks.size() * sizeof(int2));
    g.o_seg = take((size_t)2 * g.nj * sizeof(Segment));
    g.o_job = take((size_t)g.nj * sizeof(Job));
    g.o_tab.resize(g.nj);
    g.o_th.resize(g.nj);
    for (int j = 0; j < g.nj; ++j) {
      size_t toff = 0;
      g.o_tab[j] = take(staged_bytes(J(j)->mh, S->fp64, &toff));
      g.o_th[j] = g.o_tab[j] + toff;
      g.max_nint = std::max(g.max_nint, J(j)->mh.N - 1);
    }
    groups.push_back(std::move(g));
  }
  // grown geometrically: batches grow step by step while jobs become active, and each
  // reallocation of pinned or device memory costs milliseconds (a device free synchronises)
  if (off > B.h_batch.bytes || off > B.d_batch.bytes) {
    const size_t cap = std::max(off, 2 * std::max(B.h_batch.bytes, B.d_batch.bytes));
    if (B.h_batch.alloc(cap, true) != hipSuccess || B.d_batch.alloc(cap) != hipSuccess)
      return S->fail(MIPWA_E_NOMEM, "batch buffer allocation failed");
  }
  char* hb = B.h_batch.as<char>();
  char* db = B.d_batch.as<char>();
  for (const Group& g : groups) {
    std::memcpy(hb + g.o_map, g.map.data(), g.map.size() * sizeof(int2));
    std::memcpy(hb + g.o_task, g.tasks.data(), g.tasks.size() * sizeof(int2));
    Segment* sg = reinterpret_cast<Segment*>(hb + g.o_seg);
    Job* jb = reinterpret_cast<Job*>(hb + g.o_job);
    std::memset(sg, 0, (size_t)2 * g.nj * sizeof(Segment));
    std::memset(jb, 0, (size_t)g.nj * sizeof(Job));
    for (int j = 0; j < g.nj; ++j) {
      SJob* J = batch[g.jobs[j]];
      std::memcpy(hb + g.o_tab[j], J->staged.data(), J->staged.size());
      const PointSet* ps[2] = {&J->ev, &J->norm->ps};
      const int nbs[2] = {J->nb_d, J->nb_q};
      for (int k = 0; k < 2; ++k) {
        Segment& s = sg[2 * j + k];
        s.tt = ps[k]->tt.p;
        s.ss = ps[k]->ss.p;
        s.w = k ? ps[k]->w.p : nullptr;
        s.cache = ps[k]->cache.p;
        s.tiles = ps[k]->tiles.as<Tile>();
        s.table = db + g.o_tab[j];
        s.records = J->d_rec.as<double>() + (size_t)(k ? J->nb_d : 0) * J->rs;
        s.n = ps[k]->n;
        s.n_tiles = ps[k]->n_tiles;
        s.kind = k;
        if (k) {
          // the normalisation as a quadratic form over the shared set's cells and the job's moments
          s.kind = 2;
          s.tiles = ps[k]->cells.as<Tile>();
          s.n_tiles = ps[k]->n_cells;
          s.cache = J->mom;
        }
        s.nint = J->mh.N - 1;
        s.rs = J->rs;
        s.n_blocks = nbs[k];
        s.job = j;
        s.g0 = k ? J->G_d : 0;
      }
      Job& q = jb[j];
      q.tab64 = reinterpret_cast<const double*>(db + g.o_th[j]);
      q.consts = J->d_consts.as<double>();
      q.out = B.h_res_dev + st.res_off[g.jobs[j]];
      q.seq_out = B.h_seq_dev + g.jobs[j];
      q.grec = J->d_grec.as<double>();
      q.n_ev = (double)J->ev.n;
      q.c_eps = 0.0;
      q.G_d = J->G_d;
      q.G_n = J->G_n;
      q.N = J->mh.N;
      q.R = J->mh.R;
      q.rs = J->rs;
      q.otf = 0;
    }
  }
  // a sampled step: fold the previous sample (complete unless its step is the one in flight) and
  // bracket this step's kernels
  st.timed = S->ev_step[0] && st.seq % kStepTimingPeriod == 0;
  std::unique_lock<std::mutex> tl(S->timing_mu, std::defer_lock);
  if (st.timed) {
    tl.lock();
    if (S->step_timed_unread) {
      float ms = 0;
      if (hipEventQuery(S->ev_step[1]) == hipSuccess &&
          hipEventElapsedTime(&ms, S->ev_step[0], S->ev_step[1]) == hipSuccess) {
        S->step_dev_ms += ms;
        S->n_step_timed += 1;
      }
      (void)hipGetLastError();
    }
    S->step_timed_unread = false;
    if (hipEventRecord(S->ev_step[0], S->stream) != hipSuccess) return S->fail(MIPWA_E_HIP, "step timing event");
  }
  if (launch_upload(db, B.h_batch.dev, off, S->stream) != hipSuccess)
    return S->fail(MIPWA_E_HIP, "batch upload failed");
  for (const Group& g : groups) {
    const ModelHost& mh0 = batch[g.jobs[0]]->mh;
    if (launch_eval(S->fp64, g.R, false, reinterpret_cast<const Segment*>(db + g.o_seg),
                    reinterpret_cast<const int2*>(db + g.o_map), reinterpret_cast<const Job*>(db + g.o_job),
                    (int)g.map.size(), kServeWaves, g.max_nint,
                    S->fp64 ? (const void*)&mh0.kin64 : (const void*)&mh0.kin32, nullptr, 1, S->sweep_order,
                    S->stream) != hipSuccess)
      return S->fail(MIPWA_E_HIP, "batched likelihood kernel failed");
    if (launch_reduce(reinterpret_cast<const Segment*>(db + g.o_seg), reinterpret_cast<const Job*>(db + g.o_job),
                      reinterpret_cast<const int2*>(db + g.o_task), (int)g.tasks.size(), g.nj, nullptr, S->stream,
                      st.seq) != hipSuccess)
      return S->fail(MIPWA_E_HIP, "batched reduction kernels failed");
  }
  S->sweep_order ^= 1;
  if (st.timed) {
    if (hipEventRecord(S->ev_step[1], S->stream) != hipSuccess) return S->fail(MIPWA_E_HIP, "step timing event");
    S->step_timed_unread = true;
  }
  return MIPWA_OK;
}

// Wait for a launched step's results: spin on the jobs' sequence words, which flip as soon as the
// finish has written each job's results, without waiting for the stream's completion signal.  The
// stream is queried now and then so that a failed launch is still reported.
int wait_step(mipwa_server* S, Step& st) {
  mipwa_server::StepBufs& B = S->bufs[st.buf];
  const unsigned long long* words = B.h_seq.as<unsigned long long>();
  for (size_t i = 0; i < st.batch.size(); ++i) {
    const unsigned long long* w = words + i;
    for (unsigned long long it = 1; __atomic_load_n(w, __ATOMIC_ACQUIRE) != st.seq; ++it) {
      if ((it & 1023) == 0) {
        const hipError_t q = hipStreamQuery(S->stream);
        if (q == hipSuccess && __atomic_load_n(w, __ATOMIC_ACQUIRE) != st.seq)
          return S->fail(MIPWA_E_HIP, "a step ended without publishing its results");
        if (q != hipSuccess && q != hipErrorNotReady)
          return S->fail(MIPWA_E_HIP, std::string("batch failed: ") + hipGetErrorString(q));
      }
      _mm_pause();
    }
  }
  const double* res = B.h_res.as<double>();
  for (size_t i = 0; i < st.batch.size(); ++i) {
    SJob* J = st.batch[i];
    const double* o = res + st.res_off[i];
    J->f = o[0];
    J->g.assign(o + 1, o + 1 + J->mh.P);
  }
  return MIPWA_OK;
}

// Whether every job of a launched step has its results (non-blocking).
bool step_ready(mipwa_server* S, const Step& st) {
  const unsigned long long* words = S->bufs[st.buf].h_seq.as<unsigned long long>();
  for (size_t i = 0; i < st.batch.size(); ++i)
    if (__atomic_load_n(words + i, __ATOMIC_ACQUIRE) != st.seq) return false;
  return true;
}

// Hand a waited-for step's results (or its failure) back to its jobs' threads.
void hand_back(mipwa_server* S, Step& st, int rc) {
  const std::string step_err = rc ? S->last_error() : std::string();
  for (SJob* J : st.batch) {
    {
      std::lock_guard<std::mutex> jl(J->m);
      if (rc) {
        J->f = NAN;
        J->step_rc = rc;
        J->step_err = step_err;
      }
      J->done = true;
    }
    J->cv.notify_one();
  }
}


void sched_loop(mipwa_server* S) {
  (void)hipSetDevice(S->device);
  // Up to two steps in flight on the stream.  While one runs, the jobs of the other (whose results
  // have been handed back) compute their next points and the next step is formed and queued behind
  // the running one, so the host's share of a step overlaps the device's.  A step formed while none is
  // in flight takes at most half of the active jobs: the rest form the next step at once, which splits
  // the jobs into two groups that then alternate.
  std::deque<Step> flight;
  std::unique_lock<std::mutex> lk(S->mu);
  auto finish_oldest = [&]() {
    Step st = std::move(flight.front());
    flight.pop_front();
    lk.unlock();
    const auto t_g = Clock::now();
    const int rc = wait_step(S, st);
    S->t_gpu += std::chrono::duration<double>(Clock::now() - t_g).count();
    lk.lock();
    for (SJob* J : st.batch) J->inflight = false;
    S->n_inflight -= (int)st.batch.size();
    S->steps += 1;
    S->batch_sum += (double)st.batch.size();
    lk.unlock();
    const auto t_e = Clock::now();
    hand_back(S, st, rc);
    lk.lock();
    S->t_wake += std::chrono::duration<double>(Clock::now() - t_e).count();
    if (S->steps % 256 == 1) trace(S, "step %lld: batch %zu of %d active", S->steps, st.batch.size(), S->n_active);
  };
  while (!S->stop) {
    const auto t_0 = Clock::now();
    admit(S);
    for (auto& kv : S->jobs)
      if (kv.second->retired && kv.second->worker.joinable()) kv.second->worker.join();
    S->t_admit += std::chrono::duration<double>(Clock::now() - t_0).count();
    auto admissible = [&] {
      if (S->queue.empty()) return false;
      SJob* J = S->queue.front();
      return J->cancel || S->running == 0 || S->used + J->bytes <= S->budget;
    };
    if (flight.empty()) {
      const auto t_a = Clock::now();
      S->cv_sched.wait(lk, [&] { return S->stop || S->n_req > 0 || admissible(); });
      S->t_idle += std::chrono::duration<double>(Clock::now() - t_a).count();
      if (S->stop) break;
      if (S->n_req == 0) continue;
    } else if (flight.size() == 2) {
      finish_oldest();
      continue;
    } else {
      // one step in flight: form the next as soon as a job outside it asks, else hand back its results
      const auto t_a = Clock::now();
      while (!S->stop && S->n_req == 0 && !step_ready(S, flight.front()))
        S->cv_sched.wait_for(lk, std::chrono::microseconds(20));
      S->t_idle += std::chrono::duration<double>(Clock::now() - t_a).count();
      if (S->stop) break;
      if (S->n_req == 0) {
        finish_oldest();
        continue;
      }
    }
    // batching window: until every active job outside the steps in flight has asked, or
    // kBatchWindowUs after this point
    const auto t_b = Clock::now();
    const auto deadline = t_b + std::chrono::microseconds(kBatchWindowUs);
    while (!S->stop && S->n_req < S->n_active - S->n_inflight)
      if (S->cv_sched.wait_until(lk, deadline) == std::cv_status::timeout) break;
    if (S->stop) break;
    S->t_window += std::chrono::duration<double>(Clock::now() - t_b).count();
    const size_t cap = flight.empty() && S->n_active >= 2 ? (size_t)(S->n_active + 1) / 2 : (size_t)S->n_active;
    Step st;
    st.buf = S->next_buf;
    for (auto& kv : S->jobs) {
      SJob* J = kv.second.get();
      if (st.batch.size() >= cap) break;
      if (J->state != ACTIVE || !J->req || J->inflight) continue;
      J->req = false;
      S->n_req -= 1;
      if (J->cancel) continue;  // its worker withdraws
      J->inflight = true;
      st.batch.push_back(J);
    }
    if (st.batch.empty()) continue;
    S->n_inflight += (int)st.batch.size();
    lk.unlock();
    const auto t_d = Clock::now();
    const bool overlapped = !flight.empty();
    const int rc = launch_step(S, st);
    S->t_stage += std::chrono::duration<double>(Clock::now() - t_d).count();
    lk.lock();
    if (rc) {
      // nothing of this step runs: its jobs end with the failure
      for (SJob* J : st.batch) J->inflight = false;
      S->n_inflight -= (int)st.batch.size();
      lk.unlock();
      hand_back(S, st, rc);
      lk.lock();
      continue;
    }
    S->next_buf ^= 1;
    if (overlapped) S->n_overlapped += 1;
    flight.push_back(std::move(st));
  }
  // stopping: the steps in flight still end, and their jobs get their results
  while (!flight.empty()) finish_oldest();
}

}  // namespace

// Streams, events and the memory pool of a server (any of them may be missing): every stream is
// drained first, so no freed block is still in use when the pool is destroyed.
static void release_device_objects(mipwa_server* S) {
  for (hipStream_t st : S->load_st)
    if (st) (void)hipStreamSynchronize(st);
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (hipEvent_t e : S->ev_step)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t st : S->load_st)
    if (st) (void)hipStreamDestroy(st);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  if (S->pool) (void)hipMemPoolDestroy(S->pool);
}

extern "C" {

int mipwa_server_create(int device, int precision, size_t budget, mipwa_server** out) {
  if (!out || (precision != MIPWA_FP64 && precision != MIPWA_MIXED)) return MIPWA_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MIPWA_E_INVAL;
  auto S = new (std::nothrow) mipwa_server();
  if (!S) return MIPWA_E_NOMEM;
  S->device = device;
  S->fp64 = precision == MIPWA_FP64;
  (void)hipSetDevice(device);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = (size_t)64 << 30;
  S->budget = budget ? budget : (size_t)(0.8 * (double)free_b);
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof(props));
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = device;
  uint64_t keep = UINT64_MAX;  // freed memory stays in the pool until the server is destroyed
  bool ok = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreate(&S->ev_step[0]) == hipSuccess && hipEventCreate(&S->ev_step[1]) == hipSuccess &&
            hipMemPoolCreate(&S->pool, &props) == hipSuccess &&
            hipMemPoolSetAttribute(S->pool, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess;
  for (int i = 0; ok && i < kLoadStreams; ++i)
    ok = hipStreamCreateWithFlags(&S->load_st[i], hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    release_device_objects(S);
    delete S;
    return MIPWA_E_HIP;
  }
  // step buffers sized up front for a few hundred jobs per step: allocating pinned or device memory
  // during the steps costs milliseconds each time (they still grow if a step needs more)
  for (auto& B : S->bufs) {
    if (B.h_batch.alloc(kBatchBytes0, true) != hipSuccess || B.d_batch.alloc(kBatchBytes0) != hipSuccess ||
        B.h_res.alloc(kResultBytes0, true) != hipSuccess ||
        hipHostGetDevicePointer((void**)&B.h_res_dev, B.h_res.p, 0) != hipSuccess ||
        B.h_seq.alloc(kSeqBytes0, true) != hipSuccess ||
        hipHostGetDevicePointer((void**)&B.h_seq_dev, B.h_seq.p, 0) != hipSuccess) {
      release_device_objects(S);
      delete S;
      return MIPWA_E_NOMEM;
    }
    std::memset(B.h_seq.p, 0, B.h_seq.bytes);
  }
  S->sched = std::thread(sched_loop, S);
  *out = S;
  return MIPWA_OK;
}

int mipwa_server_set_norm(mipwa_server* S, const double* s12, const double* s13, const double* w, int64_t n) {
  if (!S) return MIPWA_E_INVAL;
  if (!s12 || !s13 || !w || n < 1) return S->fail(MIPWA_E_INVAL, "need n >= 1 normalisation points with weights");
  std::lock_guard<std::mutex> g(S->norm_mu);
  if (!S->norms.empty()) return S->fail(MIPWA_E_STATE, "the normalisation sample is already in use");
  S->n12.assign(s12, s12 + n);
  S->n13.assign(s13, s13 + n);
  S->nw.assign(w, w + n);
  return MIPWA_OK;
}

static int submit_job(mipwa_server* S, const mipwa_model* model, const double* s12, const double* s13, int64_t n,
                      const double* theta0, const unsigned char* fixed, const mipwa_fit_opts* opts, int64_t* job_id,
                      bool borrow) {
  if (!S) return MIPWA_E_INVAL;
  size_t n_norm = 0;
  {
    std::lock_guard<std::mutex> g(S->norm_mu);
    n_norm = S->n12.size();
  }
  if (n_norm == 0) return S->fail(MIPWA_E_STATE, "set the normalisation sample first");
  if (!s12 || !s13 || n < 1 || !theta0 || !job_id) return S->fail(MIPWA_E_INVAL, "need events, theta0 and job_id");
  auto J = std::make_unique<SJob>();
  std::string err;
  int rc = J->mh.init(model, err);
  if (rc) return S->fail(rc, err);
  const int P = J->mh.P, N = J->mh.N, R = J->mh.R;
  rc = J->mh.check_theta(theta0, err);
  if (rc) return S->fail(rc, err);
  J->fixed.assign(P, 0);
  if (fixed) {
    J->fixed.assign(fixed, fixed + P);
  } else {
    if (R > 0) J->fixed[2 * N] = J->fixed[2 * N + 1] = 1;
    for (int p = 2 * N + 2 * R; p < P; ++p) J->fixed[p] = 1;
  }
  for (int p = 2 * N + 2 * R; p < P; ++p)
    if (!J->fixed[p]) return S->fail(MIPWA_E_INVAL, "serving jobs keep masses and widths fixed");
  if (borrow) {
    J->ev12 = s12;
    J->ev13 = s13;
  } else {
    J->ev_host.reset(alloc_events(n));
    if (!J->ev_host) return S->fail(MIPWA_E_NOMEM, "no host memory for the job's events");
    copy_events(J->ev_host.get(), J->ev_host.get() + n, s12, s13, n);
    J->ev12 = J->ev_host.get();
    J->ev13 = J->ev_host.get() + n;
  }
  J->n = n;
  J->theta0.assign(theta0, theta0 + P);
  J->tol = opts && opts->tol_edm > 0 ? opts->tol_edm : 1e-4;
  J->max_iter = opts && opts->max_iter > 0 ? opts->max_iter : 1000;
  J->hessian = opts ? opts->hessian != 0 : false;
  const size_t real = S->fp64 ? 8 : 4;
  J->bytes = (size_t)n * ((2 + 2 * R) * real + 16) + (size_t)(n / kTile + 1) * 2 * sizeof(Tile) +
             n_norm * 2 * (size_t)std::max(R, 1) * real +
             (size_t)(2 * kMaxSegBlocks + 32) * record_size(N - 1, R, false) * 8;
  if (J->bytes > S->budget) return S->fail(MIPWA_E_NOMEM, "the job alone exceeds the HBM budget");
  std::lock_guard<std::mutex> lk(S->mu);
  J->id = S->next_id++;
  J->t_submit = Clock::now();
  if (!S->any_submit) {
    S->any_submit = true;
    S->t_first_submit = J->t_submit;
  }
  *job_id = J->id;
  S->queue.push_back(J.get());
  S->jobs[J->id] = std::move(J);
  S->cv_sched.notify_all();
  return MIPWA_OK;
}

int mipwa_server_submit(mipwa_server* S, const mipwa_model* model, const double* s12, const double* s13, int64_t n,
                        const double* theta0, const unsigned char* fixed, const mipwa_fit_opts* opts,
                        int64_t* job_id) {
  return submit_job(S, model, s12, s13, n, theta0, fixed, opts, job_id, false);
}

int mipwa_server_submit_borrowed(mipwa_server* S, const mipwa_model* model, const double* s12, const double* s13,
                                 int64_t n, const double* theta0, const unsigned char* fixed,
                                 const mipwa_fit_opts* opts, int64_t* job_id) {
  return submit_job(S, model, s12, s13, n, theta0, fixed, opts, job_id, true);
}

namespace {
int copy_result(mipwa_server* S, SJob* J, double* theta_out, mipwa_fit_info* info, double* latency) {
  if (J->state != FINISHED) return MIPWA_E_BUSY;
  if (J->status == MIPWA_E_CANCELLED) return MIPWA_E_CANCELLED;
  if (J->status != MIPWA_OK && J->status != MIPWA_E_NOCONV) return S->fail(J->status, J->err);
  if (theta_out) std::copy(J->result.theta.begin(), J->result.theta.end(), theta_out);
  if (info) {
    info->nll = J->result.nll;
    info->edm = J->result.edm;
    info->n_iter = J->result.n_iter;
    info->n_eval = J->result.n_eval;
    info->status = J->status;
  }
  if (latency) *latency = std::chrono::duration<double>(J->t_done - J->t_submit).count();
  return J->status;
}
}  // namespace

int mipwa_server_poll(mipwa_server* S, int64_t id, double* theta_out, mipwa_fit_info* info, double* latency_s) {
  if (!S) return MIPWA_E_INVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return S->fail(MIPWA_E_INVAL, "unknown job");
  return copy_result(S, it->second.get(), theta_out, info, latency_s);
}

int mipwa_server_wait(mipwa_server* S, int64_t id, double timeout_s, double* theta_out, mipwa_fit_info* info,
                      double* latency_s) {
  if (!S) return MIPWA_E_INVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return S->fail(MIPWA_E_INVAL, "unknown job");
  SJob* J = it->second.get();
  auto ready = [&] { return J->state == FINISHED; };
  if (timeout_s > 0)
    S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
  else
    S->cv_done.wait(lk, ready);
  return copy_result(S, J, theta_out, info, latency_s);
}

int mipwa_server_cancel(mipwa_server* S, int64_t id) {
  if (!S) return MIPWA_E_INVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return S->fail(MIPWA_E_INVAL, "unknown job");
  SJob* J = it->second.get();
  J->cancel = true;
  wake(J);
  S->cv_sched.notify_all();
  return MIPWA_OK;
}

int mipwa_server_stats(mipwa_server* S, mipwa_serve_stats* st) {
  if (!S || !st) return MIPWA_E_INVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(st, 0, sizeof(*st));
  std::vector<double> lat = S->latencies;
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double q) {
    if (lat.empty()) return 0.0;
    const double pos = q * (lat.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < lat.size() ? lat[i] * (1 - f) + lat[i + 1] * f : lat[i];
  };
  st->n_done = (int64_t)lat.size();
  st->p50_s = pct(0.50);
  st->p99_s = pct(0.99);
  const double span = std::chrono::duration<double>(S->t_last_done - S->t_first_submit).count();
  st->fits_per_s = span > 0 ? lat.size() / span : 0.0;
  for (auto& kv : S->jobs) {
    if (kv.second->state == QUEUED) st->n_queued += 1;
    if (kv.second->state == LOADING || kv.second->state == ACTIVE) st->n_active += 1;
  }
  st->peak_bytes = (int64_t)S->peak;
  st->steps = S->steps;
  st->mean_batch = S->steps ? S->batch_sum / S->steps : 0.0;
  std::lock_guard<std::mutex> tl(S->timing_mu);
  if (S->step_timed_unread) {  // the last sample: its step has long finished unless a step is running
    float ms = 0;
    if (hipEventQuery(S->ev_step[1]) == hipSuccess && hipEventElapsedTime(&ms, S->ev_step[0], S->ev_step[1]) == hipSuccess) {
      S->step_dev_ms += ms;
      S->n_step_timed += 1;
      S->step_timed_unread = false;
    }
    (void)hipGetLastError();
  }
  st->step_device_s = S->n_step_timed ? 1e-3 * S->step_dev_ms / S->n_step_timed : 0.0;
  st->device_busy = span > 0 ? st->step_device_s * S->steps / span : 0.0;
  return MIPWA_OK;
}

const char* mipwa_server_last_error(const mipwa_server* S) {
  if (!S) return "server is NULL";
  thread_local std::string copy;  // the message stays valid while other threads fail
  copy = S->last_error();
  return copy.c_str();
}

void mipwa_server_destroy(mipwa_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (auto& kv : S->jobs) {
      kv.second->cancel = true;
      wake(kv.second.get());
    }
    S->cv_sched.notify_all();
  }
  {
    std::lock_guard<std::mutex> g(S->load_mu);  // jobs waiting for a loader stream give up
    for (SJob* J : S->load_wait) J->load_cv.notify_one();
  }
  if (S->sched.joinable()) S->sched.join();
  for (auto& kv : S->jobs)
    if (kv.second->worker.joinable()) kv.second->worker.join();
  trace(S, "scheduler: %lld steps (%lld launched behind another); idle %.3f s, batching window %.3f s, staging "
        "and launch %.3f s, waiting for results %.3f s, results to the jobs %.3f s, admission and joins %.3f s",
        S->steps, S->n_overlapped, S->t_idle, S->t_window, S->t_stage, S->t_gpu, S->t_wake, S->t_admit);
  (void)hipSetDevice(S->device);
  // the jobs' and sets' memory goes back to the pool after the last step; then the pool goes
  S->jobs.clear();
  S->norms.clear();
  release_device_objects(S);
  delete S;
}

}  // extern "C"
