// mipwa_eval_noalloc: the evaluation of mipwa_eval_async for callers that cannot allocate device
// memory.  Its scratch (launch descriptors, resonance constants, per-block and group records) lives in
// one file-scope device array per GPU instead of context buffers sized on first use.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.h"
#include "mipwa.h"

using namespace mipwa;

#ifndef MIPWA_NOALLOC_SCRATCH_BYTES
#define MIPWA_NOALLOC_SCRATCH_BYTES (8u << 20)
#endif

namespace {

constexpr size_t kScratchBytes = (size_t)MIPWA_NOALLOC_SCRATCH_BYTES;
constexpr size_t kAlign = 256;

}  // namespace

// One copy per GPU, held until the process ends.  In host code this name is a stand-in for the
// device symbol, never a device address: host code uses the pointer from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<unsigned char*> g_scratch_ptr;  // per device, filled on the first call on that device

// Device address of this device's `scratch` (the caller has made `device` current).
hipError_t scratch_base(int device, unsigned char** out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Everything the descriptors of one evaluation hold, passed by value to the kernel that writes them
// into the scratch.
struct SetupArgs {
  Segment seg[2];
  Job job;
  double res64[kResWords * kMaxRes];
  int nb_d, B, n_res64, pad;
};

__global__ __launch_bounds__(256) void k_noalloc_setup(SetupArgs a, Segment* __restrict__ seg, Job* __restrict__ job,
                                                       double* __restrict__ res64, int2* __restrict__ block_map) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.B) block_map[i] = i < a.nb_d ? int2{0, i} : int2{1, i - a.nb_d};
  if (i < a.n_res64) res64[i] = a.res64[i];
  if (i == 0) {
    seg[0] = a.seg[0];
    seg[1] = a.seg[1];
    *job = a.job;
  }
}

}  // namespace

#define NACHK(expr, what)                                                            \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return ctx->fail(MIPWA_E_HIP, std::string(what) + ": " +  \
                                                              hipGetErrorString(e_)); \
  } while (0)

extern "C" int mipwa_eval_noalloc(mipwa_ctx* ctx, void* stream, double* d_out) {
  if (!ctx) return MIPWA_E_INVAL;
  if (!d_out) return ctx->fail(MIPWA_E_INVAL, "d_out is NULL");
  if (!ctx->ev.loaded || !ctx->nm.loaded) return ctx->fail(MIPWA_E_STATE, "load events and normalisation points first");
  if (!ctx->have_theta) return ctx->fail(MIPWA_E_STATE, "set parameters first");
  if (ctx->use_qform())
    return ctx->fail(MIPWA_E_STATE, "the quadratic-form normalisation keeps per-cell moments in context memory; "
                                    "use MIPWA_NORM_POINTS with mipwa_eval_noalloc");
  (void)hipSetDevice(ctx->device);
  unsigned char* base = nullptr;
  NACHK(scratch_base(ctx->device, &base), "scratch address");
  const mipwa_ctx::LaunchPlan L = ctx->plan_launch();
  const int T = L.G_d + L.G_n;
  // scratch layout: segments | job | resonance constants | block map | records | group records
  size_t off = 0;
  const size_t o_seg = off;
  off += up(2 * sizeof(Segment));
  const size_t o_job = off;
  off += up(sizeof(Job));
  const size_t o_res = off;
  off += up(sizeof(double) * kResWords * kMaxRes);
  const size_t o_bmap = off;
  off += up(sizeof(int2) * L.B);
  const size_t o_rec = off;
  off += up(sizeof(double) * (size_t)L.B * L.rs);
  const size_t o_grec = off;
  off += up(sizeof(double) * (size_t)T * L.rs);
  if (off > kScratchBytes)
    return ctx->fail(MIPWA_E_INVAL, "this evaluation needs " + std::to_string(off) + " bytes of scratch (" +
                                        std::to_string(L.B) + " blocks of " + std::to_string(L.rs) +
                                        "-double records); mipwa_eval_noalloc has " + std::to_string(kScratchBytes) +
                                        ": use fewer blocks (mipwa_set_launch) or mipwa_eval_async");
  Segment* d_seg = reinterpret_cast<Segment*>(base + o_seg);
  Job* d_job = reinterpret_cast<Job*>(base + o_job);
  double* d_res = reinterpret_cast<double*>(base + o_res);
  int2* d_bmap = reinterpret_cast<int2*>(base + o_bmap);
  double* d_rec = reinterpret_cast<double*>(base + o_rec);
  double* d_grec = reinterpret_cast<double*>(base + o_grec);

  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = ctx->order_after_last(st);
  if (rc) return rc;
  rc = ctx->stage_params();
  if (rc) return rc;
  SetupArgs a;
  std::memset(&a, 0, sizeof(a));
  ctx->make_segments(L, d_rec, a.seg);
  ctx->make_job(L, d_grec, a.job);
  a.job.out = d_out;
  a.job.seq_out = nullptr;
  a.nb_d = L.nb_d;
  a.B = L.B;
  const bool rebuild = !ctx->otf && ctx->shapes_changed();
  if (rebuild) {
    ctx->mh.res_table(ctx->theta.data(), a.res64);
    a.n_res64 = kResWords * ctx->mh.R;
  }
  const int n_setup = std::max(L.B, std::max(a.n_res64, 1));
  (void)hipGetLastError();
  k_noalloc_setup<<<(n_setup + 255) / 256, 256, 0, st>>>(a, d_seg, d_job, d_res, d_bmap);
  NACHK(hipGetLastError(), "descriptor kernel");
  if (rebuild) {
    // the resonance amplitudes of both point sets at the new masses and widths; the context's own
    // evaluations see the same cache state
    for (int k = 0; k < 2; ++k)
      NACHK(launch_cache(ctx->fp64, ctx->mh.R, &a.seg[k], d_res, ctx->mh.kin64, st), "resonance cache kernel");
    ctx->cache_shape.assign(ctx->theta.begin() + 2 * ctx->mh.N + 2 * ctx->mh.R, ctx->theta.end());
    ctx->cache_valid = true;
    ctx->mom_valid = false;
  }
  if (!ctx->use_arg) {
    NACHK(launch_upload(ctx->d_blob.p, ctx->h_blob.dev, ctx->upload16(), st), "parameter upload");
    NACHK(hipEventRecord(ctx->ev_staged, st), "event");
  }
  const ArgTable* args = ctx->use_arg ? &ctx->h_args : nullptr;
  NACHK(launch_eval(ctx->fp64, ctx->mh.R, ctx->otf, d_seg, d_bmap, d_job, L.B, L.waves, ctx->mh.N - 1,
                    ctx->fp64 ? (const void*)&ctx->mh.kin64 : (const void*)&ctx->mh.kin32, args, L.parts, ctx->sweep_order,
                    st),
        "likelihood kernel");
  // the group sums take the layout by value: no task list in the scratch
  GroupPlan plan{};
  for (int k = 0; k < 2; ++k) {
    plan.records[k] = a.seg[k].records;
    plan.n_blocks[k] = a.seg[k].n_blocks;
  }
  plan.grec = d_grec;
  plan.G_d = L.G_d;
  plan.G_n = L.G_n;
  plan.rs = L.rs;
  NACHK(launch_reduce(d_seg, d_job, nullptr, 0, 1, args, st, 0, d_out, &a.job, &plan), "reduction kernels");
  NACHK(hipEventRecord(ctx->ev_done, st), "event");
  ctx->last_st = st;
  ctx->sweep_order ^= 1;
  return MIPWA_OK;
}
