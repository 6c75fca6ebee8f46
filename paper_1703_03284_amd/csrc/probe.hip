// mipwa_read_bandwidth: the rate at which this GPU streams a large buffer from HBM into registers
// with plain 16-byte loads and no arithmetic to speak of.  It is the measured ceiling that the
// likelihood sweep's bandwidth is compared with beside the datasheet peak.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mipwa.h"

namespace {

__global__ __launch_bounds__(256) void k_fill(float4* __restrict__ a, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a[i] = make_float4(1.0f, 2.0f, 3.0f, (float)(i & 7));
}

using F4v = float __attribute__((ext_vector_type(4)));

// Each thread sums a grid-strided run of 16-byte loads with non-temporal hints (as the sweep reads its
// point streams) and writes one float, so the loads cannot be dropped.
__global__ __launch_bounds__(256) void k_read(const float4* __restrict__ a4, long long n, float* __restrict__ out) {
  const F4v* a = reinterpret_cast<const F4v*>(a4);
  float s = 0.0f;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const F4v v0 = __builtin_nontemporal_load(a + i);
    const F4v v1 = __builtin_nontemporal_load(a + i + stride);
    const F4v v2 = __builtin_nontemporal_load(a + i + 2 * stride);
    const F4v v3 = __builtin_nontemporal_load(a + i + 3 * stride);
    s += (v0.x + v1.y) + (v2.z + v3.w);
  }
  for (; i < n; i += stride) {
    const F4v v = __builtin_nontemporal_load(a + i);
    s += v.x;
  }
  out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int mipwa_read_bandwidth(int device, int64_t bytes, int reps, double* gbs) {
  if (bytes < (1 << 20) || reps < 1 || !gbs) return MIPWA_E_INVAL;
  if (hipSetDevice(device) != hipSuccess) return MIPWA_E_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return MIPWA_E_HIP;
  const long long n = bytes / 16;
  const int cus = std::max(prop.multiProcessorCount, 1);
  const int blocks = 32 * cus;  // the most grid the probe tries (blocks of 256 threads)
  void *a = nullptr, *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t st = nullptr;
  int rc = MIPWA_OK;
  if (hipMalloc(&a, (size_t)n * 16) != hipSuccess || hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) {
    rc = MIPWA_E_NOMEM;
  } else if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
             hipEventCreate(&e1) != hipSuccess) {
    rc = MIPWA_E_HIP;
  } else {
    k_fill<<<blocks, 256, 0, st>>>(static_cast<float4*>(a), n);
    k_read<<<blocks, 256, 0, st>>>(static_cast<const float4*>(a), n, static_cast<float*>(out));  // warm-up
    // the best over grids of 4, 8, 16 and 32 blocks per CU
    float best = 0.0f;
    for (int g = 4; g <= 32 && rc == MIPWA_OK; g *= 2) {
      for (int r = 0; r < reps && rc == MIPWA_OK; ++r) {
        float ms = 0.0f;
        if (hipEventRecord(e0, st) != hipSuccess) rc = MIPWA_E_HIP;
        k_read<<<g * cus, 256, 0, st>>>(static_cast<const float4*>(a), n, static_cast<float*>(out));
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          rc = MIPWA_E_HIP;
        else if (best == 0.0f || ms < best)
          best = ms;
      }
    }
    if (rc == MIPWA_OK) *gbs = (double)n * 16.0 / (best * 1e-3) / 1e9;
  }
  if (st) (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  if (a) (void)hipFree(a);
  if (out) (void)hipFree(out);
  return rc;
}
