// Issue-rate probe behind the tile kernel's roofline: the v_sad_u8 lane
// operations per second the GPU sustains when every wavefront slot issues
// them back to back. Declared in include/sbs.h.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "../../include/sbs.h"
#include "sbs_internal.h"

namespace {

constexpr int kChains = 16;   // accumulators per lane (each feeds its own next step)
constexpr int kUnroll = 8;    // steps per loop trip

// Every step is one v_sad_u8 per chain whose operands are the chain's own
// value, so nothing can be folded or hoisted; a wavefront issues dependent
// VALU instructions back to back, and the chains leave the scheduler free to
// interleave them. The sums are written out so that none of it is dead.
__global__ __launch_bounds__(64) void k_probe_sad(int32_t trips, uint32_t seed, uint32_t* out) {
  uint32_t acc[kChains];
  const uint32_t x = seed ^ (0x9E3779B9u * (blockIdx.x * 64u + threadIdx.x));
#pragma unroll
  for (int k = 0; k < kChains; ++k) acc[k] = x + 0x01010101u * (uint32_t)k;
  for (int t = 0; t < trips; ++t) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int k = 0; k < kChains; ++k) acc[k] = __builtin_amdgcn_sad_u8(acc[k], x, acc[k]);
  }
  uint32_t s = 0u;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s ^= acc[k];
  out[blockIdx.x * 64u + threadIdx.x] = s;
}

}  // namespace

extern "C" int sbs_probe_sad_rate(int32_t blocks, int32_t trips, double* lane_ops_per_s, double* ms) {
  if (blocks < 1 || trips < 1 || !lane_ops_per_s || !ms) return sbs::report_error(SBS_ERR_INVALID_ARG, "probe: bad arguments");
  uint32_t* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&out, (size_t)blocks * 64 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_probe_sad, dim3(blocks), dim3(64), 0, 0, trips, 12345u, out);   // warm-up
    e = hipEventRecord(e0, 0);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_probe_sad, dim3(blocks), dim3(64), 0, 0, trips, 54321u, out);
    e = hipEventRecord(e1, 0);
  }
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  if (e != hipSuccess) return sbs::report_error(SBS_ERR_HIP, hipGetErrorString(e));
  *ms = t;
  *lane_ops_per_s = (double)blocks * 64.0 * trips * kUnroll * kChains / (t * 1e-3);
  return SBS_OK;
}
