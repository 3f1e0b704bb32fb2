// Single-frame disparity search in a fixed device scratch array: the entry
// point for callers that cannot allocate (code under stream capture, serving
// loops that forbid allocation). Same kernels, layout and results as
// sbs_sad_disparity with a caller workspace; declared in include/sbs.h.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <map>
#include <mutex>

#include "../../include/sbs.h"
#include "sbs_internal.h"

namespace sbs {
int validate_frame(const sbs_frame& f);
size_t workspace_bound(const sbs_frame& f);
int run_single_into(const sbs_frame& f, void* workspace, size_t ws_bytes, hipStream_t s);
int fail_message(int status, const char* msg);
}  // namespace sbs

using namespace sbs;

// The scratch itself: one copy per GPU, held from the library's first use on
// that GPU until the process ends. Host code never passes this name to a
// kernel or a copy (on the host it is only a stand-in for the symbol); it
// uses the device address looked up per device below.
static __device__ __align__(256) uint8_t scratch[SBS_SCRATCH_BYTES];

namespace {

// The persistent part of the workspace header is the error word; the queue
// heads and every per-frame region are reset by the launch sequence itself.
__global__ void k_clear_header(uint32_t* words, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) words[i] = 0u;
}

std::mutex g_mu;
std::map<int, void*> g_ptr;   // device -> device address of `scratch`

// Device address of this device's scratch, looked up (and its header
// cleared, stream-ordered) the first time the current device calls in.
int scratch_ptr(hipStream_t s, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_message(SBS_ERR_HIP, hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ptr.find(dev);
  if (it == g_ptr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char msg[256];
      snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return fail_message(SBS_ERR_HIP, msg);
    }
    hipLaunchKernelGGL(k_clear_header, dim3(1), dim3(256), 0, s, (uint32_t*)p, (int)(kHeaderBytes / 4));
    e = hipGetLastError();
    if (e != hipSuccess) return fail_message(SBS_ERR_HIP, hipGetErrorString(e));
    it = g_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return SBS_OK;
}

}  // namespace

extern "C" int sbs_sad_disparity_noalloc(const uint8_t* left, const uint8_t* right, int32_t W, int32_t H, int32_t C,
                                         int64_t pitch_bytes, const uint32_t* boundary_idx, int64_t n, int32_t block,
                                         int32_t dmax, uint8_t* out_disp, uint32_t* out_cost, void* stream) {
  sbs_frame f{left, right, W, H, C, pitch_bytes, boundary_idx, n, block, dmax, out_disp, out_cost};
  int st = validate_frame(f);
  if (st != SBS_OK) return st;
  if (n == 0) return SBS_OK;
  const size_t need = workspace_bound(f);
  if (need > (size_t)SBS_SCRATCH_BYTES) {
    char msg[256];
    snprintf(msg, sizeof msg, "frame needs %zu workspace bytes, more than the fixed scratch of %zu bytes", need,
             (size_t)SBS_SCRATCH_BYTES);
    return fail_message(SBS_ERR_WORKSPACE, msg);
  }
  void* ws = nullptr;
  st = scratch_ptr((hipStream_t)stream, &ws);
  if (st != SBS_OK) return st;
  return run_single_into(f, ws, (size_t)SBS_SCRATCH_BYTES, (hipStream_t)stream);
}
