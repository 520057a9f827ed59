// noalloc.hip -- moment fields into host memory without any device allocation,
// for callers that cannot allocate (code between HIP graph captures, serving
// loops, harnesses that forbid hipMalloc).
//
// rflbm_get_moments into a host array stages the fields in a device buffer of
// the whole field size that it allocates and frees on every call.  The variant
// here passes them through a fixed device array instead, `scratch` below,
// chunk by chunk: the moments kernel fills the array for a range of nodes, the
// fields of that range are copied to their places in the host array, and the
// next range follows on the same stream.  Values are bit for bit those of
// rflbm_get_moments (same kernel).
//
// The array exists once per GPU for the life of the process.  In host code its
// name is only a stand-in: the device address of each GPU's copy is looked up
// once per device (hipGetSymbolAddress with that device current) and only that
// address is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rflbm.h"
#include "kernels.hpp"
#include "lattice.hpp"

namespace rflbm {
namespace {

constexpr size_t kScratchBytes = size_t{8} << 20;  // 8 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex[kMaxDevices];
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up on first use; the caller
// holds g_scratch_mutex[device].
rflbm_status scratch_on(int device, void** out) {
  if (!g_scratch_ptr[device]) {
    int current = 0;
    RFLBM_HIP(hipGetDevice(&current));
    if (current != device) RFLBM_HIP(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (current != device) (void)hipSetDevice(current);
    if (e != hipSuccess) return hip_fail(RFLBM_EHIP, "hipGetSymbolAddress(scratch)", e);
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return RFLBM_OK;
}

}  // namespace
}  // namespace rflbm

using namespace rflbm;

extern "C" rflbm_status rflbm_get_moments_host_noalloc(rflbm_lattice* L, uint32_t mask, float* dst) {
  if (!L) return fail(RFLBM_EINVAL, "lattice is NULL");
  if (!dst) return fail(RFLBM_EINVAL, "dst is NULL");
  if (mask == 0 || (mask & ~7u)) return fail(RFLBM_EINVAL, "mask must select RHO, J and/or PI");
  const uint64_t nf = ((mask & 1u) ? 1 : 0) + ((mask & 2u) ? 3 : 0) + ((mask & 4u) ? 6 : 0);
  if (L->device < 0 || L->device >= kMaxDevices) return fail(RFLBM_EINVAL, "device index out of range");
  // one call at a time per GPU in this process: the array is shared
  std::lock_guard<std::mutex> lock(g_scratch_mutex[L->device]);
  void* ptr = nullptr;
  if (rflbm_status s = scratch_on(L->device, &ptr)) return s;
  float* stage = static_cast<float*>(ptr);
  const uint64_t N = node_count(L->p);
  // nodes per chunk: every selected field of a chunk fits the array
  const uint64_t chunk = kScratchBytes / (nf * sizeof(float)) / 256 * 256;
  const GatherArgs g = gather_args(L, L->p, L->t);
  for (uint64_t n0 = 0; n0 < N; n0 += chunk) {
    const uint64_t cnt = N - n0 < chunk ? N - n0 : chunk;
    RFLBM_HIP(launch_get_moments_range(L->p.storage, g, mask, n0, cnt, stage, cnt, L->stream));
    for (uint64_t f = 0; f < nf; ++f)
      RFLBM_HIP(hipMemcpyAsync(dst + f * N + n0, stage + f * cnt, cnt * sizeof(float), hipMemcpyDeviceToHost,
                               L->stream));
  }
  RFLBM_HIP(hipStreamSynchronize(L->stream));
  return RFLBM_OK;
}
