// Opt-in range validation of operand values (debug mode).
//
// The transforms and element-wise operations take operand values in
// [0, f q) for a per-call input factor f (Sections 3 and 4 state these as
// preconditions); out-of-range values give unspecified output and are not
// checked on the hot path.  With validation on (environment NTT_VALIDATE=1 at
// the first call, or ntt_set_validate(1)), every entry point that reads
// operand values first checks them on the device and returns NTT_ERANGE when
// one is out of range.  The check reduces into a per-device flag with vector
// atomics, then waits for the caller's stream: it is a debugging aid, not
// for graph capture or for timing.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"
#include "ntt_common.h"

namespace nttamd {

struct RangeBounds {
  u64 b[NTT_MAX_LIMBS];       // exclusive upper bound of limb l's values
};

template <typename T>
__global__ void range_check_kernel(const T* data, u64 n, u64 total, u32 num_limbs, const RangeBounds bounds,
                                   u32* flag) {
  u32 bad = 0;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (u64)gridDim.x * blockDim.x) {
    const u32 limb = (u32)((i / n) % num_limbs);
    bad |= (u64)data[i] >= bounds.b[limb] ? 1u : 0u;
  }
  if (bad) atomicOr(flag, 1u);
}

__global__ void clear_flag_kernel(u32* flag) { *flag = 0u; }

namespace {

std::atomic<int> g_validate{-1};
std::mutex g_flag_mu;
std::vector<u32*> g_flags;     // per device, allocated on first use

u32* device_flag() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_flag_mu);
  if ((size_t)dev >= g_flags.size()) g_flags.resize(dev + 1, nullptr);
  if (!g_flags[dev]) {
    u32* p = nullptr;
    if (hipMalloc(&p, 256) != hipSuccess) return nullptr;
    g_flags[dev] = p;
  }
  return g_flags[dev];
}

}  // namespace

bool validate_enabled() {
  int v = g_validate.load(std::memory_order_relaxed);
  if (v < 0) {
    const char* e = getenv("NTT_VALIDATE");
    v = (e && strcmp(e, "1") == 0) ? 1 : 0;
    int expected = -1;
    g_validate.compare_exchange_strong(expected, v);
    v = g_validate.load();
  }
  return v == 1;
}

void set_validate(bool on) { g_validate.store(on ? 1 : 0); }

void free_validate_buffers() {
  std::lock_guard<std::mutex> lk(g_flag_mu);
  for (u32*& p : g_flags) {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
}

ntt_status check_range(const void* data, int bits, uint64_t n, const uint64_t* moduli, uint64_t num_limbs,
                       uint64_t num_polys, uint64_t factor, hipStream_t stream) {
  if (!validate_enabled()) return NTT_OK;
  if (!data || !moduli || n == 0 || num_limbs == 0 || num_limbs > NTT_MAX_LIMBS || num_polys == 0)
    return NTT_OK;                          // argument errors are reported by the call itself
  u32* flag = device_flag();
  if (!flag) return NTT_EDEVICE;
  RangeBounds bounds;
  for (uint64_t l = 0; l < num_limbs; ++l) {
    const unsigned __int128 b = (unsigned __int128)moduli[l] * factor;
    bounds.b[l] = b > ~0ull ? ~0ull : (u64)b;
  }
  const uint64_t total = n * num_limbs * num_polys;
  const unsigned threads = 256;
  const uint64_t want = (total + threads - 1) / threads;
  const unsigned blocks = (unsigned)(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, stream, flag);
  if (bits == 32)
    hipLaunchKernelGGL(range_check_kernel<u32>, dim3(blocks), dim3(threads), 0, stream,
                       static_cast<const u32*>(data), (u64)n, (u64)total, (u32)num_limbs, bounds, flag);
  else
    hipLaunchKernelGGL(range_check_kernel<u64>, dim3(blocks), dim3(threads), 0, stream,
                       static_cast<const u64*>(data), (u64)n, (u64)total, (u32)num_limbs, bounds, flag);
  if (hipGetLastError() != hipSuccess) return NTT_EDEVICE;
  u32 host = 0;
  if (hipMemcpyAsync(&host, flag, sizeof(u32), hipMemcpyDeviceToHost, stream) != hipSuccess) return NTT_EDEVICE;
  if (hipStreamSynchronize(stream) != hipSuccess) return NTT_EDEVICE;
  return host ? NTT_ERANGE : NTT_OK;
}

}  // namespace nttamd
