// probe.hip -- memory-latency probe behind pasgal_probe_latency: the time of
// one dependent device-memory access, which bounds a traversal from below
// (a BFS whose source has eccentricity e makes at least e accesses one after
// the other). Measurement support only; no traversal uses it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "devutil.h"
#include "engine.h"
#include "kern.h"
#include "pasgal.h"

namespace pg {
namespace {

// A bijection of [0, mask + 1) for mask + 1 a power of two: odd multipliers
// and right xorshifts, each invertible on k-bit values, so consecutive
// positions land far apart and every slot is used once.
__device__ __forceinline__ uint32_t chase_perm(uint32_t i, uint32_t mask) {
  uint32_t x = (i * 0x9E3779B1u) & mask;
  x ^= x >> 7;
  x = (x * 0x85EBCA77u) & mask;
  x ^= x >> 13;
  x = (x * 0xC2B2AE3Du) & mask;
  x ^= x >> 11;
  return x;
}

// next[perm(i)] = perm(i + 1): one cycle through all slots in permuted order.
__global__ void chase_build_kernel(uint32_t *next, uint32_t mask) {
  const uint64_t n = (uint64_t)mask + 1u;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    next[chase_perm((uint32_t)i, mask)] = chase_perm((uint32_t)((i + 1u) & mask), mask);
}

// One lane walks the cycle; out[0] = wall-clock ticks of the walk, out[1] =
// the last slot (keeps the walk observable).
template <int KIND>
__global__ void chase_kernel(uint32_t *next, uint32_t start, uint32_t steps, unsigned long long *out) {
  if (threadIdx.x != 0) return;
  uint32_t idx = start;
  const long long t0 = wall_clock64();
  for (uint32_t s = 0; s < steps; ++s) {
    if (KIND == PASGAL_PROBE_LOAD)
      idx = next[idx];
    else if (KIND == PASGAL_PROBE_COHERENT)
      idx = ld_ag(&next[idx]);
    else
      idx = add_ag(&next[idx], 0u);
  }
  __builtin_amdgcn_s_waitcnt(0);
  const long long t1 = wall_clock64();
  out[0] = (unsigned long long)(t1 - t0);
  out[1] = idx;
}

}  // namespace
}  // namespace pg

using namespace pg;

extern "C" int pasgal_probe_latency(int64_t bytes, int32_t steps, int32_t kind, double *ns_per_hop,
                                    const pasgal_opts *opts) {
  if (!ns_per_hop || bytes < 4096 || bytes > (1ll << 32) || steps < 1 || steps > (1 << 24) ||
      kind < PASGAL_PROBE_LOAD || kind > PASGAL_PROBE_ATOMIC || !opts_valid(opts))
    return PASGAL_EINVAL;
  const Opts o = resolve_opts(opts);
  hipStream_t s = o.stream;
  uint32_t bits = 0;
  while (bits < 30 && (4ll << (bits + 1)) <= bytes) bits++;
  const uint32_t mask = (1u << bits) - 1u;
  uint32_t *next = nullptr;
  unsigned long long *dout = nullptr;
  hipError_t e = hipMalloc(&next, 4ull << bits);
  if (e != hipSuccess) return hip_fail(e);
  int rc = PASGAL_OK;
  unsigned long long hout[2] = {0, 0};
  if ((e = hipMalloc(&dout, sizeof(hout))) != hipSuccess) {
    rc = hip_fail(e);
  } else {
    const uint64_t n = (uint64_t)mask + 1u;
    const unsigned grid = (unsigned)std::min<uint64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(chase_build_kernel, dim3(grid), dim3(256), 0, s, next, mask);
    e = hipGetLastError();
    const uint32_t start = 0;  // any slot lies on the cycle
    if (e == hipSuccess) {
      if (kind == PASGAL_PROBE_LOAD)
        hipLaunchKernelGGL(chase_kernel<PASGAL_PROBE_LOAD>, dim3(1), dim3(64), 0, s, next, start, (uint32_t)steps, dout);
      else if (kind == PASGAL_PROBE_COHERENT)
        hipLaunchKernelGGL(chase_kernel<PASGAL_PROBE_COHERENT>, dim3(1), dim3(64), 0, s, next, start, (uint32_t)steps,
                           dout);
      else
        hipLaunchKernelGGL(chase_kernel<PASGAL_PROBE_ATOMIC>, dim3(1), dim3(64), 0, s, next, start, (uint32_t)steps,
                           dout);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hout, dout, sizeof(hout), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e);
    hipFree(dout);
  }
  hipFree(next);
  if (rc != PASGAL_OK) return rc;
  *ns_per_hop = (double)hout[0] * 1e6 / (double)dev_info().wall_khz / (double)steps;
  return PASGAL_OK;
}
