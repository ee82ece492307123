// devutil.h -- device helpers shared by the gfx950 kernels: agent-scope
// relaxed atomics (coherent across the XCDs without cache maintenance),
// wavefront (64-lane) scans and reductions, and a 256-thread block scan.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pg {

#define AG __HIP_MEMORY_SCOPE_AGENT
constexpr uint32_t INF32 = 0xFFFFFFFFu;

template <class T>
__device__ __forceinline__ T ld_ag(T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, AG);
}
template <class T>
__device__ __forceinline__ void st_ag(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, AG);
}
template <class T>
__device__ __forceinline__ T add_ag(T *p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, AG);
}
template <class T>
__device__ __forceinline__ T or_ag(T *p, T v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, AG);
}
template <class T>
__device__ __forceinline__ T min_ag(T *p, T v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, AG);
}
template <class T>
__device__ __forceinline__ T max_ag(T *p, T v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, AG);
}
template <class T>
__device__ __forceinline__ T xchg_ag(T *p, T v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, AG);
}
__device__ __forceinline__ uint32_t cas_ag(uint32_t *p, uint32_t expect, uint32_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED, AG);
  return expect;  // old value
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t mbcnt64(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, uint32_t ln) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d);
    if (ln >= (uint32_t)d) x += y;
  }
  return x;
}
__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = max(x, (uint32_t)__shfl_xor(x, d));
  return x;
}
__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = min(x, (uint32_t)__shfl_xor(x, d));
  return x;
}
__device__ __forceinline__ unsigned long long shfl64(unsigned long long x, int src) {
  uint32_t lo = __shfl((uint32_t)x, src), hi = __shfl((uint32_t)(x >> 32), src);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// Exclusive scan of one value per thread over a 256-thread workgroup; total
// receives the sum of all 256 values.
__device__ inline int32_t block_excl_scan_256(int32_t x, int32_t &total) {
  __shared__ int32_t wsum[4];
  const uint32_t ln = lane_id(), wid = threadIdx.x >> 6;
  int32_t incl = (int32_t)wave_incl_scan((uint32_t)x, ln);
  if (ln == 63) wsum[wid] = incl;
  __syncthreads();
  int32_t off = 0, tot = 0;
  for (uint32_t w = 0; w < 4; w++) {
    if (w < wid) off += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  total = tot;
  return off + incl - x;
}

}  // namespace pg
