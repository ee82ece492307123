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
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }
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
// The same scans with DPP row shifts and three lane reads instead of one
// LDS permute round trip per doubling step. All 64 lanes must be active.
// A row is 16 lanes; row_shr:n gives lane l the value of lane l - n of its
// row, and 0 where that lies before the row's first lane.
template <int N>
__device__ __forceinline__ uint32_t row_shr(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x110 + N, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t lane_read(uint32_t x, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}
// Inclusive prefix sum over the wavefront.
__device__ __forceinline__ uint32_t wave_incl_sum_dpp(uint32_t x, uint32_t ln) {
  x += row_shr<1>(x);
  x += row_shr<2>(x);
  x += row_shr<4>(x);
  x += row_shr<8>(x);  // prefix sum within each row
  const uint32_t r0 = lane_read(x, 15), r1 = lane_read(x, 31), r2 = lane_read(x, 47);
  const uint32_t row = ln >> 4;
  return x + (row >= 1 ? r0 : 0u) + (row >= 2 ? r1 : 0u) + (row >= 3 ? r2 : 0u);
}
// Inclusive prefix maximum over the wavefront (unsigned).
__device__ __forceinline__ uint32_t wave_incl_max_dpp(uint32_t x, uint32_t ln) {
  x = max(x, row_shr<1>(x));
  x = max(x, row_shr<2>(x));
  x = max(x, row_shr<4>(x));
  x = max(x, row_shr<8>(x));  // prefix maximum within each row
  const uint32_t r0 = lane_read(x, 15), r1 = lane_read(x, 31), r2 = lane_read(x, 47);
  const uint32_t row = ln >> 4;
  // selects, not a chain of conditionals (which compiles to branches)
  return max(max(x, row >= 1 ? r0 : 0u), max(row >= 2 ? r1 : 0u, row >= 3 ? r2 : 0u));
}
// Maximum over the wavefront, the same in every lane.
__device__ __forceinline__ uint32_t wave_max_dpp(uint32_t x, uint32_t ln) {
  return lane_read(wave_incl_max_dpp(x, ln), 63);
}
// Arc dealing: lane L owns the arcs [excl, excl + deg) of a concatenation of
// the lanes' rows (disjoint ranges that cover [0, total)). Returns the lane
// that owns arc j0 + ln, for j0 < total; lanes past total get the last owner.
// mk is 64 words of this wavefront's LDS. Each lane whose range meets
// [j0, j0 + 64) marks where it starts there (position 0 for the range that
// began earlier); a prefix maximum carries each mark forward over its range.
__device__ __forceinline__ uint32_t wave_arc_owner(uint32_t excl, uint32_t deg, uint32_t j0, uint32_t *mk,
                                                   uint32_t ln) {
  mk[ln] = 0u;
  wave_sync();
  if (deg != 0u && excl < j0 + 64u && excl + deg > j0) mk[excl > j0 ? excl - j0 : 0u] = ln + 1u;
  wave_sync();
  const uint32_t m = mk[ln];
  wave_sync();
  return wave_incl_max_dpp(m, ln) - 1u;
}
__device__ __forceinline__ unsigned long long shfl64(unsigned long long x, int src) {
  uint32_t lo = __shfl((uint32_t)x, src), hi = __shfl((uint32_t)(x >> 32), src);
  return ((unsigned long long)hi << 32) | lo;
}

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
