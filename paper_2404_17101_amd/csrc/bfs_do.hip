// bfs_do.hip -- direction-optimizing BFS (the paper's BFS also uses the
// direction optimization of Beamer et al.; Parallel BFS paragraph).
//
// Level-synchronous. A level is expanded
//  * top-down while the frontier is small: frontier vertices relax their
//    out-arcs and an atomicCAS from "unreached" admits each vertex once (the
//    plain level kernel), or
//  * bottom-up while it is large: every unreached vertex scans its in-arcs
//    (rows of G^T) and stops at the first in-neighbour found in the frontier
//    (dist == level). Only the vertex's own thread writes its distance, so no
//    atomic is needed, and most scans stop after a few arcs.
// Switching rule (Beamer): top-down -> bottom-up when the arcs out of the
// frontier exceed 1/alpha of the arcs out of the unreached vertices;
// bottom-up -> top-down when the frontier holds fewer than n/beta vertices.
// Beamer's alpha = 14 was set for CPUs; here a bottom-up level costs plain
// loads only, so switching earlier pays: alpha = 100 by default (RMAT-24:
// 7.9 ms against 15 ms at alpha = 14), beta = 24.
// The frontier of a level is the set {v : dist[v] == level}; a top-down level
// after a bottom-up one first collects it into a queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "devutil.h"
#include "engine.h"
#include "kern.h"
#include "pasgal.h"

namespace pg {

namespace {

// per-level counters (device): new frontier size, arcs out of it, arcs checked
struct DoCtr {
  unsigned long long nf, mf, checked, pad;
};

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += shfl64(x, (int)(lane_id() ^ (uint32_t)d));
  return x;
}

__global__ void do_seed_kernel(uint32_t *dist, uint32_t *queue, uint32_t src) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    dist[src] = 0u;
    queue[0] = src;
  }
}

// Arcs out of the queue's vertices (the queue's length is read on the device).
__global__ void __launch_bounds__(256) degsum_kernel(const int32_t *__restrict__ off,
                                                     const uint32_t *__restrict__ q, const uint32_t *qlen,
                                                     DoCtr *ctr) {
  const uint32_t len = *qlen;
  unsigned long long s = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < len; base += stride) {
    const uint64_t i = base + lane_id();
    if (i < len) {
      const uint32_t v = q[i];
      s += (unsigned long long)(off[v + 1] - off[v]);
    }
  }
  s = wave_sum64(s);
  if (lane_id() == 0 && s) add_ag(&ctr->mf, s);
}

// Bottom-up level: every unreached vertex looks for an in-neighbour at
// distance `level` and stops at the first one.
__global__ void __launch_bounds__(256) bottom_up_kernel(const int32_t *__restrict__ off,
                                                        const int32_t *__restrict__ t_off,
                                                        const int32_t *__restrict__ t_tgt, uint32_t n,
                                                        uint32_t *dist, uint32_t level, DoCtr *ctr) {
  unsigned long long nf = 0, mf = 0, checked = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
    const uint64_t v = base + lane_id();
    if (v < n && dist[v] == INF32) {
      const int32_t b = t_off[v], e = t_off[v + 1];
      for (int32_t k = b; k < e; k++) {
        checked++;
        if (dist[t_tgt[k]] == level) {
          dist[v] = level + 1u;
          nf++;
          mf += (unsigned long long)(off[v + 1] - off[v]);
          break;
        }
      }
    }
  }
  nf = wave_sum64(nf);
  mf = wave_sum64(mf);
  checked = wave_sum64(checked);
  if (lane_id() == 0) {
    if (nf) add_ag(&ctr->nf, nf);
    if (mf) add_ag(&ctr->mf, mf);
    if (checked) add_ag(&ctr->checked, checked);
  }
}

// Queue of the vertices at distance `level` (order unspecified).
__global__ void __launch_bounds__(256) collect_kernel(const uint32_t *__restrict__ dist, uint32_t n, uint32_t level,
                                                      uint32_t *__restrict__ q, uint32_t *qlen) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
    const uint64_t v = base + lane_id();
    const bool in = v < n && dist[v] == level;
    const unsigned long long bal = __ballot(in);
    if (bal) {
      uint32_t at = 0;
      if (lane_id() == 0) at = add_ag(qlen, (uint32_t)__popcll(bal));
      at = __shfl(at, 0);
      if (in) q[at + mbcnt64(bal)] = (uint32_t)v;
    }
  }
}

int blocks_for(uint64_t items) {
  uint64_t b = (items + 255) / 256;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(b, 8192));
}

}  // namespace

}  // namespace pg

using namespace pg;

extern "C" int pasgal_bfs_do(const pasgal_csr *g, const pasgal_csr *gt, int32_t src, int32_t *dist_out,
                             int32_t alpha, int32_t beta, const pasgal_opts *opts, pasgal_stats *stats) {
  if (!csr_valid(g) || !dist_out || src < 0 || src >= g->n || !opts_valid(opts)) return PASGAL_EINVAL;
  if (gt && (!csr_valid(gt) || gt->n != g->n || gt->m != g->m)) return PASGAL_EINVAL;
  const pasgal_csr *t = gt ? gt : g;
  Opts o = resolve_opts(opts);
  if (o.flags & PASGAL_FLAG_ASYNC) return PASGAL_EINVAL;
  const double a = alpha > 0 ? (double)alpha : (alpha == 0 ? 100.0 : 0.0);  // 0.0: never bottom-up
  const double bt = beta > 0 ? (double)beta : (beta == 0 ? 24.0 : 0.0);   // 0.0: never back to top-down
  Workspace *w = workspace_for(o.stream);
  if (!w) return PASGAL_ENOMEM;
  std::lock_guard<std::mutex> lk(w->mu);
  if (int arc = collect_async(*w)) return arc;
  hipStream_t s = o.stream;
  int rc;
  if (o.flags & PASGAL_FLAG_VALIDATE) {
    if ((rc = validate_csr_device(*w, g, s))) return rc;
    if (gt && (rc = validate_csr_device(*w, gt, s))) return rc;
  }
  const uint64_t n = (uint64_t)g->n, m = (uint64_t)g->m;
  if ((rc = grow(w->pf[0], 4 * n)) || (rc = grow(w->pf[1], 4 * n)) || (rc = grow(w->ctl, sizeof(Ctl))) ||
      (rc = grow(w->aux, sizeof(DoCtr) + 16)) || (rc = grow_host(w->h_ctl, sizeof(Ctl))) ||
      (rc = grow_host(w->h_aux, sizeof(DoCtr) + 16)))
    return rc;
  Ctl *ctl = (Ctl *)w->ctl.p;
  DoCtr *ctr = (DoCtr *)w->aux.p;
  uint32_t *qlen = (uint32_t *)((uint8_t *)w->aux.p + sizeof(DoCtr));  // queue length for collect/degsum
  DoCtr *h = (DoCtr *)w->h_aux.p;
  uint32_t *dist = (uint32_t *)dist_out;
  hipError_t e;
  auto fail = [&](hipError_t x) { return hip_fail(x); };
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
  if ((e = hipEventRecord(w->ev0, s)) != hipSuccess) return fail(e);
  if ((e = launch_fill_u32(dist, n, INF32, s)) != hipSuccess) return fail(e);
  if ((e = launch_fill_u32((uint32_t *)w->ctl.p, sizeof(Ctl) / 4, 0u, s)) != hipSuccess) return fail(e);
  if ((e = launch_fill_u32((uint32_t *)w->aux.p, (sizeof(DoCtr) + 16) / 4, 0u, s)) != hipSuccess) return fail(e);
  (void)hipGetLastError();
  hipLaunchKernelGGL(do_seed_kernel, dim3(1), dim3(64), 0, s, dist, (uint32_t *)w->pf[0].p, (uint32_t)src);
  // level-0 frontier {src}: its arcs
  if ((e = launch_fill_u32(qlen, 1, 1u, s)) != hipSuccess) return fail(e);
  hipLaunchKernelGGL(degsum_kernel, dim3(1), dim3(256), 0, s, g->offsets, (const uint32_t *)w->pf[0].p,
                     (const uint32_t *)qlen, ctr);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  if ((e = hipMemcpyAsync(h, ctr, sizeof(DoCtr), hipMemcpyDeviceToHost, s)) != hipSuccess) return fail(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
  if ((e = hipEventRecord(w->evk, s)) != hipSuccess) return fail(e);

  uint64_t nf = 1, mf = h->mf, seen_arcs = h->mf;
  uint32_t level = 0;
  int cur = 0;  // queue buffer of the current frontier (top-down)
  bool bottom_up = false, have_queue = true;
  int64_t expansions = 0, checked = 0, maxf = 1, visited = 1;
  uint32_t *h_td = (uint32_t *)((uint8_t *)w->h_aux.p + sizeof(DoCtr));  // top-down level: next frontier size
  while (nf > 0) {
    const uint64_t mu = m - std::min(m, seen_arcs);  // arcs out of unreached vertices
    if (!bottom_up && a > 0.0 && (double)mf > (double)mu / a) {
      bottom_up = true;
    } else if (bottom_up && bt > 0.0 && (double)nf < (double)n / bt) {
      bottom_up = false;
      have_queue = false;
    }
    if ((e = launch_fill_u32((uint32_t *)w->aux.p, sizeof(DoCtr) / 4, 0u, s)) != hipSuccess) return fail(e);
    if (bottom_up) {
      (void)hipGetLastError();
      hipLaunchKernelGGL(bottom_up_kernel, dim3(blocks_for(n)), dim3(256), 0, s, g->offsets, t->offsets, t->targets,
                         (uint32_t)n, dist, level, ctr);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      if ((e = hipMemcpyAsync(h, ctr, sizeof(DoCtr), hipMemcpyDeviceToHost, s)) != hipSuccess) return fail(e);
    } else {
      if (!have_queue) {
        if ((e = launch_fill_u32(qlen, 1, 0u, s)) != hipSuccess) return fail(e);
        (void)hipGetLastError();
        hipLaunchKernelGGL(collect_kernel, dim3(blocks_for(n)), dim3(256), 0, s, (const uint32_t *)dist,
                           (uint32_t)n, level, (uint32_t *)w->pf[cur].p, qlen);
        if ((e = hipGetLastError()) != hipSuccess) return fail(e);
        have_queue = true;
      }
      expansions += (int64_t)nf;
      // the level kernel appends to cnt[(level+1)%3]; after bottom-up levels
      // that slot was not cleared by a previous top-down level
      uint32_t *next_cnt = &ctl->cnt[(level + 1) % 3];
      if ((e = launch_fill_u32(next_cnt, 1, 0u, s)) != hipSuccess) return fail(e);
      if ((e = launch_plain_bfs_level(g->offsets, g->targets, dist, (const uint32_t *)w->pf[cur].p, (uint32_t)nf,
                                      (uint32_t *)w->pf[cur ^ 1].p, ctl->cnt, level, ctl, s)) != hipSuccess)
        return fail(e);
      (void)hipGetLastError();
      hipLaunchKernelGGL(degsum_kernel, dim3(blocks_for(n / 4 + 1)), dim3(256), 0, s, g->offsets,
                         (const uint32_t *)w->pf[cur ^ 1].p, (const uint32_t *)next_cnt, ctr);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      if ((e = hipMemcpyAsync(h_td, next_cnt, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return fail(e);
      if ((e = hipMemcpyAsync(h, ctr, sizeof(DoCtr), hipMemcpyDeviceToHost, s)) != hipSuccess) return fail(e);
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
    if (bottom_up) {
      nf = h->nf;
      checked += (int64_t)h->checked;
    } else {
      nf = *h_td;
      cur ^= 1;
    }
    mf = h->mf;
    seen_arcs += mf;
    visited += (int64_t)nf;
    maxf = std::max<int64_t>(maxf, (int64_t)nf);
    level++;
    if (nf > n) return PASGAL_EINTERNAL;
  }
  if ((e = hipEventRecord(w->ev1, s)) != hipSuccess) return fail(e);
  if ((e = hipMemcpyAsync(w->h_ctl.p, w->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return fail(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
  if (stats) {
    const Ctl &c = *(const Ctl *)w->h_ctl.p;
    memset(stats, 0, sizeof(*stats));
    stats->rounds = level;
    stats->expansions = expansions;
    stats->arcs_scanned = (int64_t)c.stats[ST_ARCS] + checked;
    stats->relax_success = visited - 1;
    stats->published = (int64_t)c.stats[ST_SUCCESS];
    stats->max_frontier = maxf;
    float ms = 0, kms = 0;
    hipEventElapsedTime(&ms, w->ev0, w->ev1);
    hipEventElapsedTime(&kms, w->evk, w->ev1);
    (void)hipGetLastError();
    stats->device_ms = ms;
    stats->kernel_ms = kms;
  }
  return PASGAL_OK;
}
