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

// per-level counters (device): new frontier size, arcs out of it, arcs checked;
// with many sources, the union of the new frontier's bits
struct DoCtr {
  unsigned long long nf, mf, checked, bits;
};

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x |= shfl64(x, (int)(lane_id() ^ (uint32_t)d));
  return x;
}

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

// ---- many sources at once: one bit per source in 64-bit words ----------
// visited[v] holds the sources that have reached v, cur[v] those that reached
// it in the current level and nxt[v] those reaching it in the next one. A
// source q's distance to v is the level at which bit q first appears at v.

// Seeds: bit q at sources[q]; a distance output of 0 there.
__global__ void ms_seed_kernel(const int32_t *__restrict__ src, int32_t k, unsigned long long *visited,
                               unsigned long long *cur, const MsQuery *__restrict__ qs) {
  const int q = (int)threadIdx.x;
  if (blockIdx.x != 0 || q >= k) return;
  const uint32_t v = (uint32_t)src[q];
  or_ag(&visited[v], 1ull << q);
  or_ag(&cur[v], 1ull << q);
  if (qs[q].dist) qs[q].dist[v] = 0;
}

// Distance outputs of the bits in nb: level + 1 at w.
__device__ __forceinline__ void ms_write_dist(const MsQuery *__restrict__ qs, unsigned long long nb, uint32_t w,
                                              uint32_t d) {
  while (nb) {
    const int q = __builtin_ctzll(nb);
    nb &= nb - 1;
    if (qs[q].dist) qs[q].dist[w] = (int32_t)d;
  }
}

// Top-down level: one wavefront per frontier vertex, its out-arcs dealt over
// the lanes. A target gains the frontier bits it has not seen (atomicOr on
// visited decides which lane owns each new bit); the first lane to give it a
// next-frontier bit queues it.
__global__ void __launch_bounds__(256) ms_top_down_kernel(const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ tgt,
                                                          const uint32_t *__restrict__ fq, const uint32_t *fq_len,
                                                          unsigned long long *visited,
                                                          const unsigned long long *__restrict__ cur,
                                                          unsigned long long *nxt, uint32_t *nq, uint32_t *nq_len,
                                                          const MsQuery *__restrict__ qs, uint32_t level,
                                                          DoCtr *ctr) {
  const uint32_t len = *fq_len;
  const uint32_t ln = lane_id();
  const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  unsigned long long nf = 0, mf = 0, checked = 0, bits = 0;
  for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < len; i += waves) {
    const uint32_t u = fq[i];
    const unsigned long long c = cur[u];
    const int32_t b = off[u], e = off[u + 1];
    for (int32_t j = b + (int32_t)ln; j < e; j += 64) {
      checked++;
      const uint32_t w = (uint32_t)tgt[j];
      const unsigned long long m = c & ~ld_ag(&visited[w]);
      if (!m) continue;
      const unsigned long long nb = m & ~or_ag(&visited[w], m);
      if (!nb) continue;
      bits |= nb;
      if (or_ag(&nxt[w], nb) == 0ull) {
        nq[add_ag(nq_len, 1u)] = w;
        nf++;
        mf += (unsigned long long)(off[w + 1] - off[w]);
      }
      ms_write_dist(qs, nb, w, level + 1u);
    }
  }
  nf = wave_sum64(nf);
  mf = wave_sum64(mf);
  checked = wave_sum64(checked);
  bits = wave_or64(bits);
  if (ln == 0) {
    if (nf) add_ag(&ctr->nf, nf);
    if (mf) add_ag(&ctr->mf, mf);
    if (checked) add_ag(&ctr->checked, checked);
    if (bits) or_ag(&ctr->bits, bits);
  }
}

// Bottom-up level: every vertex still missing some bit of `active` (the
// bits present in the current frontier: no other bit can arrive this level)
// scans its in-arcs, gathering the frontier bits it misses, and stops once it
// has them all. Only v's own thread writes visited[v] and nxt[v] here.
__global__ void __launch_bounds__(256) ms_bottom_up_kernel(const int32_t *__restrict__ off,
                                                           const int32_t *__restrict__ t_off,
                                                           const int32_t *__restrict__ t_tgt, uint32_t n,
                                                           unsigned long long *visited,
                                                           const unsigned long long *__restrict__ cur,
                                                           unsigned long long *nxt, unsigned long long active,
                                                           const MsQuery *__restrict__ qs, uint32_t level,
                                                           DoCtr *ctr) {
  unsigned long long nf = 0, mf = 0, checked = 0, bits = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
    const uint64_t v = base + lane_id();
    if (v >= n) continue;
    const unsigned long long vis = visited[v];
    const unsigned long long want = active & ~vis;
    unsigned long long acc = 0;
    if (want) {
      const int32_t b = t_off[v], e = t_off[v + 1];
      for (int32_t j = b; j < e; j++) {
        checked++;
        acc |= cur[t_tgt[j]];
        if ((acc & want) == want) break;
      }
      acc &= want;
    }
    nxt[v] = acc;
    if (acc) {
      visited[v] = vis | acc;
      bits |= acc;
      nf++;
      mf += (unsigned long long)(off[v + 1] - off[v]);
      ms_write_dist(qs, acc, (uint32_t)v, level + 1u);
    }
  }
  nf = wave_sum64(nf);
  mf = wave_sum64(mf);
  checked = wave_sum64(checked);
  bits = wave_or64(bits);
  if (lane_id() == 0) {
    if (nf) add_ag(&ctr->nf, nf);
    if (mf) add_ag(&ctr->mf, mf);
    if (checked) add_ag(&ctr->checked, checked);
    if (bits) or_ag(&ctr->bits, bits);
  }
}

// Queue of the vertices with a frontier bit (order unspecified).
__global__ void __launch_bounds__(256) ms_collect_kernel(const unsigned long long *__restrict__ cur, uint32_t n,
                                                         uint32_t *__restrict__ q, uint32_t *qlen) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
    const uint64_t v = base + lane_id();
    const bool in = v < n && cur[v] != 0ull;
    const unsigned long long bal = __ballot(in);
    if (bal) {
      uint32_t at = 0;
      if (lane_id() == 0) at = add_ag(qlen, (uint32_t)__popcll(bal));
      at = __shfl(at, 0);
      if (in) q[at + mbcnt64(bal)] = (uint32_t)v;
    }
  }
}

// Distance outputs start unreached (blockIdx.y = query).
__global__ void ms_fill_dist_kernel(const MsQuery *__restrict__ qs, uint32_t n) {
  int32_t *d = qs[blockIdx.y].dist;
  if (!d) return;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) d[v] = -1;
}

// Reach outputs: bit 0 of mask1[v] = source q reached v.
__global__ void ms_reach_out_kernel(const MsQuery *__restrict__ qs, const unsigned long long *__restrict__ visited,
                                    uint32_t n) {
  unsigned long long *m = qs[blockIdx.y].mask1;
  if (!m) return;
  const int q = (int)blockIdx.y;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) m[v] = (visited[v] >> q) & 1ull;
}

int blocks_for(uint64_t items) {
  uint64_t b = (items + 255) / 256;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(b, 8192));
}

}  // namespace

}  // namespace pg

using namespace pg;

namespace pg {

namespace {
// Holds a gate from construction (or open()) to close(); closes at scope exit.
struct GateHold {
  LevelGate *g;
  bool held = false;
  explicit GateHold(LevelGate *gate) : g(gate) { open(); }
  void open() {
    if (g && !held) {
      g->enter();
      held = true;
    }
  }
  void close() {
    if (g && held) {
      g->leave();
      held = false;
    }
  }
  ~GateHold() { close(); }
};
}  // namespace

int bfs_do_gated(const pasgal_csr *g, const pasgal_csr *gt, int32_t src, int32_t *dist_out, int32_t alpha,
                 int32_t beta, const pasgal_opts *opts, pasgal_stats *stats, LevelGate *gate) {
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
  GateHold hold(gate);  // the set-up below, then one hold per level
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
  hold.close();
  while (nf > 0) {
    hold.open();
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
    hold.close();
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
  hold.open();
  if ((e = hipEventRecord(w->ev1, s)) != hipSuccess) return fail(e);
  if ((e = hipMemcpyAsync(w->h_ctl.p, w->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return fail(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
  hold.close();
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

}  // namespace pg

extern "C" int pasgal_bfs_do(const pasgal_csr *g, const pasgal_csr *gt, int32_t src, int32_t *dist_out,
                             int32_t alpha, int32_t beta, const pasgal_opts *opts, pasgal_stats *stats) {
  return bfs_do_gated(g, gt, src, dist_out, alpha, beta, opts, stats, nullptr);
}

namespace pg {

int ms_bfs_do_gated(const pasgal_csr *g, const pasgal_csr *gt, int32_t k, const int32_t *src, const MsQuery *qs,
                    unsigned long long *visited_out, int32_t alpha, int32_t beta, const pasgal_opts *opts,
                    pasgal_stats *stats, LevelGate *gate) {
  if (!csr_valid(g) || k < 1 || k > 64 || !src || !qs || !opts_valid(opts)) return PASGAL_EINVAL;
  if (gt && (!csr_valid(gt) || gt->n != g->n || gt->m != g->m)) return PASGAL_EINVAL;
  for (int q = 0; q < k; q++)
    if (src[q] < 0 || src[q] >= g->n) return PASGAL_EINVAL;
  const pasgal_csr *t = gt ? gt : g;
  Opts o = resolve_opts(opts);
  if (o.flags & PASGAL_FLAG_ASYNC) return PASGAL_EINVAL;
  // bottom-up levels of several sources stop only once every missing bit is
  // found, so they cost more than one source's: go bottom-up later (RMAT-24,
  // 16 sources: 29 ms at alpha 14, 156 ms at 100 when one source is a hub;
  // 64 sources: 53 against 180 ms)
  const double a = alpha > 0 ? (double)alpha : (alpha == 0 ? (k == 1 ? 100.0 : 14.0) : 0.0);
  const double bt = beta > 0 ? (double)beta : (beta == 0 ? 24.0 : 0.0);
  Workspace *w = workspace_for(o.stream);
  if (!w) return PASGAL_ENOMEM;
  std::lock_guard<std::mutex> lk(w->mu);
  if (int arc = collect_async(*w)) return arc;
  hipStream_t s = o.stream;
  const uint64_t n = (uint64_t)g->n, m = (uint64_t)g->m;
  int rc;
  // visited | cur | nxt words, two queues, counters, the query table and sources
  const size_t bq = sizeof(MsQuery) * (size_t)k, bs = 4 * (size_t)k;
  if ((rc = grow(w->tmp_state, 8 * n)) || (rc = grow(w->fval[0], 8 * n)) || (rc = grow(w->fval[1], 8 * n)) ||
      (rc = grow(w->pf[0], 4 * n)) || (rc = grow(w->pf[1], 4 * n)) || (rc = grow(w->aux, sizeof(DoCtr) + 16)) ||
      (rc = grow(w->seeds, bq + bs + 16)) || (rc = grow_host(w->h_aux, sizeof(DoCtr) + 16)) ||
      (rc = grow_host(w->h_stage, bq + bs + 16)))
    return rc;
  unsigned long long *visited = visited_out ? visited_out : (unsigned long long *)w->tmp_state.p;
  unsigned long long *cur = (unsigned long long *)w->fval[0].p, *nxt = (unsigned long long *)w->fval[1].p;
  uint32_t *qa = (uint32_t *)w->pf[0].p, *qb = (uint32_t *)w->pf[1].p;
  DoCtr *ctr = (DoCtr *)w->aux.p;
  uint32_t *qlen = (uint32_t *)((uint8_t *)w->aux.p + sizeof(DoCtr));
  MsQuery *dqs = (MsQuery *)w->seeds.p;
  int32_t *dsrc = (int32_t *)((uint8_t *)w->seeds.p + bq);
  DoCtr *h = (DoCtr *)w->h_aux.p;
  uint32_t *h_len = (uint32_t *)((uint8_t *)w->h_aux.p + sizeof(DoCtr));
  memcpy(w->h_stage.p, qs, bq);
  memcpy((uint8_t *)w->h_stage.p + bq, src, bs);
  unsigned long long bfs_mask = 0, reach_any = 0;
  for (int q = 0; q < k; q++) {
    if (qs[q].dist) bfs_mask |= 1ull << q;
    if (qs[q].mask1) reach_any = 1;
  }
  const unsigned long long active = k == 64 ? ~0ull : ((1ull << k) - 1ull);
  hipError_t e;
  auto fail = [&](hipError_t x) { return hip_fail(x); };
  GateHold hold(gate);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
  if ((e = hipEventRecord(w->ev0, s)) != hipSuccess) return fail(e);
  if ((e = hipMemcpyAsync(w->seeds.p, w->h_stage.p, bq + bs, hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail(e);
  if ((e = launch_fill_u64(visited, n, 0ull, s)) != hipSuccess) return fail(e);
  if ((e = launch_fill_u64(cur, n, 0ull, s)) != hipSuccess) return fail(e);
  if ((e = launch_fill_u64(nxt, n, 0ull, s)) != hipSuccess) return fail(e);
  (void)hipGetLastError();
  if (bfs_mask) hipLaunchKernelGGL(ms_fill_dist_kernel, dim3(blocks_for(n / 4 + 1), k), dim3(256), 0, s, dqs, (uint32_t)n);
  hipLaunchKernelGGL(ms_seed_kernel, dim3(1), dim3(64), 0, s, dsrc, k, visited, cur, dqs);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  // the seed queue: the distinct sources
  if ((e = launch_fill_u32(qlen, 1, 0u, s)) != hipSuccess) return fail(e);
  if ((e = launch_fill_u32((uint32_t *)ctr, sizeof(DoCtr) / 4, 0u, s)) != hipSuccess) return fail(e);
  (void)hipGetLastError();
  hipLaunchKernelGGL(ms_collect_kernel, dim3(blocks_for(n)), dim3(256), 0, s, (const unsigned long long *)cur,
                     (uint32_t)n, qa, qlen);
  hipLaunchKernelGGL(degsum_kernel, dim3(blocks_for(n / 4 + 1)), dim3(256), 0, s, g->offsets, (const uint32_t *)qa,
                     (const uint32_t *)qlen, ctr);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  if ((e = hipMemcpyAsync(h, ctr, sizeof(DoCtr), hipMemcpyDeviceToHost, s)) != hipSuccess) return fail(e);
  if ((e = hipMemcpyAsync(h_len, qlen, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return fail(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
  if ((e = hipEventRecord(w->evk, s)) != hipSuccess) return fail(e);
  hold.close();

  uint64_t nf = *h_len, mf = h->mf, seen_arcs = h->mf;
  uint32_t level = 0;
  bool bottom_up = false, have_queue = true;
  int64_t checked = 0, maxf = (int64_t)nf, levels = 0;
  unsigned long long fbits = active;  // bits present in the current frontier
  while (nf > 0) {
    hold.open();
    const uint64_t mu = m - std::min(m, seen_arcs);
    if (!bottom_up && a > 0.0 && (double)mf > (double)mu / a) {
      bottom_up = true;
    } else if (bottom_up && bt > 0.0 && (double)nf < (double)n / bt) {
      bottom_up = false;
      have_queue = false;
    }
    if ((e = launch_fill_u32((uint32_t *)ctr, sizeof(DoCtr) / 4, 0u, s)) != hipSuccess) return fail(e);
    if (bottom_up) {
      (void)hipGetLastError();
      hipLaunchKernelGGL(ms_bottom_up_kernel, dim3(blocks_for(n)), dim3(256), 0, s, g->offsets, t->offsets,
                         t->targets, (uint32_t)n, visited, (const unsigned long long *)cur, nxt, fbits, dqs, level,
                         ctr);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    } else {
      if (!have_queue) {
        if ((e = launch_fill_u32(qlen, 1, 0u, s)) != hipSuccess) return fail(e);
        (void)hipGetLastError();
        hipLaunchKernelGGL(ms_collect_kernel, dim3(blocks_for(n)), dim3(256), 0, s, (const unsigned long long *)cur,
                           (uint32_t)n, qa, qlen);
        if ((e = hipGetLastError()) != hipSuccess) return fail(e);
        have_queue = true;
      }
      // the next frontier's words start empty; its queue gets the length
      if ((e = launch_fill_u64(nxt, n, 0ull, s)) != hipSuccess) return fail(e);
      uint32_t *nlen = qlen + 1;
      if ((e = launch_fill_u32(nlen, 1, 0u, s)) != hipSuccess) return fail(e);
      (void)hipGetLastError();
      const uint64_t waves = std::min<uint64_t>(nf, 8192ull * 4);
      hipLaunchKernelGGL(ms_top_down_kernel, dim3((int)((waves + 3) / 4)), dim3(256), 0, s, g->offsets, g->targets,
                         (const uint32_t *)qa, (const uint32_t *)qlen, visited, (const unsigned long long *)cur, nxt,
                         qb, nlen, dqs, level, ctr);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      if ((e = hipMemcpyAsync(qlen, nlen, 4, hipMemcpyDeviceToDevice, s)) != hipSuccess) return fail(e);
      std::swap(qa, qb);
    }
    if ((e = hipMemcpyAsync(h, ctr, sizeof(DoCtr), hipMemcpyDeviceToHost, s)) != hipSuccess) return fail(e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
    hold.close();
    nf = h->nf;
    mf = h->mf;
    fbits = h->bits;
    checked += (int64_t)h->checked;
    seen_arcs += mf;
    maxf = std::max<int64_t>(maxf, (int64_t)nf);
    std::swap(cur, nxt);
    level++;
    levels++;
    if (nf > n || level > n + 1) return PASGAL_EINTERNAL;
  }
  hold.open();
  if (reach_any) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(ms_reach_out_kernel, dim3(blocks_for(n / 4 + 1), k), dim3(256), 0, s, dqs,
                       (const unsigned long long *)visited, (uint32_t)n);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  }
  if ((e = hipEventRecord(w->ev1, s)) != hipSuccess) return fail(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
  hold.close();
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->rounds = levels;
    stats->arcs_scanned = checked;
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

}  // namespace pg

extern "C" int pasgal_bfs_do_multi(const pasgal_csr *g, const pasgal_csr *gt, int32_t k, const int32_t *sources,
                                   int32_t *dist_out, uint64_t *reach_out, int32_t alpha, int32_t beta,
                                   const pasgal_opts *opts, pasgal_stats *stats) {
  if (!csr_valid(g) || k < 1 || k > 64 || !sources) return PASGAL_EINVAL;
  MsQuery qs[64];
  for (int q = 0; q < k; q++) {
    qs[q].dist = dist_out ? dist_out + (size_t)q * (size_t)g->n : nullptr;
    qs[q].mask1 = nullptr;
  }
  return ms_bfs_do_gated(g, gt, k, sources, qs, (unsigned long long *)reach_out, alpha, beta, opts, stats, nullptr);
}
