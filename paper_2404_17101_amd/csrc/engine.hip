// engine.hip -- host side of libpasgal.so: argument checks, grow-only device
// workspaces, the round drivers (persistent VGC launch, or one launch per
// level), transpose, validation and the batched form. The served form lives
// in server.cpp. Every exported function is declared in include/pasgal.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "engine.h"
#include "kern.h"
#include "pasgal.h"

namespace pg {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PASGAL_ENOMEM : PASGAL_EHIP;
}

const DevInfo &dev_info() {
  static std::mutex mu;
  static std::map<int, DevInfo> cache;
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  DevInfo d{};
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
    d.cus = p.multiProcessorCount;
    d.lds_per_cu = p.maxSharedMemoryPerMultiProcessor ? p.maxSharedMemoryPerMultiProcessor : 65536;
    d.lds_per_block = p.sharedMemPerBlock;
    d.coop = p.cooperativeLaunch;
  }
  int wcr = 0;
  hipDeviceGetAttribute(&wcr, hipDeviceAttributeWallClockRate, dev);
  d.wall_khz = wcr > 0 ? wcr : 100000;
  d.device = dev;
  cache[dev] = d;
  return cache[dev];
}

int grow(DBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return PASGAL_OK;
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  size_t want = bytes + bytes / 8;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    hipGetLastError();
    b.p = nullptr;
    e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      hipGetLastError();
      b.p = nullptr;
      return hip_fail(e);
    }
    want = bytes;
  }
  b.bytes = want;
  return PASGAL_OK;
}

int grow_host(HBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return PASGAL_OK;
  if (b.p) hipHostFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  hipError_t e = hipHostMalloc(&b.p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    b.p = nullptr;
    return hip_fail(e);
  }
  b.bytes = bytes;
  return PASGAL_OK;
}

void free_buf(DBuf &b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}
void free_hbuf(HBuf &b) {
  if (b.p) hipHostFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

Workspace::~Workspace() {
  for (DBuf *b : {&ctl, &fv[0], &fv[1], &fq[0], &fq[1], &fval[0], &fval[1], &dirty, &qi, &qword, &seeds, &pf[0],
                  &pf[1], &stamp, &tmp_state, &tscratch, &plain_src, &aux, &imp})
    free_buf(*b);
  free_hbuf(h_ctl);
  free_hbuf(h_stage);
  free_hbuf(h_aux);
  free_hbuf(h_src);
  if (ext_free) ext_free(ext);
  if (ev0) hipEventDestroy(ev0);
  if (evk) hipEventDestroy(evk);
  if (ev1) hipEventDestroy(ev1);
}

static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

Workspace *workspace_for(hipStream_t s) {
  int dev = 0;
  hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto key = std::make_pair(dev, s);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) return it->second;
  Workspace *w = new (std::nothrow) Workspace();
  if (!w) return nullptr;
  w->stream = s;
  if (hipEventCreate(&w->ev0) != hipSuccess || hipEventCreate(&w->evk) != hipSuccess ||
      hipEventCreate(&w->ev1) != hipSuccess) {
    delete w;
    return nullptr;
  }
  g_ws[key] = w;
  return w;
}

int collect_async(Workspace &w) {
  if (!w.async_pending) return PASGAL_OK;
  hipError_t e = hipStreamSynchronize(w.stream);
  if (e != hipSuccess) return hip_fail(e);
  w.async_pending = false;
  return ((const Ctl *)w.h_ctl.p)->abort ? PASGAL_ETIMEOUT : PASGAL_OK;
}

// Every workspace, on every device (pasgal_shutdown).
static void destroy_workspaces() {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  int cur = 0;
  hipGetDevice(&cur);
  int last = -1;
  for (auto &kv : g_ws) {
    Workspace *w = kv.second;
    { std::lock_guard<std::mutex> wl(w->mu); }  // a call still inside it finishes first
    if (kv.first.first != last) {
      // kernels still running may use the buffers: wait for the device
      hipSetDevice(kv.first.first);
      hipDeviceSynchronize();
      last = kv.first.first;
    }
    delete w;
  }
  g_ws.clear();
  hipSetDevice(cur);
  (void)hipGetLastError();
}

Opts resolve_opts(const pasgal_opts *o) {
  Opts r;
  pasgal_opts d;
  pasgal_opts_default(&d);
  if (!o) o = &d;
  r.mode = o->mode;
  r.tau = o->tau > 0 ? (uint32_t)o->tau : 1024u;
  r.wg = o->wg_size > 0 ? o->wg_size : 1024;
  r.bpc = o->blocks_per_cu > 0 ? o->blocks_per_cu : 1;
  r.cap = o->frontier_capacity;
  r.flags = o->flags;
  r.timeout_ms = o->timeout_ms > 0 ? o->timeout_ms : 20000;
  r.stream = (hipStream_t)o->stream;
  r.window = o->window > 0 ? (uint32_t)o->window : (o->window == 0 ? 32u : 0u);
  r.min_chunk = o->min_chunk > 0 ? (uint32_t)std::min(o->min_chunk, 64) : 1u;
  r.prefetch = (o->flags & PASGAL_FLAG_PREFETCH) != 0 && !(o->flags & PASGAL_FLAG_NO_PREFETCH);
  r.test_first = (o->flags & PASGAL_FLAG_TEST_FIRST) != 0;  // entry points may turn it on by default
  r.heavy = o->heavy_arcs > 0 ? (uint32_t)o->heavy_arcs : (o->heavy_arcs == 0 ? 512u : 0u);
  r.cpw = o->chunks_per_wave > 0 ? (uint32_t)std::min(o->chunks_per_wave, 64) : 1u;
  r.share = o->device_share > 0 ? o->device_share : ((o->flags & PASGAL_FLAG_HALF_DEVICE) ? 50 : 0);
  if (o->filter_slots > 0) {
    uint32_t f = 1;
    while (f * 2 <= (uint32_t)std::min(o->filter_slots, 4096)) f *= 2;  // round down to a power of two
    r.filt = f;
  } else {
    r.filt = o->filter_slots == 0 ? 256u : 0u;
  }
  return r;
}

int SliceBufs::ensure(uint64_t entries, bool multi) {
  if (entries == 0) return PASGAL_OK;
  int rc;
  for (int i = 0; i < 2; i++) {
    if ((rc = grow(v[i], 4 * entries)) || (rc = grow(val[i], 8 * entries)) || (rc = grow(b[i], 4 * entries)))
      return rc;
    if (multi && (rc = grow(q[i], 4 * entries))) return rc;
  }
  cap = std::max<uint64_t>(cap, entries);
  return PASGAL_OK;
}

void SliceBufs::apply(VgcArgs &a, uint32_t heavy, uint32_t hcap, bool multi) const {
  a.heavy = hcap ? heavy : 0u;
  a.hcap = a.heavy ? hcap : 0u;
  for (int i = 0; i < 2; i++) {
    a.hv[i] = (uint32_t *)v[i].p;
    a.hq[i] = multi ? (uint32_t *)q[i].p : nullptr;
    a.hval[i] = (unsigned long long *)val[i].p;
    a.hb[i] = (int32_t *)b[i].p;
  }
}

SliceBufs::~SliceBufs() {
  for (int i = 0; i < 2; i++)
    for (DBuf *d : {&v[i], &q[i], &val[i], &b[i]}) free_buf(*d);
}

uint32_t slice_capacity(uint64_t m, uint32_t heavy, uint64_t frontier_cap) {
  if (heavy == 0) return 0;
  uint64_t c = 2 * m / heavy + 4096;
  c = std::min<uint64_t>(c, std::max<uint64_t>(frontier_cap, 64));
  return (uint32_t)std::min<uint64_t>(c, 0x7FFFFFFFull);
}

bool opts_valid(const pasgal_opts *o) {
  if (!o) return true;
  if (o->mode != PASGAL_MODE_VGC && o->mode != PASGAL_MODE_PLAIN) return false;
  if (o->wg_size > 0 && (o->wg_size % 64 != 0 || o->wg_size > 1024)) return false;
  if (o->blocks_per_cu > 32) return false;
  if (o->min_chunk > 64) return false;
  if (o->device_share < 0 || o->device_share > 99) return false;
  return true;
}

bool csr_valid(const pasgal_csr *g) {
  return g && g->n > 0 && g->m >= 0 && g->offsets && (g->m == 0 || g->targets);
}

// Persistent-launch geometry for a kernel and LDS budget.
bool coop_launch(const Opts &o) { return dev_info().coop != 0 && o.share == 0; }

int vgc_geometry(int kind, bool multi, const Opts &o, LaunchGeom &lg) {
  const DevInfo &di = dev_info();
  const int waves = o.wg / 64;
  // a launch on a share of every CU sizes its workgroups for that share of a
  // CU's LDS
  const size_t lds_cu = o.share ? di.lds_per_cu * (size_t)o.share / 100 : di.lds_per_cu;
  const size_t lds_cap_block = std::min<size_t>(lds_cu / (size_t)o.bpc, di.lds_per_block);
  // dynamic LDS leaves room for the kernel's static arrays (round header,
  // counts, query table or source-implication tables)
  const void *fn = vgc_kernel_ptr(kind, multi, o.prefetch, o.test_first);
  hipFuncAttributes fattr{};
  if (hipFuncGetAttributes(&fattr, fn) != hipSuccess) {
    (void)hipGetLastError();
    fattr.sharedSizeBytes = 4096;
  }
  const size_t kStatic = fattr.sharedSizeBytes + 256;
  // stage 128 entries; ring = largest power of two that fits
  const uint32_t S = 128;
  const bool pf = o.prefetch;
  auto largest_ring = [&](uint32_t F) {
    uint32_t Q = 4096;
    while (Q > 64 && vgc_lds_bytes(kind, multi, pf, waves, Q, S, F) + kStatic > lds_cap_block) Q >>= 1;
    return Q;
  };
  // The LDS filter (distance kinds) may take at most half of the ring it
  // would otherwise get; a smaller filter is tried before that.
  const uint32_t Q0 = largest_ring(0);
  uint32_t F = (kind == KIND_REACH) ? 0u : o.filt;
  while (F > 0 && (largest_ring(F) < Q0 / 2 || largest_ring(F) < 64 ||
                   vgc_lds_bytes(kind, multi, pf, waves, largest_ring(F), S, F) + kStatic > lds_cap_block))
    F >>= 1;
  if (F < 16) F = 0;
  const uint32_t Q = largest_ring(F);
  if (vgc_lds_bytes(kind, multi, pf, waves, Q, S, F) + kStatic > lds_cap_block) return PASGAL_EINVAL;
  lg.ring = Q;
  lg.stage = S;
  lg.filt = F;
  lg.block = o.wg;
  lg.pf = pf;
  lg.lds = vgc_lds_bytes(kind, multi, pf, waves, Q, S, F);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lg.lds);
  if (e != hipSuccess) {
    hipGetLastError();
  }
  int nb = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, lg.block, lg.lds);
  if (e != hipSuccess) return hip_fail(e);
  if (nb < 1) return PASGAL_EINVAL;
  if (o.share) {
    // a workgroup whose waves do not spread evenly over the CU's four SIMDs
    // can leave a SIMD without room for the other launch's waves: two 6-wave
    // workgroups per CU beside two 2-wave ones never all became resident
    if (waves % 4 != 0) return PASGAL_EINVAL;
    // its waves may take at most its share of the wave slots the kernel's
    // registers allow, so that the rest is left for the launch beside it
    int nw = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nw, fn, 64, 0);
    if (e != hipSuccess) return hip_fail(e);
    if ((int64_t)waves * o.bpc * 100 > (int64_t)o.share * nw + 50 || nb < o.bpc) return PASGAL_EINVAL;
  }
  const int bpc = std::min(nb, o.bpc);
  lg.grid = bpc * di.cus;
  return PASGAL_OK;
}

int ensure_frontier(Workspace &w, uint64_t cap, bool multi) {
  int rc;
  for (int i = 0; i < 2; i++) {
    if ((rc = grow(w.fv[i], 4 * cap))) return rc;
    if ((rc = grow(w.fval[i], 8 * cap))) return rc;
    if (multi && (rc = grow(w.fq[i], 4 * cap))) return rc;
  }
  w.cap = (uint32_t)cap;
  return PASGAL_OK;
}

uint64_t default_cap(int64_t requested, uint64_t nvert) {
  uint64_t cap = requested > 0 ? (uint64_t)requested : std::max<uint64_t>(2 * nvert, 65536);
  if (cap < 64) cap = 64;
  if (cap > 0x7FFFFFFFull) cap = 0x7FFFFFFFull;
  return cap;
}

void fill_stats_from_ctl(const Ctl &c, pasgal_stats *st, bool add) {
  if (!st) return;
  if (!add) memset(st, 0, sizeof(*st));
  st->rounds += c.rounds;
  st->expansions += (int64_t)c.stats[ST_EXPAND];
  st->arcs_scanned += (int64_t)c.stats[ST_ARCS];
  st->relax_success += (int64_t)c.stats[ST_SUCCESS];
  st->published += (int64_t)c.stats[ST_PUBLISH];
  st->overflow += (int64_t)c.stats[ST_OVERFLOW];
  st->stale += (int64_t)c.stats[ST_STALE];
  st->steps += (int64_t)c.stats[ST_STEPS];
  st->filtered += (int64_t)c.stats[ST_FILTERED];
  st->max_frontier = std::max<int64_t>(st->max_frontier, c.max_frontier);
}

// One query (or one mask word) on one CSR, persistent VGC launch. With
// implications (reach), seed i is source i of the mask word (bit i).
static int run_vgc_single(Workspace &w, int kind, const pasgal_csr *g, void *state, const uint32_t *sv,
                          const unsigned long long *sval, int nseed, const Opts &o, pasgal_stats *st,
                          bool add_stats, const uint32_t *wgt = nullptr, bool implications = false) {
  hipStream_t s = o.stream;
  const uint64_t n = (uint64_t)g->n;
  const uint64_t cap = default_cap(o.cap, n);
  int rc;
  LaunchGeom lg;
  if ((rc = vgc_geometry(kind, false, o, lg))) return rc;
  if ((rc = ensure_frontier(w, cap, false))) return rc;
  const uint64_t words = (n + 31) / 32;
  if ((rc = grow(w.dirty, 4 * words))) return rc;
  if ((rc = grow(w.ctl, sizeof(Ctl)))) return rc;
  if ((rc = grow(w.qi, sizeof(QInfo)))) return rc;
  if ((rc = grow(w.qword, 2 * sizeof(int64_t)))) return rc;
  if ((rc = grow(w.seeds, sizeof(SeedEnt) * (size_t)nseed))) return rc;
  if ((rc = grow_host(w.h_ctl, sizeof(Ctl)))) return rc;
  const uint32_t hcap = slice_capacity((uint64_t)g->m, o.heavy, cap);
  if ((rc = w.slices.ensure(hcap, false))) return rc;
  const size_t imp_bytes = implications ? 64 * 8 + 64 * 4 : 0;
  const size_t stage_bytes = sizeof(QInfo) + 2 * sizeof(int64_t) + sizeof(SeedEnt) * (size_t)nseed + imp_bytes;
  if ((rc = grow_host(w.h_stage, stage_bytes))) return rc;
  if (implications && (rc = grow(w.imp, imp_bytes))) return rc;
  // host staging (pinned) -> device tables
  uint8_t *hs = (uint8_t *)w.h_stage.p;
  QInfo *hq = (QInfo *)hs;
  int64_t *hw = (int64_t *)(hs + sizeof(QInfo));
  SeedEnt *he = (SeedEnt *)(hs + sizeof(QInfo) + 2 * sizeof(int64_t));
  // the previous call on this stream may still read the staging area
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e);
  hq->sbase = 0;
  hq->dbase = 0;
  hq->vbase = 0;
  hq->nv = g->n;
  hq->r0 = 0;
  hq->pad = 0;
  hw[0] = 0;
  hw[1] = (int64_t)words;
  for (int i = 0; i < nseed; i++) {
    he[i].v = sv[i];
    he[i].q = 0;
    he[i].val = sval[i];
  }
  if (implications) {
    // sources at the same vertex imply each other from the start
    unsigned long long *himp = (unsigned long long *)(he + nseed);
    int32_t *hsrc = (int32_t *)(himp + 64);
    for (int j = 0; j < 64; j++) {
      himp[j] = 0ull;
      hsrc[j] = j < nseed ? (int32_t)sv[j] : -1;
      for (int i = 0; i < nseed && j < nseed; i++)
        if (sv[i] == sv[j]) himp[j] |= sval[i];
    }
    if ((e = hipMemcpyAsync(w.imp.p, himp, imp_bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e);
  }
  if ((e = hipMemcpyAsync(w.qi.p, hq, sizeof(QInfo), hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e);
  if ((e = hipMemcpyAsync(w.qword.p, hw, 2 * sizeof(int64_t), hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e);
  if ((e = hipMemcpyAsync(w.seeds.p, he, sizeof(SeedEnt) * (size_t)nseed, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e);

  VgcArgs a{};
  a.off = g->offsets;
  a.tgt = g->targets;
  a.wgt = wgt;
  a.state = state;
  a.dirty = (uint32_t *)w.dirty.p;
  a.qi = (const QInfo *)w.qi.p;
  a.qword = (const int64_t *)w.qword.p;
  a.dirty_words = (int64_t)words;
  a.nq = 1;
  for (int i = 0; i < 2; i++) {
    a.fr.v[i] = (uint32_t *)w.fv[i].p;
    a.fr.q[i] = nullptr;
    a.fr.val[i] = (unsigned long long *)w.fval[i].p;
  }
  a.fr.cap = (uint32_t)cap;
  a.start_buf = 0;
  a.tau = o.tau;
  a.max_rounds = 0xFFFFFFFFu;
  a.ring_cap = lg.ring;
  a.stage_cap = lg.stage;
  a.min_chunk = o.min_chunk;
  a.chunks_per_wave = o.cpw;
  a.window = o.window;
  a.timeout_ticks = (long long)o.timeout_ms * (long long)dev_info().wall_khz;
  a.round_base = 0;
  a.test_first = o.test_first ? 1u : 0u;
  a.filt = lg.filt;  // single query: keys are vertex ids
  a.ctl = (Ctl *)w.ctl.p;
  a.imp = implications ? (unsigned long long *)w.imp.p : nullptr;
  a.srcv = implications ? (const int32_t *)((unsigned long long *)w.imp.p + 64) : nullptr;
  w.slices.apply(a, o.heavy, hcap, false);

  if ((e = hipEventRecord(w.ev0, s)) != hipSuccess) return hip_fail(e);
  if (kind != KIND_REACH)
    e = launch_fill_u32((uint32_t *)state, n, 0xFFFFFFFFu, s);
  else
    e = launch_fill_u64((unsigned long long *)state, n, 0ull, s);
  if (e != hipSuccess) return hip_fail(e);
  if ((e = launch_fill_u32((uint32_t *)w.dirty.p, words, 0u, s)) != hipSuccess) return hip_fail(e);
  if ((e = launch_fill_u32((uint32_t *)w.ctl.p, sizeof(Ctl) / 4, 0u, s)) != hipSuccess) return hip_fail(e);
  if ((e = launch_seed(kind, a, (const SeedEnt *)w.seeds.p, (uint32_t)nseed, 0, 0, s)) != hipSuccess)
    return hip_fail(e);
  if ((e = hipEventRecord(w.evk, s)) != hipSuccess) return hip_fail(e);
  if ((e = launch_vgc(kind, false, lg.pf, a, lg.grid, lg.block, lg.lds, coop_launch(o), s)) != hipSuccess)
    return hip_fail(e);
  if ((e = hipEventRecord(w.ev1, s)) != hipSuccess) return hip_fail(e);
  if ((e = hipMemcpyAsync(w.h_ctl.p, w.ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e);
  if (o.flags & PASGAL_FLAG_ASYNC) {
    w.async_pending = true;
    return PASGAL_OK;
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
  const Ctl &c = *(const Ctl *)w.h_ctl.p;
  if (c.abort) return PASGAL_ETIMEOUT;
  if (st) {
    fill_stats_from_ctl(c, st, add_stats);
    float ms = 0, kms = 0;
    hipEventElapsedTime(&ms, w.ev0, w.ev1);
    hipEventElapsedTime(&kms, w.evk, w.ev1);
    st->device_ms += ms;
    st->kernel_ms += kms;
  }
  return PASGAL_OK;
}

// Level-synchronous rounds, one launch per level; the host reads the next
// frontier size back after every level.
static int run_plain(Workspace &w, int kind, const pasgal_csr *g, void *state, const uint32_t *srcs,
                     const unsigned long long *vals, int nsrc, const Opts &o, pasgal_stats *st, bool add_stats) {
  hipStream_t s = o.stream;
  const uint64_t n = (uint64_t)g->n;
  int rc;
  if ((rc = grow(w.pf[0], 4 * n))) return rc;
  if ((rc = grow(w.pf[1], 4 * n))) return rc;
  if ((rc = grow(w.ctl, sizeof(Ctl)))) return rc;
  if ((rc = grow(w.plain_src, (4 + 8) * (size_t)nsrc))) return rc;
  if (kind == KIND_REACH && (rc = grow(w.stamp, 4 * n))) return rc;
  if ((rc = grow_host(w.h_ctl, sizeof(Ctl)))) return rc;
  if ((rc = grow_host(w.h_stage, (4 + 8) * (size_t)nsrc + 64))) return rc;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e);
  uint8_t *hs = (uint8_t *)w.h_stage.p;
  unsigned long long *hv = (unsigned long long *)hs;
  uint32_t *hsrc = (uint32_t *)(hs + 8 * (size_t)nsrc);
  for (int i = 0; i < nsrc; i++) {
    hsrc[i] = srcs[i];
    hv[i] = vals ? vals[i] : 0ull;
  }
  unsigned long long *dv = (unsigned long long *)w.plain_src.p;
  uint32_t *dsrc = (uint32_t *)((uint8_t *)w.plain_src.p + 8 * (size_t)nsrc);
  if ((e = hipMemcpyAsync(w.plain_src.p, hs, (4 + 8) * (size_t)nsrc, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e);
  Ctl *ctl = (Ctl *)w.ctl.p;
  if ((e = hipEventRecord(w.ev0, s)) != hipSuccess) return hip_fail(e);
  if (kind == KIND_BFS)
    e = launch_fill_u32((uint32_t *)state, n, 0xFFFFFFFFu, s);
  else
    e = launch_fill_u64((unsigned long long *)state, n, 0ull, s);
  if (e != hipSuccess) return hip_fail(e);
  if (kind == KIND_REACH && (e = launch_fill_u32((uint32_t *)w.stamp.p, n, 0xFFFFFFFFu, s)) != hipSuccess)
    return hip_fail(e);
  if ((e = launch_fill_u32((uint32_t *)w.ctl.p, sizeof(Ctl) / 4, 0u, s)) != hipSuccess) return hip_fail(e);
  if ((e = launch_plain_seed(kind, state, (uint32_t *)w.pf[0].p, ctl->cnt, (uint32_t *)w.stamp.p, dsrc, dv,
                             (uint32_t)nsrc, s)) != hipSuccess)
    return hip_fail(e);
  uint32_t *hcnt = (uint32_t *)w.h_ctl.p;
  if ((e = hipMemcpyAsync(hcnt, &ctl->cnt[0], 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
  uint32_t ncur = *hcnt;
  uint32_t level = 0;
  if ((e = hipEventRecord(w.evk, s)) != hipSuccess) return hip_fail(e);
  int cur = 0;
  int64_t expansions = 0, maxf = 0;
  while (ncur > 0) {
    expansions += ncur;
    maxf = std::max<int64_t>(maxf, ncur);
    if (kind == KIND_BFS)
      e = launch_plain_bfs_level(g->offsets, g->targets, (uint32_t *)state, (const uint32_t *)w.pf[cur].p, ncur,
                                 (uint32_t *)w.pf[cur ^ 1].p, ctl->cnt, level, ctl, s);
    else
      e = launch_plain_reach_level(g->offsets, g->targets, (unsigned long long *)state, (uint32_t *)w.stamp.p,
                                   (const uint32_t *)w.pf[cur].p, ncur, (uint32_t *)w.pf[cur ^ 1].p, ctl->cnt,
                                   level, ctl, s);
    if (e != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpyAsync(hcnt, &ctl->cnt[(level + 1) % 3], 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
      return hip_fail(e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
    ncur = *hcnt;
    cur ^= 1;
    level++;
    if (ncur > n) return PASGAL_ECAPACITY;  // cannot happen: each vertex enters once per level
  }
  if ((e = hipEventRecord(w.ev1, s)) != hipSuccess) return hip_fail(e);
  if ((e = hipMemcpyAsync(w.h_ctl.p, w.ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
  if (st) {
    const Ctl &c = *(const Ctl *)w.h_ctl.p;
    if (!add_stats) memset(st, 0, sizeof(*st));
    st->rounds += level;
    st->expansions += expansions;
    st->arcs_scanned += (int64_t)c.stats[ST_ARCS];
    st->relax_success += (int64_t)c.stats[ST_SUCCESS];
    st->published += (int64_t)c.stats[ST_SUCCESS];
    st->max_frontier = std::max<int64_t>(st->max_frontier, maxf);
    float ms = 0, kms = 0;
    hipEventElapsedTime(&ms, w.ev0, w.ev1);
    hipEventElapsedTime(&kms, w.evk, w.ev1);
    st->device_ms += ms;
    st->kernel_ms += kms;
  }
  return PASGAL_OK;
}

int validate_csr_device(Workspace &w, const pasgal_csr *g, hipStream_t s) {
  int rc;
  if ((rc = grow(w.ctl, sizeof(Ctl)))) return rc;
  if ((rc = grow_host(w.h_ctl, sizeof(Ctl)))) return rc;
  hipError_t e;
  if ((e = launch_fill_u32((uint32_t *)w.ctl.p, sizeof(Ctl) / 4, 0u, s)) != hipSuccess) return hip_fail(e);
  if ((e = launch_validate(g->offsets, g->targets, g->n, g->m, (Ctl *)w.ctl.p, s)) != hipSuccess) return hip_fail(e);
  if ((e = hipMemcpyAsync(w.h_ctl.p, w.ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
  return ((const Ctl *)w.h_ctl.p)->bad_csr ? PASGAL_ECSR : PASGAL_OK;
}

}  // namespace pg

using namespace pg;

extern "C" {

void pasgal_opts_default(pasgal_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->mode = PASGAL_MODE_VGC;
  o->tau = 0;  // each entry point's default (1024; pasgal_sssp: by mean degree)
  o->wg_size = 1024;
  o->blocks_per_cu = 1;
  o->frontier_capacity = 0;
  o->flags = 0;
  o->timeout_ms = 20000;
  o->stream = nullptr;
  o->window = 0;
  o->min_chunk = 1;
  o->heavy_arcs = 512;
  o->filter_slots = 256;
}

const char *pasgal_strerror(int code) {
  switch (code) {
    case PASGAL_OK: return "ok";
    case PASGAL_EINVAL: return "invalid argument";
    case PASGAL_ENOMEM: return "out of memory";
    case PASGAL_EHIP: return "HIP runtime error";
    case PASGAL_ECSR: return "malformed CSR graph";
    case PASGAL_ECAPACITY: return "capacity exceeded";
    case PASGAL_EAGAIN: return "resource busy, try again";
    case PASGAL_ETIMEOUT: return "device-side wait timed out";
    case PASGAL_ENOTFOUND: return "not found";
    case PASGAL_EINTERNAL: return "internal consistency check failed";
    default: return "unknown error";
  }
}

int pasgal_last_hip_error(void) { return g_last_hip; }
int pasgal_version(void) { return PASGAL_VERSION; }

void pasgal_shutdown(void) { destroy_workspaces(); }

int pasgal_wait(void *stream) {
  hipStream_t s = (hipStream_t)stream;
  Workspace *w = workspace_for(s);
  if (!w) return PASGAL_ENOMEM;
  std::lock_guard<std::mutex> lk(w->mu);
  if (int rc = collect_async(*w)) return rc;
  hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? PASGAL_OK : hip_fail(e);
}

int pasgal_bfs_ex(const pasgal_csr *g, int32_t src, int32_t *dist_out, const pasgal_opts *opts, pasgal_stats *stats) {
  if (!csr_valid(g) || !dist_out || src < 0 || src >= g->n || !opts_valid(opts)) return PASGAL_EINVAL;
  Opts o = resolve_opts(opts);
  if (o.mode == PASGAL_MODE_PLAIN && (o.flags & PASGAL_FLAG_ASYNC)) return PASGAL_EINVAL;
  // arc ranges carried in the local queue: about 5% faster single-source BFS
  // (only with local searches beyond the roots: at tau 1 no carried range is used)
  if (!(o.flags & PASGAL_FLAG_NO_PREFETCH) && o.tau > 1) o.prefetch = true;
  Workspace *w = workspace_for(o.stream);
  if (!w) return PASGAL_ENOMEM;
  std::lock_guard<std::mutex> lk(w->mu);
  if (int arc = collect_async(*w)) return arc;
  int rc;
  if (o.flags & PASGAL_FLAG_VALIDATE) {
    if ((rc = validate_csr_device(*w, g, o.stream))) return rc;
  }
  const uint32_t sv = (uint32_t)src;
  const unsigned long long val = 0ull;
  if (o.mode == PASGAL_MODE_PLAIN)
    return run_plain(*w, KIND_BFS, g, dist_out, &sv, &val, 1, o, stats, false);
  return run_vgc_single(*w, KIND_BFS, g, dist_out, &sv, &val, 1, o, stats, false);
}

int pasgal_sssp(const pasgal_csr *g, const uint32_t *weights, int32_t src, uint32_t *dist_out,
                const pasgal_opts *opts, pasgal_stats *stats) {
  if (!csr_valid(g) || !dist_out || (g->m > 0 && !weights) || src < 0 || src >= g->n || !opts_valid(opts))
    return PASGAL_EINVAL;
  Opts o = resolve_opts(opts);
  // default tau by mean out-degree: no local search beyond the roots on dense graphs
  if (!opts || opts->tau <= 0) o.tau = (int64_t)g->m > 8 * (int64_t)g->n ? 1u : 1024u;
  if (o.mode == PASGAL_MODE_PLAIN) o.tau = 1;
  // arc ranges carried in the local queue, as for BFS (road4096 26.3 -> 24.9 ms);
  // at tau 1 no carried range is used (RMAT-22 21.7 -> 22.6 ms with them)
  if (!(o.flags & PASGAL_FLAG_NO_PREFETCH) && o.tau > 1) o.prefetch = true;
  Workspace *w = workspace_for(o.stream);
  if (!w) return PASGAL_ENOMEM;
  std::lock_guard<std::mutex> lk(w->mu);
  if (int arc = collect_async(*w)) return arc;
  int rc;
  hipError_t e;
  if (o.flags & PASGAL_FLAG_VALIDATE) {
    if ((rc = validate_csr_device(*w, g, o.stream))) return rc;
  }
  if (!opts || opts->window == 0) {
    // default bucket width: 8 mean arc weights. Local searches run in FIFO,
    // not distance, order, so a wider bucket costs re-expansions
    if ((rc = grow(w->aux, 64)) || (rc = grow_host(w->h_aux, 64))) return rc;
    if ((e = launch_fill_u32((uint32_t *)w->aux.p, 2, 0u, o.stream)) != hipSuccess) return hip_fail(e);
    if ((e = launch_sum_u32(weights, (uint64_t)g->m, (unsigned long long *)w->aux.p, o.stream)) != hipSuccess)
      return hip_fail(e);
    if ((e = hipMemcpyAsync(w->h_aux.p, w->aux.p, 8, hipMemcpyDeviceToHost, o.stream)) != hipSuccess)
      return hip_fail(e);
    if ((e = hipStreamSynchronize(o.stream)) != hipSuccess) return hip_fail(e);
    const unsigned long long sum = *(const unsigned long long *)w->h_aux.p;
    const double mean = g->m > 0 ? (double)sum / (double)g->m : 1.0;
    o.window = (uint32_t)std::min(std::max(8.0 * mean, 1.0), 2147483647.0);
  }
  const uint32_t sv = (uint32_t)src;
  const unsigned long long val = 0ull;
  return run_vgc_single(*w, KIND_SSSP, g, dist_out, &sv, &val, 1, o, stats, false, weights);
}

int pasgal_bfs(const pasgal_csr *g, int32_t src, int32_t *dist_out) {
  return pasgal_bfs_ex(g, src, dist_out, nullptr, nullptr);
}

int pasgal_reach_ex(const pasgal_csr *g, const int32_t *sources, int32_t k, uint64_t *label_out,
                    const pasgal_opts *opts, pasgal_stats *stats) {
  if (!csr_valid(g) || !label_out || !sources || k <= 0 || !opts_valid(opts)) return PASGAL_EINVAL;
  Opts o = resolve_opts(opts);
  if (o.mode == PASGAL_MODE_PLAIN && (o.flags & PASGAL_FLAG_ASYNC)) return PASGAL_EINVAL;
  // several sources on a graph of mean out-degree >= 4: a vertex gets most
  // of its bits before its last in-neighbours offer them again, so a plain
  // read first skips most atomics (on sparser graphs the read only lengthens
  // each level's chain of dependent accesses)
  if (k >= 2 && (int64_t)g->m >= 4 * (int64_t)g->n && !(o.flags & PASGAL_FLAG_NO_TEST_FIRST)) o.test_first = true;
  // arc ranges carried in the local queue: 4-8% faster reach, on by default
  // with local searches beyond the roots
  if (!(o.flags & PASGAL_FLAG_NO_PREFETCH) && o.tau > 1) o.prefetch = true;
  const int W = (k + 63) / 64;
  if (W > 1 && (o.flags & PASGAL_FLAG_ASYNC)) return PASGAL_EINVAL;
  Workspace *w = workspace_for(o.stream);
  if (!w) return PASGAL_ENOMEM;
  std::lock_guard<std::mutex> lk(w->mu);
  if (int arc = collect_async(*w)) return arc;
  int rc;
  // the sources are a device array: read them (after the stream's earlier
  // work, which may produce them) and check them before anything is written
  if ((rc = grow_host(w->h_src, 4 * (size_t)k))) return rc;
  hipError_t es = hipMemcpyAsync(w->h_src.p, sources, 4 * (size_t)k, hipMemcpyDeviceToHost, o.stream);
  if (es == hipSuccess) es = hipStreamSynchronize(o.stream);
  if (es != hipSuccess) return hip_fail(es);
  sources = (const int32_t *)w->h_src.p;
  for (int32_t i = 0; i < k; i++)
    if (sources[i] < 0 || sources[i] >= g->n) return PASGAL_EINVAL;
  if (o.flags & PASGAL_FLAG_VALIDATE) {
    if ((rc = validate_csr_device(*w, g, o.stream))) return rc;
  }
  if (stats) memset(stats, 0, sizeof(*stats));
  for (int word = 0; word < W; word++) {
    const int k0 = word * 64, kk = std::min(64, k - k0);
    std::vector<uint32_t> sv(kk);
    std::vector<unsigned long long> vals(kk);
    for (int i = 0; i < kk; i++) {
      sv[i] = (uint32_t)sources[k0 + i];
      vals[i] = 1ull << i;
    }
    void *state = label_out;
    if (W > 1) {
      if ((rc = grow(w->tmp_state, 8 * (size_t)g->n))) return rc;
      state = w->tmp_state.p;
    }
    if (o.mode == PASGAL_MODE_PLAIN)
      rc = run_plain(*w, KIND_REACH, g, state, sv.data(), vals.data(), kk, o, stats, true);
    else
      rc = run_vgc_single(*w, KIND_REACH, g, state, sv.data(), vals.data(), kk, o, stats, true, nullptr,
                          kk >= 2 && !(o.flags & PASGAL_FLAG_NO_IMPLICATIONS));
    if (rc) return rc;
    if (W > 1) {
      hipError_t e = launch_strided_u64((unsigned long long *)label_out, W, word,
                                        (const unsigned long long *)w->tmp_state.p, (uint64_t)g->n, o.stream);
      if (e != hipSuccess) return hip_fail(e);
      if ((e = hipStreamSynchronize(o.stream)) != hipSuccess) return hip_fail(e);
    }
  }
  return PASGAL_OK;
}

int pasgal_reach(const pasgal_csr *g, const int32_t *sources, int32_t k, uint64_t *label_out) {
  return pasgal_reach_ex(g, sources, k, label_out, nullptr, nullptr);
}

int pasgal_transpose(const pasgal_csr *g, int32_t *t_offsets, int32_t *t_targets, const pasgal_opts *opts) {
  if (!csr_valid(g) || !t_offsets || (g->m > 0 && !t_targets)) return PASGAL_EINVAL;
  Opts o = resolve_opts(opts);
  Workspace *w = workspace_for(o.stream);
  if (!w) return PASGAL_ENOMEM;
  std::lock_guard<std::mutex> lk(w->mu);
  if (int arc = collect_async(*w)) return arc;
  int rc;
  if (o.flags & PASGAL_FLAG_VALIDATE) {
    if ((rc = validate_csr_device(*w, g, o.stream))) return rc;
  }
  if ((rc = grow(w->tscratch, 4 * transpose_scratch_elems(g->n)))) return rc;
  hipError_t e = launch_transpose(g->offsets, g->targets, g->n, g->m, t_offsets, t_targets,
                                  (int32_t *)w->tscratch.p, o.stream);
  if (e != hipSuccess) return hip_fail(e);
  if ((e = hipStreamSynchronize(o.stream)) != hipSuccess) return hip_fail(e);
  return PASGAL_OK;
}

int pasgal_validate(const pasgal_csr *g, const pasgal_opts *opts) {
  if (!csr_valid(g)) return PASGAL_EINVAL;
  Opts o = resolve_opts(opts);
  Workspace *w = workspace_for(o.stream);
  if (!w) return PASGAL_ENOMEM;
  std::lock_guard<std::mutex> lk(w->mu);
  if (int arc = collect_async(*w)) return arc;
  return validate_csr_device(*w, g, o.stream);
}

}  // extern "C"
