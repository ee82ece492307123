// batch.hip -- batched form: many BFS queries over a packed CSR of many
// graphs, advanced together by one persistent VGC launch. The launch sequence
// (segmented fill of the outputs, dirty/control reset, seeding, persistent
// kernel, control read-back) is captured once in a hipGraph and replayed.
// An optional autotuner times the persistent launch over a small grid of
// (tau, workgroup size, workgroups per CU) and keeps the fastest; results are
// exact for every choice, so only time decides.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"
#include "kern.h"
#include "pasgal.h"

using namespace pg;

struct pasgal_batch {
  std::mutex mu;
  hipStream_t caller = nullptr;  // stream the caller orders the batch after
  hipStream_t stream = nullptr;  // private capturable stream (the null stream cannot be captured)
  hipEvent_t evc = nullptr;
  pasgal_csr packed{};
  int32_t nq = 0;
  int32_t *dist = nullptr;
  Opts o;
  LaunchGeom lg;
  uint64_t cap = 0;
  int64_t words = 0;
  DBuf fv[2], fq[2], fval[2], dirty, ctl, qi, qword, seeds, seg_off, seg_len;
  HBuf h_ctl;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evk0 = nullptr, evk1 = nullptr;
  VgcArgs args{};
  bool coop_in_graph = false;
  SliceBufs slices;
  uint32_t hcap = 0;
  int64_t dist_len = 0;  // values in the state array

  ~pasgal_batch() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    for (DBuf *b : {&fv[0], &fv[1], &fq[0], &fq[1], &fval[0], &fval[1], &dirty, &ctl, &qi, &qword, &seeds, &seg_off,
                    &seg_len})
      free_buf(*b);
    free_hbuf(h_ctl);
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    if (evc) hipEventDestroy(evc);
    if (evk0) hipEventDestroy(evk0);
    if (evk1) hipEventDestroy(evk1);
    if (stream) hipStreamDestroy(stream);
  }

  // order the private stream after everything already queued on the caller's stream
  hipError_t follow_caller() {
    hipError_t e = hipEventRecord(evc, caller);
    if (e != hipSuccess) return e;
    return hipStreamWaitEvent(stream, evc, 0);
  }

  // Enqueue the whole batch on the stream (also used under capture).
  hipError_t enqueue(bool cooperative) {
    hipStream_t s = stream;
    hipError_t e;
    if ((e = launch_fill_segments_u32((uint32_t *)dist, (const int64_t *)seg_off.p, (const int64_t *)seg_len.p, nq,
                                      0xFFFFFFFFu, s)) != hipSuccess)
      return e;
    if ((e = launch_fill_u32((uint32_t *)dirty.p, (uint64_t)words, 0u, s)) != hipSuccess) return e;
    if ((e = launch_fill_u32((uint32_t *)ctl.p, sizeof(Ctl) / 4, 0u, s)) != hipSuccess) return e;
    if ((e = launch_seed(KIND_BFS, args, (const SeedEnt *)seeds.p, (uint32_t)nq, 0, 0, s)) != hipSuccess) return e;
    if ((e = hipEventRecord(evk0, s)) != hipSuccess) return e;
    if ((e = launch_vgc(KIND_BFS, true, lg.pf, args, lg.grid, lg.block, lg.lds, cooperative, s)) != hipSuccess)
      return e;
    if ((e = hipEventRecord(evk1, s)) != hipSuccess) return e;
    return hipMemcpyAsync(h_ctl.p, ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s);
  }

  int configure(const Opts &oo) {
    int rc = vgc_geometry(KIND_BFS, true, oo, lg);
    if (rc) return rc;
    o = oo;
    args.tau = o.tau;
    args.ring_cap = lg.ring;
    args.stage_cap = lg.stage;
    args.min_chunk = o.min_chunk;
    args.chunks_per_wave = o.cpw;
    args.window = o.window;
    args.test_first = o.test_first ? 1u : 0u;
    // filter keys are 32-bit state indices: exact only below 2^32 values
    args.filt = dist_len < (int64_t(1) << 32) ? lg.filt : 0u;
    args.timeout_ticks = (long long)o.timeout_ms * (long long)dev_info().wall_khz;
    slices.apply(args, o.heavy, hcap, true);
    return PASGAL_OK;
  }

  // Reallocate the frontier buffers (and the slice buffers sized from them)
  // at a smaller capacity; the launch arguments follow.
  int shrink_frontier(uint64_t c) {
    int rc = PASGAL_OK;
    for (int i = 0; i < 2 && !rc; i++) {
      for (DBuf *d : {&fv[i], &fq[i], &fval[i]}) free_buf(*d);
      rc = grow(fv[i], 4 * c);
      if (!rc) rc = grow(fq[i], 4 * c);
      if (!rc) rc = grow(fval[i], 8 * c);
    }
    if (rc) return rc;
    cap = c;
    for (int i = 0; i < 2; i++) {
      args.fr.v[i] = (uint32_t *)fv[i].p;
      args.fr.q[i] = (uint32_t *)fq[i].p;
      args.fr.val[i] = (unsigned long long *)fval[i].p;
    }
    args.fr.cap = (uint32_t)c;
    hcap = std::min<uint32_t>(hcap, (uint32_t)std::max<uint64_t>(c, 64));
    return PASGAL_OK;
  }

  // Direct (uncaptured) run; returns the device time in ms through *ms.
  int run_direct(float *ms) {
    hipError_t e;
    if ((e = follow_caller()) != hipSuccess) return hip_fail(e);
    if ((e = hipEventRecord(ev0, stream)) != hipSuccess) return hip_fail(e);
    if ((e = enqueue(coop_launch(o))) != hipSuccess) return hip_fail(e);
    if ((e = hipEventRecord(ev1, stream)) != hipSuccess) return hip_fail(e);
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e);
    if (((const Ctl *)h_ctl.p)->abort) return PASGAL_ETIMEOUT;
    if (ms) hipEventElapsedTime(ms, ev0, ev1);
    return PASGAL_OK;
  }

  int capture() {
    if (exec) {
      hipGraphExecDestroy(exec);
      exec = nullptr;
    }
    if (graph) {
      hipGraphDestroy(graph);
      graph = nullptr;
    }
    // A cooperative launch node is tried first; where capture does not take
    // one, the persistent kernel is captured as an ordinary launch of the same
    // occupancy-sized grid (the device-side barrier deadline still bounds it).
    hipError_t last = hipSuccess;
    for (int attempt = 0; attempt < 2; attempt++) {
      const bool coop = (attempt == 0) && coop_launch(o);
      hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e);
      hipError_t ee = enqueue(coop);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(stream, &g);
      if (ee != hipSuccess || e != hipSuccess) {
        last = ee != hipSuccess ? ee : e;
        (void)hipGetLastError();
        if (g) hipGraphDestroy(g);
        continue;
      }
      e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        last = e;
        (void)hipGetLastError();
        hipGraphDestroy(g);
        exec = nullptr;
        continue;
      }
      graph = g;
      coop_in_graph = coop;
      return PASGAL_OK;
    }
    return hip_fail(last);
  }
};

extern "C" {

int pasgal_batch_create(const pasgal_batch_desc *d, const pasgal_opts *opts, uint32_t batch_flags,
                        pasgal_batch **out) {
  if (!out || !d || !csr_valid(&d->packed) || d->ngraphs <= 0 || !d->vbase || d->nqueries <= 0 || !d->q_graph ||
      !d->q_source || !d->q_out || !d->dist_out || d->dist_len <= 0 || !opts_valid(opts))
    return PASGAL_EINVAL;
  *out = nullptr;
  if (d->vbase[0] != 0 || d->vbase[d->ngraphs] != d->packed.n) return PASGAL_EINVAL;
  for (int32_t g = 0; g < d->ngraphs; g++)
    if (d->vbase[g + 1] <= d->vbase[g]) return PASGAL_EINVAL;
  const int32_t nq = d->nqueries;
  std::vector<QInfo> qi(nq);
  std::vector<int64_t> qword(nq + 1), segoff(nq), seglen(nq);
  std::vector<SeedEnt> seeds(nq);
  int64_t words = 0, total_state = 0;
  for (int32_t q = 0; q < nq; q++) {
    const int32_t g = d->q_graph[q];
    if (g < 0 || g >= d->ngraphs) return PASGAL_EINVAL;
    const int32_t nv = d->vbase[g + 1] - d->vbase[g];
    const int32_t src = d->q_source[q];
    if (src < 0 || src >= nv) return PASGAL_EINVAL;
    const int64_t o = d->q_out[q];
    if (o < 0 || o + nv > d->dist_len) return PASGAL_EINVAL;
    qi[q].sbase = o - d->vbase[g];
    qi[q].dbase = words;
    qi[q].vbase = d->vbase[g];
    qi[q].nv = nv;
    qi[q].r0 = 0;
    qi[q].pad = 0;
    qword[q] = words;
    words += (nv + 31) / 32;
    segoff[q] = o;
    seglen[q] = nv;
    total_state += nv;
    seeds[q].v = (uint32_t)(d->vbase[g] + src);
    seeds[q].q = (uint32_t)q;
    seeds[q].val = 0;
  }
  qword[nq] = words;
  {  // output regions must not overlap
    std::vector<std::pair<int64_t, int64_t>> r(nq);
    for (int32_t q = 0; q < nq; q++) r[q] = {segoff[q], seglen[q]};
    std::sort(r.begin(), r.end());
    for (int32_t q = 1; q < nq; q++)
      if (r[q - 1].first + r[q - 1].second > r[q].first) return PASGAL_EINVAL;
  }
  pasgal_batch *b = new (std::nothrow) pasgal_batch();
  if (!b) return PASGAL_ENOMEM;
  Opts o = resolve_opts(opts);
  b->caller = o.stream;
  b->packed = d->packed;
  b->nq = nq;
  b->dist = d->dist_out;
  b->dist_len = d->dist_len;
  b->words = words;
  int rc = PASGAL_OK;
  hipError_t e;
  if ((e = hipEventCreate(&b->ev0)) != hipSuccess || (e = hipEventCreate(&b->ev1)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->evc, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreate(&b->evk0)) != hipSuccess || (e = hipEventCreate(&b->evk1)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) {
    delete b;
    return hip_fail(e);
  }
  b->cap = o.cap > 0 ? default_cap(o.cap, 0)
                     : std::min<uint64_t>(std::max<uint64_t>((uint64_t)total_state / 4, 1u << 20), 0x7FFFFFFFull);
  for (int i = 0; i < 2 && !rc; i++) {
    rc = grow(b->fv[i], 4 * b->cap);
    if (!rc) rc = grow(b->fq[i], 4 * b->cap);
    if (!rc) rc = grow(b->fval[i], 8 * b->cap);
  }
  if (!rc) rc = grow(b->dirty, 4 * (size_t)words);
  if (!rc) rc = grow(b->ctl, sizeof(Ctl));
  if (!rc) rc = grow(b->qi, sizeof(QInfo) * nq);
  if (!rc) rc = grow(b->qword, sizeof(int64_t) * (nq + 1));
  if (!rc) rc = grow(b->seeds, sizeof(SeedEnt) * nq);
  if (!rc) rc = grow(b->seg_off, sizeof(int64_t) * nq);
  if (!rc) rc = grow(b->seg_len, sizeof(int64_t) * nq);
  if (!rc) rc = grow_host(b->h_ctl, sizeof(Ctl));
  // a hub may be cut once per query that expands it
  b->hcap = slice_capacity((uint64_t)d->packed.m * (uint64_t)std::min(nq, 8), o.heavy, b->cap);
  if (!rc) rc = b->slices.ensure(b->hcap, true);
  if (rc) {
    delete b;
    return rc;
  }
  hipStream_t s = b->stream;
  if ((e = b->follow_caller()) != hipSuccess) {
    delete b;
    return hip_fail(e);
  }
  if ((e = hipMemcpyAsync(b->qi.p, qi.data(), sizeof(QInfo) * nq, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(b->qword.p, qword.data(), sizeof(int64_t) * (nq + 1), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(b->seeds.p, seeds.data(), sizeof(SeedEnt) * nq, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(b->seg_off.p, segoff.data(), sizeof(int64_t) * nq, hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(b->seg_len.p, seglen.data(), sizeof(int64_t) * nq, hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    delete b;
    return hip_fail(e);
  }
  VgcArgs &a = b->args;
  a.off = d->packed.offsets;
  a.tgt = d->packed.targets;
  a.state = d->dist_out;
  a.dirty = (uint32_t *)b->dirty.p;
  a.qi = (const QInfo *)b->qi.p;
  a.qword = (const int64_t *)b->qword.p;
  a.dirty_words = words;
  a.nq = nq;
  for (int i = 0; i < 2; i++) {
    a.fr.v[i] = (uint32_t *)b->fv[i].p;
    a.fr.q[i] = (uint32_t *)b->fq[i].p;
    a.fr.val[i] = (unsigned long long *)b->fval[i].p;
  }
  a.fr.cap = (uint32_t)b->cap;
  a.start_buf = 0;
  a.max_rounds = 0xFFFFFFFFu;
  a.round_base = 0;
  a.ctl = (Ctl *)b->ctl.p;

  if (batch_flags & PASGAL_BATCH_AUTOTUNE) {
    const int taus[] = {16, 64, 256, 1024, 4096};
    const int wgs[] = {256, 512, 1024};
    const int bpcs[] = {1, 2, 4};
    float best = 1e30f;
    Opts best_o = o;
    bool any = false;
    for (int t : taus)
      for (int wg : wgs)
        for (int bpc : bpcs) {
          if (wg * bpc > 2048) continue;
          Opts c = o;
          c.tau = (uint32_t)t;
          c.wg = wg;
          c.bpc = bpc;
          if (b->configure(c) != PASGAL_OK) continue;
          if (b->lg.grid != bpc * dev_info().cus) continue;  // not all blocks resident
          float ms = 0;
          rc = b->run_direct(&ms);
          if (rc == PASGAL_OK) rc = b->run_direct(&ms);
          if (rc != PASGAL_OK) {
            if (rc == PASGAL_ETIMEOUT) continue;
            delete b;
            return rc;
          }
          if (ms < best) {
            best = ms;
            best_o = c;
            any = true;
          }
        }
    if (!any) {
      delete b;
      return PASGAL_ETIMEOUT;
    }
    o = best_o;
    // Frontier capacity: the smallest of cap, cap/4, cap/16 (at least 64 Ki
    // entries) whose time stays within 5% of the best. A smaller frontier
    // sends overflow through the dirty bitmaps, exact but usually slower, so
    // this only trades footprint for time where it costs nothing.
    if ((rc = b->configure(o))) {
      delete b;
      return rc;
    }
    const uint64_t full = b->cap;
    uint64_t chosen = full;
    for (uint64_t c = full / 4; c >= (1u << 16) && c >= full / 16; c /= 4) {
      b->args.fr.cap = (uint32_t)c;
      float ms = 0;
      rc = b->run_direct(&ms);
      if (rc == PASGAL_OK) rc = b->run_direct(&ms);
      if (rc == PASGAL_ETIMEOUT) break;
      if (rc != PASGAL_OK) {
        delete b;
        return rc;
      }
      if (ms <= 1.05f * best) chosen = c;
    }
    b->args.fr.cap = (uint32_t)full;
    if (chosen < full && (rc = b->shrink_frontier(chosen))) {
      delete b;
      return rc;
    }
  }
  if ((rc = b->configure(o))) {
    delete b;
    return rc;
  }
  if ((rc = b->capture())) {
    delete b;
    return rc;
  }
  *out = b;
  return PASGAL_OK;
}

int pasgal_batch_run(pasgal_batch *b, pasgal_stats *st) {
  if (!b) return PASGAL_EINVAL;
  std::lock_guard<std::mutex> lk(b->mu);
  hipError_t e;
  if ((e = b->follow_caller()) != hipSuccess) return hip_fail(e);
  if ((e = hipEventRecord(b->ev0, b->stream)) != hipSuccess) return hip_fail(e);
  if ((e = hipGraphLaunch(b->exec, b->stream)) != hipSuccess) return hip_fail(e);
  if ((e = hipEventRecord(b->ev1, b->stream)) != hipSuccess) return hip_fail(e);
  if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return hip_fail(e);
  const Ctl &c = *(const Ctl *)b->h_ctl.p;
  if (c.abort) return PASGAL_ETIMEOUT;
  if (st) {
    fill_stats_from_ctl(c, st, false);
    float ms = 0, kms = 0;
    hipEventElapsedTime(&ms, b->ev0, b->ev1);
    if (hipEventElapsedTime(&kms, b->evk0, b->evk1) != hipSuccess) {
      (void)hipGetLastError();  // event nodes inside the graph are not timeable here: use the graph time
      kms = ms;
    }
    st->device_ms = ms;
    st->kernel_ms = kms;
  }
  return PASGAL_OK;
}

int pasgal_batch_config(const pasgal_batch *b, pasgal_opts *chosen) {
  if (!b || !chosen) return PASGAL_EINVAL;
  pasgal_opts_default(chosen);
  chosen->tau = (int32_t)b->o.tau;
  chosen->wg_size = b->o.wg;
  chosen->blocks_per_cu = b->o.bpc;
  chosen->frontier_capacity = (int64_t)b->cap;
  chosen->timeout_ms = b->o.timeout_ms;
  chosen->stream = b->caller;
  chosen->flags = 0u;
  return PASGAL_OK;
}

void pasgal_batch_destroy(pasgal_batch *b) { delete b; }

}  // extern "C"
