// server.hip -- served form: a request loop over graphs resident in device
// memory, with continuous batching.
//
//  * Graphs are copied into one server-owned packed CSR (global vertex ids),
//    so a single persistent launch can advance requests on any of them.
//  * Each request's state (dist or mask array, plus its dirty bitmap) is
//    carved from an arena of memory_budget bytes; a request is admitted when
//    a slot is free and its state fits (first-fit allocator on the host).
//  * The scheduler thread runs slices: one persistent VGC launch per kind
//    (BFS, reach), each on its own stream, of at most slice_rounds rounds
//    over every admitted request of that kind. When both kinds have work,
//    the two launches run at the same time, each sized to half of every
//    compute unit; a kind running alone takes the whole device. The frontier
//    survives between slices, newly admitted requests are seeded into it at
//    the slice boundary (a launch made while a single request is resident and
//    none is queued runs the single-query kernel until the request finishes,
//    or until a submission changes a word in coherent host memory that the
//    launch polls once per round), and
//    a census kernel that follows each launch on its
//    stream (reading the launch's exit record on the device) flags the
//    requests that still have work. One copy back and one wait per slice and
//    kind: finished requests get their result copy enqueued and are
//    completed, and their memory returned, once the stream has passed the
//    copy. Requests therefore join and leave while others are still being
//    traversed on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "arena.h"
#include "devgate.h"
#include "engine.h"
#include "kern.h"
#include "pasgal.h"

// BFS requests and single-source reach requests on low-diameter graphs (mean
// out-degree above 8) do not join the batched launches: another host thread
// serves them in batches of up to 64 per graph with the multi-source
// direction-optimizing BFS (one bit per request; a reach request's mask bit
// is its source's bit of the reached set), from copies of the graph and of
// its transpose that pasgal_server_add_graph makes. Its levels and the
// batched launches take turns on the device (see DevGate).

using namespace pg;

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  int64_t id = 0;
  pasgal_request r{};
  bool dobfs = false;  // served by the direction-optimizing BFS (BFS, or reach from one source)
  bool dense = false;  // its graph has mean out-degree above 8
  double t_submit = 0, t_admit = 0;
  int64_t rounds = 0;
  int slot = -1;
  uint32_t r0 = 0;  // lane round in which the request was seeded
  int64_t off = -1, bytes = 0, dirty_off = 0;
  int32_t vbase = 0, nv = 0;
};

// One multi-query VGC engine per request kind.
struct Lane {
  int kind = KIND_BFS;
  uint64_t cap = 0;
  hipStream_t stream = nullptr;
  // stat: the control block, then one "has work" flag per slot (census)
  DBuf fv[2], fq[2], fval[2], stat, qi, qword, seeds;
  SliceBufs slices;
  HBuf h_stat, h_stage;
  uint32_t cur_buf = 0, cur_cnt = 0, cur_ovf = 0;
  uint32_t round_abs = 0;  // rounds run so far by this lane (BFS window origin of each request)
  std::vector<Req *> slots;    // slot -> request (nullptr = free)
  std::vector<Req *> fresh;    // admitted, not yet seeded
  std::vector<Req *> copying;  // finished; result copies enqueued on the stream
  std::atomic<int> active{0};
  LaunchGeom lg_full[2], lg_half[2];  // [test-first]
  LaunchGeom lg_one[2];  // single-query kernel, whole device [test-first]: a lone request's launch
  bool one_ok = false;
  bool enqueued = false;  // a slice is in flight on the stream
  size_t stat_bytes = 0;
  Ctl *ctl() const { return (Ctl *)stat.p; }
  uint32_t *flags() const { return (uint32_t *)((uint8_t *)stat.p + ctl_bytes()); }
  static size_t ctl_bytes() { return (sizeof(Ctl) + 255) & ~(size_t)255; }
  ~Lane() {
    for (DBuf *b : {&fv[0], &fv[1], &fq[0], &fq[1], &fval[0], &fval[1], &stat, &qi, &qword, &seeds}) free_buf(*b);
    for (HBuf *b : {&h_stat, &h_stage}) free_hbuf(*b);
    if (stream) hipStreamDestroy(stream);
  }
};

// The direction-optimizing levels' side of the gate.
struct SharedGate : LevelGate {
  DevGate *d;
  explicit SharedGate(DevGate *g) : d(g) {}
  void enter() override { d->enter_shared(); }
  void leave() override { d->leave_shared(); }
};

// After a lone request's single-query launch: its frontier entries get the
// request's slot as query, and the vertices it marked in the global-id
// bitmap move to the request's own dirty bitmap (local ids), so that the
// multi-query slices and the census read them as theirs.
__global__ void __launch_bounds__(256) lone_fix_kernel(const Ctl *ctl, uint32_t *fq0, uint32_t *fq1, uint32_t cap,
                                                       uint32_t slot, const uint32_t *__restrict__ gdirty,
                                                       uint32_t *__restrict__ ldirty, uint32_t vbase, uint32_t nv) {
  const uint32_t cnt = min(ctl->final_cnt, cap);
  uint32_t *fq = ctl->final_buf ? fq1 : fq0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint64_t i = t0; i < cnt; i += stride) fq[i] = slot;
  if (!ctl->final_ovf) return;
  const uint32_t words = (nv + 31) / 32, sh = vbase & 31;
  for (uint64_t j = t0; j < words; j += stride) {
    const uint64_t g = ((uint64_t)vbase >> 5) + j;  // global word holding local bit 32j
    uint32_t w = gdirty[g] >> sh;
    if (sh) w |= gdirty[g + 1] << (32 - sh);
    if (j == words - 1 && (nv & 31)) w &= (1u << (nv & 31)) - 1u;
    if (w) ldirty[j] |= w;
  }
}

// A resident graph's own copy (local vertex ids) and its transpose, kept for
// direction-optimizing BFS requests.
struct DoGraph {
  bool on = false;
  int32_t n = 0, m = 0;
  DBuf off, tgt, toff, ttgt;
  ~DoGraph() {
    for (DBuf *b : {&off, &tgt, &toff, &ttgt}) free_buf(*b);
  }
};

}  // namespace

struct pasgal_server {
  pasgal_server_opts opts{};
  Opts vopts;       // whole-device slices
  Opts vopts_half;  // slices that run beside the other kind's, on half of every compute unit
  bool half_ok = true;
  std::vector<uint8_t> densev;  // per graph: mean out-degree above 8 (guarded by graph_mu)
  hipStream_t stream = nullptr;
  int device = 0;
  // resident packed CSR
  DBuf off, tgt;
  int32_t n_total = 0, m_total = 0;
  std::mutex graph_mu;            // guards vbase/ebase
  std::vector<int32_t> vbase{0};
  std::vector<int32_t> ebase{0};
  std::vector<uint8_t> dobfs;     // per graph: BFS requests use the direction-optimizing BFS
  // request state arena
  DBuf arena;
  Arena alloc;
  Lane lanes[2];
  // direction-optimizing BFS requests (admitted, in arrival order)
  std::vector<std::unique_ptr<DoGraph>> dograph;  // per graph id
  std::deque<Req *> do_q;          // guarded by mu
  std::atomic<int> do_active{0};  // admitted direction-optimizing requests not yet completed
  // host threads (and streams) running batches of direction-optimizing
  // requests
  static constexpr int DO_THREADS = 1;
  hipStream_t do_stream[DO_THREADS] = {};
  std::thread do_thr[DO_THREADS];
  DevGate gate;
  std::condition_variable cv_do;
  // queues
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Req *> submitted;   // not yet admitted
  std::deque<pasgal_completion> done;
  int64_t next_id = 1;
  int64_t inflight = 0;          // submitted and not completed
  bool stop = false;
  std::thread thr;
  std::mutex gpu_mu;             // serializes device work (graph adds vs loop)
  // a lone request's launch runs the single-query kernel, which marks
  // overflowing vertices in a bitmap over global vertex ids
  DBuf lone_dirty;
  // yield word: bumped by every submission, polled by long launches
  uint32_t *h_yield = nullptr;   // coherent pinned host memory
  const uint32_t *d_yield = nullptr;

  ~pasgal_server() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    if (h_yield) __atomic_fetch_add(h_yield, 1u, __ATOMIC_SEQ_CST);  // end a long launch now
    cv.notify_all();
    cv_do.notify_all();
    if (thr.joinable()) thr.join();
    for (std::thread &t : do_thr)
      if (t.joinable()) t.join();
    for (Req *r : submitted) delete r;
    for (Lane &l : lanes) {
      if (l.stream) hipStreamSynchronize(l.stream);
      for (Req *r : l.slots) delete r;
      for (Req *r : l.copying) delete r;
    }
    for (Req *r : do_q) delete r;
    for (hipStream_t &st : do_stream)
      if (st) {
        hipStreamSynchronize(st);
        hipStreamDestroy(st);
      }
    dograph.clear();
    free_buf(off);
    free_buf(tgt);
    free_buf(arena);
    free_buf(lone_dirty);
    if (h_yield) hipHostFree(h_yield);
    if (stream) hipStreamDestroy(stream);
  }

  void complete(Req *r, int status) {
    pasgal_completion c{};
    c.id = r->id;
    c.tag = r->r.tag;
    c.status = status;
    c.graph = r->r.graph;
    c.t_submit_ms = r->t_submit;
    c.t_admit_ms = r->t_admit;
    c.t_done_ms = now_ms();
    c.rounds = r->rounds;
    {
      std::lock_guard<std::mutex> lk(mu);
      done.push_back(c);
      inflight--;
    }
    cv_done.notify_all();
    delete r;
  }

  int64_t state_bytes(const Req *r) const {
    if (r->dobfs)  // the distances or mask words, unless they go straight to the caller's array
      return r->r.out ? 0 : (r->r.kind == PASGAL_REQ_BFS ? 4 : 8) * (int64_t)r->nv;
    const int64_t es = r->r.kind == PASGAL_REQ_BFS ? 4 : 8;
    const int64_t words = ((int64_t)r->nv + 31) / 32;
    return ((es * r->nv + 255) & ~(int64_t)255) + 4 * words;
  }

  // Admit queued requests while slots and memory allow (FIFO, head-of-line),
  // under the queue lock, so that every request counts as queued or as
  // admitted at any time.
  void admit() {
    std::lock_guard<std::mutex> lk(mu);
    while (!submitted.empty()) {
      Req *r = submitted.front();
      if (r->dobfs) {
        const int64_t bytes = state_bytes(r);
        const int64_t o = bytes > 0 ? alloc.alloc(bytes) : 0;
        if (o < 0) break;
        submitted.pop_front();
        r->off = bytes > 0 ? o : -1;
        r->bytes = bytes;
        r->t_admit = now_ms();
        do_q.push_back(r);
        do_active++;
        cv_do.notify_one();
        continue;
      }
      Lane &L = lanes[r->r.kind == PASGAL_REQ_BFS ? 0 : 1];
      int slot = -1;
      for (size_t i = 0; i < L.slots.size(); i++)
        if (!L.slots[i]) {
          slot = (int)i;
          break;
        }
      const int64_t bytes = state_bytes(r);
      const int64_t o = slot >= 0 ? alloc.alloc(bytes) : -1;
      if (o < 0) break;  // keep arrival order: later requests wait too
      submitted.pop_front();
      r->off = o;
      r->bytes = bytes;
      const int64_t es = r->r.kind == PASGAL_REQ_BFS ? 4 : 8;
      r->dirty_off = o + ((es * r->nv + 255) & ~(int64_t)255);
      r->slot = slot;
      r->t_admit = now_ms();
      L.slots[slot] = r;
      L.fresh.push_back(r);
      L.active++;
    }
  }

  // Return a request's arena memory (the allocator is shared by the loop and
  // the direction-optimizing thread; it is used under the queue lock).
  void release(Req *r) {
    if (r->bytes <= 0) return;
    std::lock_guard<std::mutex> lk(mu);
    alloc.release(r->off, r->bytes);
  }

  void fail_lane(Lane &L, int status) {
    if (L.stream) hipStreamSynchronize(L.stream);
    (void)hipGetLastError();
    L.enqueued = false;
    finish_copies(L);
    for (size_t i = 0; i < L.slots.size(); i++)
      if (L.slots[i]) {
        Req *r = L.slots[i];
        release(r);
        L.slots[i] = nullptr;
        complete(r, status);
      }
    L.fresh.clear();
    L.active = 0;
    L.cur_cnt = 0;
    L.cur_ovf = 0;
  }

  // After a wait on the lane's stream: the result copies enqueued before it
  // are done, so those requests complete and their memory is returned.
  void finish_copies(Lane &L) {
    for (Req *r : L.copying) {
      release(r);
      complete(r, PASGAL_OK);
    }
    L.copying.clear();
  }

  // Enqueue one slice of one kind on the lane's stream (no wait): tables,
  // state of fresh requests, seeds, the persistent launch, the census and one
  // copy back of the control block and flags. half: the launch runs beside
  // the other kind's, on half of every compute unit. lone: the launch runs
  // until its work is done or the yield word differs from ybase. Returns a
  // PASGAL_* code.
  int enqueue_slice(Lane &L, bool half, bool lone = false, uint32_t ybase = 0) {
    hipStream_t s = L.stream;
    const int kind = L.kind;
    const int nslots = (int)L.slots.size();
    const size_t es = kind == KIND_BFS ? 4 : 8;
    // test-first: as asked, else when a request of the launch is on a graph
    // with mean out-degree above 8
    bool any_dense = false;
    for (const Req *r : L.slots) any_dense = any_dense || (r && r->dense);
    const bool tf = (opts.flags & PASGAL_FLAG_TEST_FIRST) ? true
                    : (opts.flags & PASGAL_FLAG_NO_TEST_FIRST) ? false
                                                               : any_dense;
    const LaunchGeom &lg = half ? L.lg_half[tf] : L.lg_full[tf];
    Opts vo = half ? vopts_half : vopts;
    vo.test_first = tf;
    // query tables over all slots (inactive slots own no words)
    std::vector<QInfo> qi(nslots);
    std::vector<int64_t> qword(nslots + 1, 0);
    int64_t words = 0;
    for (int i = 0; i < nslots; i++) {
      const Req *r = L.slots[i];
      qword[i] = words;
      if (r) {
        qi[i].sbase = r->off / (int64_t)es - r->vbase;
        qi[i].dbase = r->dirty_off / 4;
        qi[i].vbase = r->vbase;
        qi[i].nv = r->nv;
        qi[i].r0 = r->r0;
        qi[i].pad = 0;
        words += (r->nv + 31) / 32;
      } else {
        qi[i] = QInfo{0, 0, 0, 0, 0, 0};
      }
    }
    qword[nslots] = words;
    std::vector<SeedEnt> seeds;
    std::vector<int64_t> segoff, seglen, doff, dlen;
    for (Req *r : L.fresh) {
      r->r0 = L.round_abs;
      qi[r->slot].r0 = r->r0;
      for (int k = 0; k < r->r.nsources; k++) {
        SeedEnt e;
        e.v = (uint32_t)(r->vbase + r->r.sources[k]);
        e.q = (uint32_t)r->slot;
        e.val = kind == KIND_BFS ? 0ull : (1ull << k);
        seeds.push_back(e);
      }
      segoff.push_back(r->off / (int64_t)es);
      seglen.push_back(r->nv);
      doff.push_back(r->dirty_off / 4);
      dlen.push_back((r->nv + 31) / 32);
    }
    const size_t nseed = seeds.size(), nfresh = L.fresh.size();
    // pinned staging: qi | qword | seeds | segoff | seglen | doff | dlen
    const size_t b_qi = sizeof(QInfo) * nslots, b_qw = sizeof(int64_t) * (nslots + 1),
                 b_se = sizeof(SeedEnt) * std::max<size_t>(nseed, 1), b_sg = sizeof(int64_t) * std::max<size_t>(nfresh, 1);
    int rc;
    if ((rc = grow_host(L.h_stage, b_qi + b_qw + b_se + 4 * b_sg))) return rc;
    if ((rc = grow(L.seeds, b_se + 4 * b_sg))) return rc;
    uint8_t *hs = (uint8_t *)L.h_stage.p;
    memcpy(hs, qi.data(), b_qi);
    memcpy(hs + b_qi, qword.data(), b_qw);
    uint8_t *hx = hs + b_qi + b_qw;
    if (nseed) memcpy(hx, seeds.data(), sizeof(SeedEnt) * nseed);
    int64_t *hseg = (int64_t *)(hx + b_se);
    for (size_t i = 0; i < nfresh; i++) {
      hseg[i] = segoff[i];
      hseg[b_sg / 8 + i] = seglen[i];
      hseg[2 * b_sg / 8 + i] = doff[i];
      hseg[3 * b_sg / 8 + i] = dlen[i];
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(L.qi.p, hs, b_qi, hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpyAsync(L.qword.p, hs + b_qi, b_qw, hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpyAsync(L.seeds.p, hx, b_se + 4 * b_sg, hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_fail(e);
    const int64_t *dsegoff = (const int64_t *)((uint8_t *)L.seeds.p + b_se);
    const int64_t *dseglen = dsegoff + b_sg / 8, *ddoff = dsegoff + 2 * b_sg / 8, *ddlen = dsegoff + 3 * b_sg / 8;
    if (nfresh) {
      if (kind == KIND_BFS)
        e = launch_fill_segments_u32((uint32_t *)arena.p, dsegoff, dseglen, (int32_t)nfresh, 0xFFFFFFFFu, s);
      else
        e = launch_fill_segments_u64((unsigned long long *)arena.p, dsegoff, dseglen, (int32_t)nfresh, 0ull, s);
      if (e != hipSuccess) return hip_fail(e);
      if ((e = launch_fill_segments_u32((uint32_t *)arena.p, ddoff, ddlen, (int32_t)nfresh, 0u, s)) != hipSuccess)
        return hip_fail(e);
    }
    VgcArgs a{};
    a.off = (const int32_t *)off.p;
    a.tgt = (const int32_t *)tgt.p;
    a.state = arena.p;
    a.dirty = (uint32_t *)arena.p;
    a.qi = (const QInfo *)L.qi.p;
    a.qword = (const int64_t *)L.qword.p;
    a.dirty_words = words;
    a.nq = nslots;
    for (int i = 0; i < 2; i++) {
      a.fr.v[i] = (uint32_t *)L.fv[i].p;
      a.fr.q[i] = (uint32_t *)L.fq[i].p;
      a.fr.val[i] = (unsigned long long *)L.fval[i].p;
    }
    a.fr.cap = (uint32_t)L.cap;
    a.start_buf = L.cur_buf;
    a.tau = vo.tau;
    a.max_rounds = lone ? 0x40000000u : (uint32_t)opts.slice_rounds;
    if (lone) {
      a.yield = d_yield;
      a.yield_base = ybase;
    }
    a.ring_cap = lg.ring;
    a.stage_cap = lg.stage;
    a.min_chunk = vo.min_chunk;
    a.chunks_per_wave = vo.cpw;
    a.window = vo.window;
    a.round_base = L.round_abs;
    a.test_first = vo.test_first ? 1u : 0u;
    // filter keys are 32-bit state indices: exact only below 2^32 values
    a.filt = (uint64_t)arena.bytes / es < (1ull << 32) ? lg.filt : 0u;
    a.timeout_ticks = (long long)vo.timeout_ms * (long long)dev_info().wall_khz;
    a.ctl = L.ctl();
    // a hub may be cut once per request that expands it
    const uint32_t hcap = slice_capacity((uint64_t)m_total * 8, vo.heavy, L.cap);
    if (int rc2 = L.slices.ensure(hcap, true)) return rc2;
    L.slices.apply(a, vo.heavy, hcap, true);
    // control block and census flags start at zero
    if ((e = launch_fill_u32((uint32_t *)L.stat.p, L.stat_bytes / 4, 0u, s)) != hipSuccess) return hip_fail(e);
    if ((e = launch_seed(kind, a, (const SeedEnt *)L.seeds.p, (uint32_t)nseed, L.cur_cnt, L.cur_ovf, s)) !=
        hipSuccess)
      return hip_fail(e);
    // a lone request with no dirty bits pending runs in the single-query
    // kernel (faster on one query), on its own state region addressed by
    // global vertex id, with a global-id dirty bitmap; lone_fix_kernel then
    // hands its frontier back in the multi-query layout
    Req *one = nullptr;
    if (lone && !half && L.one_ok && L.cur_ovf == 0)
      for (Req *r : L.slots)
        if (r) one = r;
    if (one) {
      const LaunchGeom &l1 = L.lg_one[tf];
      const uint64_t gwords = ((uint64_t)n_total + 31) / 32 + 1;
      if (int rc2 = grow(lone_dirty, 4 * gwords)) return rc2;
      VgcArgs b = a;
      b.state = (uint8_t *)arena.p + one->off - (int64_t)one->vbase * (int64_t)es;
      b.dirty = (uint32_t *)lone_dirty.p;
      b.dirty_words = (int64_t)gwords;
      b.qi = nullptr;
      b.qword = nullptr;
      b.nq = 1;
      for (int i = 0; i < 2; i++) b.fr.q[i] = nullptr;
      b.round_base = L.round_abs - one->r0;  // the request's own window origin
      b.ring_cap = l1.ring;
      b.stage_cap = l1.stage;
      b.filt = l1.filt;  // keys are global vertex ids
      L.slices.apply(b, vo.heavy, hcap, false);
      if ((e = launch_fill_u32((uint32_t *)lone_dirty.p, gwords, 0u, s)) != hipSuccess) return hip_fail(e);
      if ((e = launch_vgc(kind, false, l1.pf, b, l1.grid, l1.block, l1.lds, coop_launch(vo), s)) != hipSuccess)
        return hip_fail(e);
      (void)hipGetLastError();
      const uint32_t fix_items = std::max<uint32_t>((uint32_t)std::min<uint64_t>(L.cap, 1u << 30), ((uint32_t)one->nv + 31) / 32);
      const int fix_blocks = (int)std::max<uint64_t>(1, std::min<uint64_t>(8192, ((uint64_t)fix_items + 255) / 256));
      hipLaunchKernelGGL(lone_fix_kernel, dim3(fix_blocks), dim3(256), 0, s, (const Ctl *)L.ctl(), (uint32_t *)L.fq[0].p,
                         (uint32_t *)L.fq[1].p, (uint32_t)L.cap, (uint32_t)one->slot, (const uint32_t *)lone_dirty.p,
                         (uint32_t *)((uint8_t *)arena.p + one->dirty_off), (uint32_t)one->vbase, (uint32_t)one->nv);
      if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e);
    } else if ((e = launch_vgc(kind, true, lg.pf, a, lg.grid, lg.block, lg.lds, coop_launch(vo), s)) != hipSuccess) {
      return hip_fail(e);
    }
    if ((e = launch_census((const uint32_t *)L.fq[0].p, (const uint32_t *)L.fq[1].p, L.ctl(), (uint32_t)L.cap,
                           L.flags(), (const QInfo *)L.qi.p, (const int64_t *)L.qword.p, (const uint32_t *)arena.p,
                           nslots, s)) != hipSuccess)
      return hip_fail(e);
    if ((e = hipMemcpyAsync(L.h_stat.p, L.stat.p, L.stat_bytes, hipMemcpyDeviceToHost, s)) != hipSuccess)
      return hip_fail(e);
    L.fresh.clear();
    L.enqueued = true;
    return PASGAL_OK;
  }

  // After the wait on the lane's stream: read the slice's exit record and
  // census, enqueue the result copies of finished requests (they complete
  // after the next wait) and free their slots.
  int finish_slice(Lane &L) {
    L.enqueued = false;
    const Ctl c = *(const Ctl *)L.h_stat.p;
    if (c.abort) return PASGAL_ETIMEOUT;
    L.cur_buf = c.final_buf;
    L.cur_cnt = c.final_cnt;
    L.cur_ovf = c.final_ovf;
    L.round_abs += c.rounds;
    const uint32_t *flags = (const uint32_t *)((const uint8_t *)L.h_stat.p + Lane::ctl_bytes());
    const size_t es = L.kind == KIND_BFS ? 4 : 8;
    hipError_t e;
    for (size_t i = 0; i < L.slots.size(); i++) {
      Req *r = L.slots[i];
      if (!r) continue;
      r->rounds += c.rounds;
      if (flags[i]) continue;
      if (r->r.out) {
        if ((e = hipMemcpyAsync(r->r.out, (uint8_t *)arena.p + r->off, es * (size_t)r->nv, hipMemcpyDeviceToDevice,
                                L.stream)) != hipSuccess)
          return hip_fail(e);
      }
      L.slots[i] = nullptr;
      L.active--;
      L.copying.push_back(r);
    }
    return PASGAL_OK;
  }

  // One direction-optimizing BFS request, start to finish (synchronous).
  // A batch of direction-optimizing requests on one graph (at most 64, one
  // source each), start to finish in one multi-source run (synchronous).
  void run_do(std::vector<Req *> &batch, hipStream_t ds) {
    const DoGraph &G = *dograph[batch[0]->r.graph];
    pasgal_csr g{G.n, G.m, (const int32_t *)G.off.p, (const int32_t *)G.tgt.p};
    pasgal_csr gt{G.n, G.m, (const int32_t *)G.toff.p, (const int32_t *)G.ttgt.p};
    pasgal_opts po;
    pasgal_opts_default(&po);
    po.stream = ds;
    po.timeout_ms = opts.timeout_ms;
    const int k = (int)batch.size();
    std::vector<int32_t> src(k);
    std::vector<MsQuery> qs(k);
    for (int q = 0; q < k; q++) {
      Req *r = batch[q];
      src[q] = r->r.sources[0];
      void *out = r->r.out ? r->r.out : (void *)((uint8_t *)arena.p + r->off);
      qs[q].dist = r->r.kind == PASGAL_REQ_BFS ? (int32_t *)out : nullptr;
      qs[q].mask1 = r->r.kind == PASGAL_REQ_BFS ? nullptr : (unsigned long long *)out;
    }
    pasgal_stats st{};
    SharedGate sg(&gate);
    const int rc = ms_bfs_do_gated(&g, &gt, k, src.data(), qs.data(), nullptr, 0, 0, &po, &st, &sg);
    for (Req *r : batch) {
      r->rounds = st.rounds;
      release(r);
      do_active--;
      complete(r, rc);
    }
  }

  // Direction-optimizing thread k: takes the oldest queued request and up to
  // 63 more queued on the same graph, in admission order, as one batch.
  void do_loop(int k) {
    hipSetDevice(device);
    std::vector<Req *> batch;
    while (true) {
      batch.clear();
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_do.wait(lk, [&] { return stop || !do_q.empty(); });
        if (stop) return;
        const int32_t gid = do_q.front()->r.graph;
        for (auto it = do_q.begin(); it != do_q.end() && batch.size() < 64;) {
          if ((*it)->r.graph == gid) {
            batch.push_back(*it);
            it = do_q.erase(it);
          } else {
            ++it;
          }
        }
      }
      run_do(batch, do_stream[k]);
      cv.notify_all();
    }
  }

  // Wait for the lane's stream; complete the requests whose copies were
  // enqueued before, and read the slice that was in flight.
  void wait_lane(Lane &L) {
    if (!L.enqueued && L.copying.empty()) return;
    hipError_t e = hipStreamSynchronize(L.stream);
    if (e != hipSuccess) {
      fail_lane(L, hip_fail(e));
      return;
    }
    finish_copies(L);
    if (L.enqueued) {
      if (int rc = finish_slice(L)) fail_lane(L, rc);
    }
  }

  void loop() {
    hipSetDevice(device);
    while (true) {
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait_for(lk, std::chrono::milliseconds(50), [&] {
          return stop || !submitted.empty() || lanes[0].active > 0 || lanes[1].active > 0 ||
                 !lanes[0].copying.empty() || !lanes[1].copying.empty();
        });
        if (stop) return;
      }
      std::lock_guard<std::mutex> g(gpu_mu);
      // read before admitting: a submission after this point ends a long launch
      const uint32_t ybase = __atomic_load_n(h_yield, __ATOMIC_SEQ_CST);
      admit();
      bool queued;
      {
        std::lock_guard<std::mutex> lk(mu);
        queued = !submitted.empty();
      }
      // with direction-optimizing requests waiting for the device, a slice
      // is short (it holds the device exclusively)
      const bool do_busy = do_active > 0;
      const bool lone = !(opts.flags & PASGAL_SERVER_FIXED_SLICES) && !queued && !do_busy &&
                        lanes[0].active + lanes[1].active == 1;
      const bool work = lanes[0].active > 0 || lanes[1].active > 0 || !lanes[0].copying.empty() ||
                        !lanes[1].copying.empty();
      if (!work) {
        // requests wait for memory that direction-optimizing requests hold
        if (queued) std::this_thread::sleep_for(std::chrono::microseconds(200));
        continue;
      }
      gate.enter_excl();
      // both kinds with work: their launches run at the same time, each on
      // half of every compute unit; otherwise one after the other, each on
      // the whole device
      const bool both = half_ok && lanes[0].active > 0 && lanes[1].active > 0;
      if (both) {
        for (Lane &L : lanes)
          if (int rc = enqueue_slice(L, true)) fail_lane(L, rc);
        for (Lane &L : lanes) wait_lane(L);
      } else {
        for (Lane &L : lanes) {
          if (L.active > 0) {
            if (int rc = enqueue_slice(L, false, lone, ybase)) fail_lane(L, rc);
          }
          wait_lane(L);
        }
      }
      gate.leave_excl();
    }
  }
};

extern "C" {

int pasgal_server_create(const pasgal_server_opts *o, pasgal_server **out) {
  if (!out) return PASGAL_EINVAL;
  *out = nullptr;
  pasgal_server *s = new (std::nothrow) pasgal_server();
  if (!s) return PASGAL_ENOMEM;
  if (o) s->opts = *o;
  pasgal_server_opts &so = s->opts;
  if (so.max_slots <= 0) so.max_slots = 256;
  if (so.slice_rounds <= 0) so.slice_rounds = 32;  // c5 saturation: 163 q/s at 32 or 64, 143 at 16
  if (so.timeout_ms <= 0) so.timeout_ms = 20000;
  if (so.memory_budget <= 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      return PASGAL_EHIP;
    }
    so.memory_budget = (int64_t)(fr / 4);
  }
  if ((so.flags & ~(uint32_t)(PASGAL_FLAG_TEST_FIRST | PASGAL_FLAG_NO_TEST_FIRST | PASGAL_SERVER_FIXED_SLICES |
                              PASGAL_SERVER_NO_DIRECTION_OPT)) ||
      so.reserved != 0) {
    delete s;
    return PASGAL_EINVAL;
  }
  if (so.max_slots > 4096) {
    delete s;
    return PASGAL_EINVAL;
  }
  hipGetDevice(&s->device);
  pasgal_opts po;
  pasgal_opts_default(&po);
  // c5 at 150 q/s offered: p50 0.43 s at tau 256, 0.97 s at 1024, 1.04 s at 4096
  po.tau = so.tau > 0 ? so.tau : 256;
  if (so.wg_size > 0) po.wg_size = so.wg_size;
  if (so.blocks_per_cu > 0) po.blocks_per_cu = so.blocks_per_cu;
  po.timeout_ms = so.timeout_ms;
  po.window = so.window;
  // arc ranges carried in the local queues: a lone 8192^2 grid BFS request
  // measured 31 ms with them against 33.5 ms without
  po.flags |= PASGAL_FLAG_PREFETCH;
  if (!opts_valid(&po)) {
    delete s;
    return PASGAL_EINVAL;
  }
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e);
  }
  void *hy = nullptr;
  if ((e = hipHostMalloc(&hy, 256, hipHostMallocCoherent | hipHostMallocMapped)) != hipSuccess) {
    delete s;
    return hip_fail(e);
  }
  s->h_yield = (uint32_t *)hy;
  *s->h_yield = 0;
  void *dy = nullptr;
  if ((e = hipHostGetDevicePointer(&dy, hy, 0)) != hipSuccess) {
    delete s;
    return hip_fail(e);
  }
  s->d_yield = (const uint32_t *)dy;
  for (hipStream_t &st : s->do_stream)
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) {
      delete s;
      return hip_fail(e);
    }
  po.stream = s->stream;
  s->vopts = resolve_opts(&po);
  // the half-device slices: half the workgroup size (each CU then holds one
  // workgroup of each kind)
  s->vopts_half = s->vopts;
  s->vopts_half.share = 50;
  s->vopts_half.wg = std::max(64, (s->vopts.wg / 2) & ~63);
  int rc = grow(s->arena, (size_t)so.memory_budget);
  if (rc) {
    delete s;
    return rc;
  }
  s->alloc.reset(so.memory_budget);
  const uint64_t cap = so.frontier_capacity > 0 ? (uint64_t)so.frontier_capacity : (64ull << 20);
  for (int k = 0; k < 2; k++) {
    Lane &L = s->lanes[k];
    L.kind = k == 0 ? KIND_BFS : KIND_REACH;
    L.cap = std::min<uint64_t>(cap, 0x7FFFFFFFull);
    L.slots.assign(so.max_slots, nullptr);
    for (int i = 0; i < 2 && !rc; i++) {
      rc = grow(L.fv[i], 4 * L.cap);
      if (!rc) rc = grow(L.fq[i], 4 * L.cap);
      if (!rc) rc = grow(L.fval[i], 8 * L.cap);
    }
    L.stat_bytes = Lane::ctl_bytes() + 4 * (size_t)so.max_slots;
    if (!rc) rc = grow(L.stat, L.stat_bytes);
    if (!rc) rc = grow(L.qi, sizeof(QInfo) * so.max_slots);
    if (!rc) rc = grow(L.qword, sizeof(int64_t) * (so.max_slots + 1));
    if (!rc) rc = grow_host(L.h_stat, L.stat_bytes);
    for (int tf = 0; tf < 2 && !rc; tf++) {
      Opts full = s->vopts, half = s->vopts_half;
      full.test_first = half.test_first = tf != 0;
      rc = vgc_geometry(L.kind, true, full, L.lg_full[tf]);
      if (!rc) L.one_ok = vgc_geometry(L.kind, false, full, L.lg_one[tf]) == PASGAL_OK && (tf == 0 || L.one_ok);
      // without room for the half-device geometry the kinds take turns
      if (!rc && vgc_geometry(L.kind, true, half, L.lg_half[tf]) != PASGAL_OK) s->half_ok = false;
    }
    if (!rc) {
      hipError_t e2 = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
      if (e2 != hipSuccess) rc = hip_fail(e2);
    }
    if (rc) {
      delete s;
      return rc;
    }
  }
  try {
    s->thr = std::thread([s] { s->loop(); });
    for (int k = 0; k < pasgal_server::DO_THREADS; k++) s->do_thr[k] = std::thread([s, k] { s->do_loop(k); });
  } catch (...) {
    delete s;
    return PASGAL_ENOMEM;
  }
  *out = s;
  return PASGAL_OK;
}

int pasgal_server_add_graph(pasgal_server *s, const pasgal_csr *g, int32_t *graph_id) {
  if (!s || !csr_valid(g) || !graph_id) return PASGAL_EINVAL;
  std::lock_guard<std::mutex> gl(s->gpu_mu);
  const int64_t n2 = (int64_t)s->n_total + g->n, m2 = (int64_t)s->m_total + g->m;
  if (n2 >= 0x7FFFFFFFLL || m2 >= 0x7FFFFFFFLL) return PASGAL_ECAPACITY;
  {  // no request may be queued or resident while the packed CSR moves
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->inflight || s->lanes[0].active || s->lanes[1].active) return PASGAL_EAGAIN;
  }
  DBuf noff, ntgt;
  int rc = grow(noff, 4 * (size_t)(n2 + 1));
  if (!rc) rc = grow(ntgt, 4 * (size_t)std::max<int64_t>(m2, 1));
  if (rc) {
    free_buf(noff);
    free_buf(ntgt);
    return rc;
  }
  hipStream_t st = s->stream;
  hipError_t e = hipSuccess;
  if (s->n_total > 0) {
    e = hipMemcpyAsync(noff.p, s->off.p, 4 * (size_t)s->n_total, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && s->m_total > 0)
      e = hipMemcpyAsync(ntgt.p, s->tgt.p, 4 * (size_t)s->m_total, hipMemcpyDeviceToDevice, st);
  }
  if (e == hipSuccess)
    e = launch_add_const((int32_t *)noff.p + s->n_total, g->offsets, (int64_t)g->n + 1, s->m_total, st);
  if (e == hipSuccess && g->m > 0)
    e = launch_add_const((int32_t *)ntgt.p + s->m_total, g->targets, g->m, s->n_total, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    free_buf(noff);
    free_buf(ntgt);
    return hip_fail(e);
  }
  // low-diameter graph: own copy and transpose for direction-optimizing BFS
  std::unique_ptr<DoGraph> dg(new (std::nothrow) DoGraph());
  if (!dg) {
    free_buf(noff);
    free_buf(ntgt);
    return PASGAL_ENOMEM;
  }
  const bool dense = (int64_t)g->m > 8 * (int64_t)g->n;
  if (dense && !(s->opts.flags & PASGAL_SERVER_NO_DIRECTION_OPT)) {
    DoGraph &D = *dg;
    D.n = g->n;
    D.m = g->m;
    const size_t bo = 4 * ((size_t)g->n + 1), bt = 4 * (size_t)std::max<int32_t>(g->m, 1);
    rc = grow(D.off, bo);
    if (!rc) rc = grow(D.tgt, bt);
    if (!rc) rc = grow(D.toff, bo);
    if (!rc) rc = grow(D.ttgt, bt);
    if (!rc) {
      e = hipMemcpyAsync(D.off.p, g->offsets, bo, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess && g->m > 0) e = hipMemcpyAsync(D.tgt.p, g->targets, 4 * (size_t)g->m, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) rc = hip_fail(e);
    }
    if (!rc) {
      pasgal_csr lc{g->n, g->m, (const int32_t *)D.off.p, (const int32_t *)D.tgt.p};
      pasgal_opts po;
      pasgal_opts_default(&po);
      po.stream = st;
      rc = pasgal_transpose(&lc, (int32_t *)D.toff.p, (int32_t *)D.ttgt.p, &po);
    }
    if (rc) {
      free_buf(noff);
      free_buf(ntgt);
      return rc;
    }
    D.on = true;
  }
  free_buf(s->off);
  free_buf(s->tgt);
  s->off = noff;
  s->tgt = ntgt;
  s->n_total = (int32_t)n2;
  s->m_total = (int32_t)m2;
  s->dograph.push_back(std::move(dg));
  const bool dob = s->dograph.back()->on;
  std::lock_guard<std::mutex> gm(s->graph_mu);
  s->vbase.push_back((int32_t)n2);
  s->ebase.push_back((int32_t)m2);
  s->dobfs.push_back(dob ? 1 : 0);
  s->densev.push_back(dense ? 1 : 0);
  *graph_id = (int32_t)s->vbase.size() - 2;
  return PASGAL_OK;
}

int pasgal_server_submit(pasgal_server *s, const pasgal_request *req, int64_t *id) {
  if (!s || !req || !id) return PASGAL_EINVAL;
  if (req->kind != PASGAL_REQ_BFS && req->kind != PASGAL_REQ_REACH) return PASGAL_EINVAL;
  int32_t nv = 0, vb = 0;
  bool dob = false, dense = false;
  {
    std::lock_guard<std::mutex> gm(s->graph_mu);
    const int32_t ng = (int32_t)s->vbase.size() - 1;
    if (req->graph < 0 || req->graph >= ng) return PASGAL_ENOTFOUND;
    vb = s->vbase[req->graph];
    nv = s->vbase[req->graph + 1] - vb;
    dob = s->dobfs[req->graph] != 0;
    dense = s->densev[req->graph] != 0;
  }
  if (req->nsources < 1 || req->nsources > 64 || (req->kind == PASGAL_REQ_BFS && req->nsources != 1))
    return PASGAL_EINVAL;
  for (int i = 0; i < req->nsources; i++)
    if (req->sources[i] < 0 || req->sources[i] >= nv) return PASGAL_EINVAL;
  Req *r = new (std::nothrow) Req();
  if (!r) return PASGAL_ENOMEM;
  r->r = *req;
  r->vbase = vb;
  r->nv = nv;
  r->dobfs = dob && (req->kind == PASGAL_REQ_BFS || req->nsources == 1);
  r->dense = dense;
  r->t_submit = now_ms();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->state_bytes(r) > s->opts.memory_budget) {
      delete r;
      return PASGAL_ECAPACITY;
    }
    if (s->submitted.size() >= 1u << 20) {
      delete r;
      return PASGAL_EAGAIN;
    }
    r->id = s->next_id++;
    s->submitted.push_back(r);
    s->inflight++;
    *id = r->id;
  }
  __atomic_fetch_add(s->h_yield, 1u, __ATOMIC_SEQ_CST);  // a long launch ends at its next round boundary
  s->cv.notify_all();
  return PASGAL_OK;
}

int pasgal_server_poll(pasgal_server *s, pasgal_completion *out, int32_t max, int32_t *count) {
  if (!s || !count || (max > 0 && !out)) return PASGAL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t c = 0;
  while (c < max && !s->done.empty()) {
    out[c++] = s->done.front();
    s->done.pop_front();
  }
  *count = c;
  return PASGAL_OK;
}

int pasgal_server_drain(pasgal_server *s, int32_t timeout_ms) {
  if (!s) return PASGAL_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok = s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms > 0 ? timeout_ms : 60000),
                                      [&] { return s->inflight == 0; });
  return ok ? PASGAL_OK : PASGAL_ETIMEOUT;
}

int pasgal_server_load(pasgal_server *s, int32_t *queued, int32_t *active, int64_t *bytes_in_use) {
  if (!s) return PASGAL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = (int32_t)s->submitted.size();
  if (active) *active = s->lanes[0].active + s->lanes[1].active + s->do_active;
  if (bytes_in_use) *bytes_in_use = s->alloc.used;
  return PASGAL_OK;
}

void pasgal_server_destroy(pasgal_server *s) { delete s; }

}  // extern "C"
