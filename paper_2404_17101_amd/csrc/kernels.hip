// kernels.hip -- gfx950 (CDNA4) kernels for frontier traversal with vertical
// granularity control (VGC).
//
// Paper mapping (PASGAL, SPAA'24):
//  * Algorithm 1 (frontier framework): rounds over a frontier F_i; every
//    vertex of F_i visits its neighbours and puts a subset into F_{i+1}.
//    plain_*_level kernels run one round per launch (VGC off).
//  * Vertical granularity control (Parallel SCC section): each frontier
//    vertex runs a local search that keeps going for about tau vertices over
//    several hops before the leftovers go to the next frontier.
//    vgc_kernel runs all rounds inside one persistent launch; one wavefront
//    runs one local search over the frontier vertices it claimed, with its
//    queue in LDS.
//  * BFS with VGC (Other Algorithms section): a vertex is (re)queued whenever
//    the search lowers its hop distance, so a vertex may be expanded more than
//    once; atomicMin keeps every stored value the length of a real walk and
//    the fixpoint is the exact hop distance.
//  * Reachability (Parallel SCC section): order is free, so the local search
//    is a LIFO stack (deep first); masks grow by atomicOr, one bit per source.
//  * The hash-bag frontier is replaced by per-wavefront LDS append buffers:
//    ballot + mbcnt give each lane its slot, one global atomicAdd reserves
//    room for a whole buffer, and the copy out is coalesced.
//
// Memory model: every datum that one workgroup writes and another reads in
// the same launch (state, frontier entries, counters, dirty bits) is accessed
// with agent-scope relaxed atomics, which gfx950 executes coherently across
// its XCDs without L2 writeback/invalidate. The grid barrier waits for each
// wave's memory operations to complete (s_waitcnt 0) before arriving. CSR
// arrays are read-only during a launch and use ordinary cached loads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "devutil.h"
#include "engine.h"
#include "kern.h"

namespace pg {

// Round state every workgroup needs after a barrier; read once per
// workgroup by thread 0 and broadcast through LDS.
struct RoundHdr {
  uint32_t ncur, ovf, nheavy, abort, yld;
};

// The per-query fields a step reads (state base, window origin), copied to
// LDS at the start of a multi-query launch of at most QLITE queries so that
// a step does not wait on a memory load for them.
struct QLite {
  int64_t sbase;
  uint32_t r0, pad;
};
constexpr int QLITE = 64;
// Typed as LDS so that a lookup is a ds_read: through a generic pointer the
// compiler merges it with the global fallback into a flat load, whose wait
// also waits for every relaxation in flight.
typedef __attribute__((address_space(3))) QLite LdsQLite;
typedef __attribute__((address_space(3))) unsigned long long LdsU64;
typedef __attribute__((address_space(3))) int32_t LdsI32;
// Source vertex -> its bits, an open-addressing table of this many slots in
// LDS (at most 64 sources: load factor at most 1/2).
constexpr int SRC_SLOTS = 128;
__device__ __forceinline__ uint32_t src_slot(uint32_t v) { return (v * 0x9E3779B1u) >> 25; }

// Grid barrier for a persistent launch whose workgroups are all resident.
// Fence-free: callers keep cross-workgroup data in agent-scope atomics.
// After the wait, thread 0 reads the counters of slot `slot` for everyone.
__device__ void grid_barrier(Ctl *ctl, uint32_t &epoch, long long deadline, uint32_t slot, RoundHdr *hdr) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    epoch += 1;
    const uint32_t target = epoch * gridDim.x;
    add_ag(&ctl->bar, 1u);
    uint32_t ab = 0, polls = 0;
    while (ld_ag(&ctl->bar) < target) {
      if ((++polls & 15u) == 0 && ld_ag(&ctl->abort)) { ab = 1; break; }
      if (wall_clock64() > deadline) {
        st_ag(&ctl->abort, 1u);
        ab = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (ld_ag(&ctl->abort)) ab = 1;
    hdr->abort = ab;
    hdr->ncur = ld_ag(&ctl->cnt[slot]);
    hdr->ovf = ld_ag(&ctl->ovf[slot]);
    hdr->nheavy = ld_ag(&ctl->hcnt[slot]);
    hdr->yld = ld_ag(&ctl->yld[slot]);
  }
  __syncthreads();
}

// ------------------------------------------------------------ VGC engine --

template <int KIND>
struct ValT;
template <>
struct ValT<KIND_BFS> { using T = uint32_t; };
template <>
struct ValT<KIND_REACH> { using T = unsigned long long; };
template <>
struct ValT<KIND_SSSP> { using T = uint32_t; };

template <int KIND, bool MULTI, bool PF, bool TF>
struct Wave {
  using Val = typename ValT<KIND>::T;
  static constexpr bool FIFO = (KIND != KIND_REACH);  // distances: local BFS order; reach: LIFO (deep first)
  static constexpr bool DIST = (KIND != KIND_REACH);  // BFS and SSSP: uint32 distances lowered by atomicMin
  // PF: local-queue entries carry their vertex's arc range, loaded while the
  // relaxing atomic is in flight, so expanding them starts at the targets.
  // TF: a plain load of the target's state before the atomic rules out
  // relaxations that cannot change it (test-first).
  // Most passes of up to this many 64-arc batches are issued together
  // (target loads, then atomics, then pushes), so that a lane has several
  // relaxations in flight. The plain multi-query BFS variant takes five: a
  // full step of 64 entries of out-degree 5 is then one block instead of two
  // (batched 16-query BFS on the 5-NN graph: 19.5 against 19.95 ms). Every
  // other variant takes four; single-query BFS gained from the wider blocks
  // too (one query on the 10M-point 5-NN graph, tau 1024 with a 32-level
  // window: 8.6 against 9.6 ms), at 3% on the 8192x8192 grid.
  static constexpr int RB = (MULTI && KIND == KIND_BFS && !PF && !TF) ? 5 : 4;
  // BFS runs a step with exactly three blocks left as one three-pass block
  // (batched 16-query BFS on the 5-NN graph: 19.5 -> 18.7 ms); reach and
  // SSSP split it into two and one, which measured 4% faster for 64-pivot
  // reach on the road grid.
  static constexpr bool TAIL3 = (KIND == KIND_BFS);
  // Source implications (reach with one query): when new bits reach the
  // vertex of source j, the sources behind them reach everything source j
  // reaches, so bit j implies them. An expansion then propagates the closure
  // of its mask under the implications known at the start of the round: only
  // true reachability facts, which let the bits of sources that reach each
  // other travel together instead of re-expanding each vertex once per bit.
  static constexpr bool IMPL = (KIND == KIND_REACH && !MULTI);

  const VgcArgs &a;
  Val *state;
  // per-wave LDS
  Val *rval, *sval;
  uint32_t *rv, *sv, *rq, *sq, *scan;
  int32_t *rb, *re;
  // Per-step record of each expanded entry (indexed by its lane), read by the
  // lanes its arcs are dealt to: the entry's first arc minus its first dealt
  // position, its value, and with several queries its query, round limit and
  // state base (recB).
  uint4 *recA;
  uint2 *recB;
  const LdsU64 *simp;   // closed implications, per workgroup (refreshed every round)
  const LdsI32 *shk;    // source hash: vertex (-1 = empty slot)
  const LdsU64 *shv;    // source hash: the bits of the sources at that vertex
  bool impl_on;
  uint32_t mstamp;  // pass number, tags the arc-owner marks of the current pass
  unsigned long long *filt;  // LDS filter: (32-bit state index << 32) | a value this wavefront saw stored there
  uint32_t fshift;           // slot = (key * golden) >> fshift
  uint32_t Q, S, ln;
  // wave-uniform
  uint32_t head, tail, scount;
  uint32_t nslot, nbuf;
  uint32_t rabs;   // absolute number of the current round (BFS window)
  uint32_t root_end;  // local-queue positions below this hold the current search's roots
  uint32_t slice_ok;  // heavy rows may be cut into slices this round
  // statistics, per wavefront and launch (32-bit: a wavefront would have to
  // scan 2^32 arcs in one launch to wrap them; widened when flushed)
  uint32_t st_expand, st_arcs, st_success, st_publish, st_overflow, st_stale, st_steps;
  uint32_t st_filt_lane;  // per lane: relaxations ruled out by a filter (summed over the wave at the end)

  __device__ __forceinline__ Wave(const VgcArgs &args, uint8_t *lds_wave) : a(args) {
    state = (Val *)a.state;
    Q = a.ring_cap;
    S = a.stage_cap;
    ln = lane_id();
    uint8_t *p = lds_wave;
    rval = (Val *)p; p += sizeof(Val) * Q;
    sval = (Val *)p; p += sizeof(Val) * S;
    rv = (uint32_t *)p; p += 4 * Q;
    sv = (uint32_t *)p; p += 4 * S;
    if (MULTI) {
      rq = (uint32_t *)p; p += 4 * Q;
      sq = (uint32_t *)p; p += 4 * S;
    } else {
      rq = sq = nullptr;
    }
    if (PF) {
      rb = (int32_t *)p; p += 4 * Q;
      re = (int32_t *)p; p += 4 * Q;
    } else {
      rb = re = nullptr;
    }
    scan = (uint32_t *)p;
    p += 64 * 4;
    recA = (uint4 *)p;
    p += 64 * 16;
    recB = (uint2 *)p;
    if (MULTI) p += 64 * 8;
    filt = (unsigned long long *)p;
    fshift = 32u - (uint32_t)__builtin_ctz(a.filt ? a.filt : 1u);
    for (uint32_t i = ln; i < a.filt; i += 64) filt[i] = ~0ull;  // key 0xFFFFFFFF: empty
    scan[ln] = 0u;  // no mark carries stamp 0
    mstamp = 0;
    wave_sync();
    head = tail = scount = 0;
    nslot = nbuf = 0;
    rabs = 0;
    root_end = 0;
    slice_ok = 0;
    qlite = nullptr;
    qlite_ok = false;
    simp = nullptr;
    shk = nullptr;
    shv = nullptr;
    impl_on = false;
    st_expand = st_arcs = st_success = st_publish = st_overflow = st_stale = st_steps = 0;
    st_filt_lane = 0;
  }

  const LdsQLite *qlite;  // LDS copy of the query table (valid when qlite_ok)
  bool qlite_ok;

  __device__ __forceinline__ int64_t sbase_of(uint32_t q) const {
    if (!MULTI) return 0;
    if (qlite_ok) return qlite[q].sbase;
    return a.qi[q].sbase;
  }

  // BFS window: distances below the limit may be expanded in this round;
  // the rest wait in the frontier (bucket width a.window per round).
  __device__ __forceinline__ uint32_t limit_of(uint32_t q) const {
    if (!DIST || a.window == 0) return 0xFFFFFFFFu;
    uint32_t r0 = 0;
    if (MULTI) r0 = qlite_ok ? qlite[q].r0 : a.qi[q].r0;
    const uint64_t lim = (uint64_t)(rabs + 1u - r0) * a.window;
    return lim > 0xFFFFFFFEull ? 0xFFFFFFFFu : (uint32_t)lim;
  }

  __device__ __forceinline__ void mark_dirty(uint32_t v, uint32_t q) {
    int64_t dbase = 0;
    uint32_t local = v;
    if (MULTI) {
      const QInfo qi = a.qi[q];
      dbase = qi.dbase;
      local = v - (uint32_t)qi.vbase;
    }
    or_ag(&a.dirty[dbase + (local >> 5)], 1u << (local & 31));
  }

  // Copy the staging buffer to the next global frontier at [base, base +
  // scount): coalesced agent-scope stores; entries past the capacity go to
  // the dirty bitmap (never dropped).
  __device__ __forceinline__ void write_stage(uint32_t base) {
    bool ovf = false;
    for (uint32_t i = ln; i < scount; i += 64) {
      const uint32_t v = sv[i];
      const Val val = sval[i];
      const uint32_t q = MULTI ? sq[i] : 0u;
      const uint32_t idx = base + i;
      if (idx >= base && idx < a.fr.cap) {
        st_ag(&a.fr.v[nbuf][idx], v);
        if (MULTI) st_ag(&a.fr.q[nbuf][idx], q);
        st_ag(&a.fr.val[nbuf][idx], (unsigned long long)val);
      } else {
        mark_dirty(v, q);
        ovf = true;
      }
    }
    const unsigned long long ob = __ballot(ovf);
    if (ob) {
      if (ln == 0) st_ag(&a.ctl->ovf[nslot], 1u);
    }
    st_overflow += __popcll(ob);
    st_publish += scount;
    scount = 0;
  }

  // Mid-round flush by one wavefront (its staging buffer is full).
  __device__ __forceinline__ void flush_stage() {
    if (scount == 0) return;
    wave_sync();
    uint32_t base = 0;
    if (ln == 0) base = add_ag(&a.ctl->cnt[nslot], scount);
    base = __shfl(base, 0);
    write_stage(base);
    wave_sync();
  }

  // End-of-round flush, collective over the workgroup: one reservation per
  // workgroup instead of one per wavefront.
  __device__ __forceinline__ void flush_stage_block(uint32_t *s_cnt, uint32_t wid, uint32_t nw) {
    wave_sync();
    if (ln == 0) s_cnt[wid] = scount;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      for (uint32_t w = 0; w < nw; w++) {
        const uint32_t c = s_cnt[w];
        s_cnt[w] = tot;
        tot += c;
      }
      s_cnt[nw] = tot ? add_ag(&a.ctl->cnt[nslot], tot) : 0u;
    }
    __syncthreads();
    const uint32_t base = s_cnt[nw] + s_cnt[wid];
    if (scount) write_stage(base);
    __syncthreads();
  }

  // Wave-collective: lanes with p append (w, q, nv) to the staging buffer.
  __device__ __forceinline__ void push_stage(bool p, uint32_t w, uint32_t q, Val nv) {
    const unsigned long long bal = __ballot(p);
    if (bal == 0) return;
    const uint32_t c = __popcll(bal);
    if (scount + c > S) flush_stage();
    if (p) {
      const uint32_t i = scount + mbcnt64(bal);
      sv[i] = w;
      sval[i] = nv;
      if (MULTI) sq[i] = q;
    }
    scount += c;
  }

  // Wave-collective push: lanes with p hand (w, q, nv) to the local queue
  // when allowed and there is room, else to the staging buffer.
  __device__ __forceinline__ void push(bool p, uint32_t w, uint32_t q, Val nv, bool ring_ok, int32_t nb = 0,
                                      int32_t ne = 0) {
    push_lim(p, w, q, nv, (DIST && a.window) ? limit_of(q) : 0xFFFFFFFFu, ring_ok, nb, ne);
  }
  // The same, with the round's limit of query q already looked up.
  __device__ __forceinline__ void push_lim(bool p, uint32_t w, uint32_t q, Val nv, uint32_t lim, bool ring_ok,
                                          int32_t nb, int32_t ne) {
    // BFS window: values at or beyond the round's limit wait for a later round
    if (DIST && a.window) {
      const bool late = p && (uint32_t)nv >= lim;
      push_stage(late, w, q, nv);
      p = p && !late;
    }
    const unsigned long long bal = __ballot(p);
    if (bal == 0) return;
    const uint32_t c = __popcll(bal);
    const uint32_t pos = mbcnt64(bal);
    if (ring_ok && (tail - head) + c <= Q) {
      if (p) {
        const uint32_t i = (tail + pos) & (Q - 1);
        rv[i] = w;
        rval[i] = nv;
        if (MULTI) rq[i] = q;
        if (PF) {
          rb[i] = nb;
          re[i] = ne;
        }
      }
      tail += c;
    } else {
      if (scount + c > S) flush_stage();
      if (p) {
        const uint32_t i = scount + pos;
        sv[i] = w;
        sval[i] = nv;
        if (MULTI) sq[i] = q;
      }
      scount += c;
    }
  }

  // Relaxation of arc (., w) carrying value val of its tail, in two halves so
  // that several relaxations per lane are in flight at once: issue() applies
  // the filters and performs the atomic; finish() records the outcome in the
  // LDS filter and reports whether the state of w changed (and the value to
  // carry).
  //  * a.test_first: a plain load first rules out relaxations that cannot
  //    change anything. It may be served by this XCD's L2 and be stale, but
  //    values only ever go down for distances and only gain bits for reach,
  //    so a stale value still proves the relaxation cannot win.
  //  * LDS filter (distances): values this wavefront saw in the state; for the
  //    same reason a remembered value <= the new one proves the atomic
  //    cannot win.
  //  * PF: the arc range of w is loaded alongside the atomic (not for a
  //    relaxation a filter ruled out: it pushes nothing).
  // A relaxation that a filter rules out keeps, as its "old" value, the value
  // that proved it (<= the offered one for distances, a superset mask for
  // reach), so finish() sees no change and the LDS filter entry it rewrites
  // is still a value the state held. Few fields, so that several can be live
  // at once without spilling.
  struct Rx {
    Val nd;   // value offered to w (distances; reach passes its mask to finish)
    Val old;  // value of w before the atomic, or the value that filtered it
    int32_t nb, ne;
  };

  __device__ __forceinline__ uint32_t filt_slot(uint32_t key) const { return (key * 0x9E3779B1u) >> fshift; }

  // ok: the lane holds a dealt arc (lanes without one pass a valid target,
  // so that every load is issued unconditionally; only the atomic is masked).
  // cur (TF): the target's state read by a plain load, issued for every pass
  // before the first atomic.
  __device__ __forceinline__ Rx relax_issue(bool ok, int64_t sb, uint32_t w, uint32_t wt, Val val, Val cur_tf) {
    Rx x;
    x.nb = x.ne = 0;
    if (DIST) {
      // SSSP distances saturate below the "unreached" value
      const uint32_t nd = (KIND == KIND_SSSP) ? (uint32_t)min((unsigned long long)val + wt, 0xFFFFFFFEull)
                                              : (uint32_t)val + 1u;
      x.nd = (Val)nd;
      uint32_t *p = (uint32_t *)&state[sb + w];
      // straight-line: each filter narrows one predicate, then a single
      // masked region performs the atomic
      bool go = ok;
      uint32_t old = 0xFFFFFFFFu;
      if (TF) {
        const uint32_t cur = (uint32_t)cur_tf;
        go = go && cur > nd;
        old = cur;
      }
      if (a.filt) {  // wave-uniform
        const uint32_t key = (uint32_t)(sb + (int64_t)w);
        const unsigned long long e = filt[filt_slot(key)];
        const bool hit = (uint32_t)(e >> 32) == key && (uint32_t)e <= nd;
        old = (go && hit) ? (uint32_t)e : old;
        go = go && !hit;
      }
      st_filt_lane += (ok && !go) ? 1u : 0u;
      if (go) {
        if (PF) {  // only for relaxations that reach the atomic
          x.nb = a.off[w];
          x.ne = a.off[w + 1];
        }
        old = min_ag(p, nd);
      }
      x.old = (Val)old;
    } else {
      unsigned long long *p = (unsigned long long *)&state[sb + w];
      const unsigned long long m = (unsigned long long)val;
      bool go = ok;
      unsigned long long old = 0;
      if (TF) {
        const unsigned long long cur = (unsigned long long)cur_tf;
        go = go && (cur & m) != m;
        old = cur;
      }
      st_filt_lane += (ok && !go) ? 1u : 0u;
      if (go) {
        if (PF) {
          x.nb = a.off[w];
          x.ne = a.off[w + 1];
        }
        old = or_ag(p, m);
      }
      x.old = (Val)old;
    }
    return x;
  }

  // Only for a lane whose relax_issue ran (a valid arc); offered is the value
  // that relax_issue got (read for reach, whose records do not keep it).
  // key: the low 32 bits of w's state index (the LDS filter's key).
  __device__ __forceinline__ bool relax_finish(const Rx &x, uint32_t key, Val offered, Val &nv) {
    if (DIST) {
      nv = x.nd;
      if (a.filt) {
        filt[filt_slot(key)] =
            ((unsigned long long)key << 32) | (unsigned long long)min((uint32_t)x.old, (uint32_t)x.nd);
      }
      return (uint32_t)x.nd < (uint32_t)x.old;
    }
    nv = (Val)((unsigned long long)x.old | (unsigned long long)offered);
    return nv != x.old;
  }

  // Heavy rows: a lane whose row has more than a.heavy arcs hands them to the
  // next round as slices of a.heavy arcs (one wavefront per slice there)
  // instead of scanning them all with this one wavefront. One reservation
  // per wavefront; slices past the buffer's capacity are not written and the
  // lane keeps those arcs ([b, e) shrinks to them), so every reserved index
  // below the capacity holds a slice.
  __device__ __forceinline__ void cut_heavy(bool act, uint32_t v, uint32_t q, Val val, int32_t &b, int32_t &e) {
    const bool hv = act && (uint32_t)(e - b) > a.heavy;
    if (!__ballot(hv)) return;
    const uint32_t k = hv ? ((uint32_t)(e - b) + a.heavy - 1) / a.heavy : 0u;
    const uint32_t incl = wave_incl_sum_dpp(k, ln);
    const uint32_t tot = lane_read(incl, 63);
    uint32_t base = 0;
    if (ln == 0) base = add_ag(&a.ctl->hcnt[nslot], tot);
    base = __shfl(base, 0);
    if (hv) {
      const uint32_t s0 = base + incl - k;
      const uint32_t fit = s0 >= a.hcap ? 0u : min(k, a.hcap - s0);
      for (uint32_t i = 0; i < fit; i++) {
        const uint32_t idx = s0 + i;
        st_ag(&a.hv[nbuf][idx], v);
        if (MULTI) st_ag(&a.hq[nbuf][idx], q);
        st_ag(&a.hval[nbuf][idx], (unsigned long long)val);
        st_ag(&a.hb[nbuf][idx], b + (int32_t)(i * a.heavy));
      }
      b = min(e, b + (int32_t)(fit * a.heavy));
    }
  }

  // Slices cut last round: slice s goes to wavefront s mod total; its arcs
  // are relaxed across the wavefront and a local search continues from what
  // they reached.
  __device__ __forceinline__ void process_heavy(uint32_t cbuf, uint32_t nheavy, uint32_t gw, uint32_t total) {
    for (uint32_t s = gw; s < nheavy; s += total) {
      const bool has = ln == 0;
      uint32_t v = 0, q = 0;
      Val val = 0;
      int32_t b = 0, e = 0;
      if (has) {
        v = ld_ag(&a.hv[cbuf][s]);
        if (MULTI) q = ld_ag(&a.hq[cbuf][s]);
        val = (Val)ld_ag(&a.hval[cbuf][s]);
        b = ld_ag(&a.hb[cbuf][s]);
        e = min(a.off[v + 1], b + (int32_t)a.heavy);
      }
      head = tail = 0;
      root_end = 0;
      const uint32_t ne = expand(has, v, q, val, true, b, e, true, true);
      if (ne) local_search(a.tau);
      head = tail = 0;
    }
  }

  // Arc dealing: the lane that owns arc j0 + ln (see wave_arc_owner), with
  // marks tagged by the pass number so that the mark words need no clearing
  // between passes.
  __device__ __forceinline__ uint32_t arc_owner(uint32_t excl, uint32_t deg, uint32_t j0) {
    if (++mstamp == (1u << 25)) {  // wave-uniform; tags wrap after 2^25 - 1 passes
      scan[ln] = 0u;
      mstamp = 1;
    }
    if (deg != 0u && excl < j0 + 64u && excl + deg > j0) scan[excl > j0 ? excl - j0 : 0u] = (mstamp << 7) | (ln + 1u);
    wave_sync();
    const uint32_t m = scan[ln];
    wave_sync();
    return wave_incl_max_dpp((m >> 7) == mstamp ? (m & 127u) : 0u, ln) - 1u;
  }

  // NP consecutive 64-arc passes starting at arc j0 (every one holds at least
  // one arc), in straight-line code: every lane loads a target in every pass
  // (lanes past the last arc repeat it), so the loads of all passes are in
  // flight together and each relaxation waits only for its own target; then
  // the atomics of all passes, then their pushes. Returns the successes.
  template <int NP>
  __device__ __forceinline__ uint32_t passes(uint32_t j0, uint32_t total, uint32_t excl, uint32_t deg, uint32_t lim1,
                                             bool ring_ok) {
    uint32_t w[NP], wt[NP], lim[NP], qo[NP];
    Val vo[NP];
    int64_t sbo[NP];
    bool okl[NP];
#pragma unroll
    for (int r = 0; r < NP; r++) {
      const uint32_t jr = j0 + 64u * (uint32_t)r;
      const uint32_t owner = arc_owner(excl, deg, jr);
      const uint32_t ai = jr + ln;
      okl[r] = ai < total;
      uint32_t bx;
      if (MULTI) {
        const uint4 R = recA[owner];
        const uint2 S = recB[owner];
        bx = R.x;
        if (DIST) {
          vo[r] = (Val)R.y;
          lim[r] = R.z;
          qo[r] = R.w;
        } else {
          qo[r] = R.y;
          vo[r] = (Val)(((unsigned long long)R.w << 32) | R.z);
          lim[r] = 0xFFFFFFFFu;
        }
        sbo[r] = (int64_t)(((unsigned long long)S.y << 32) | S.x);
      } else {
        if (DIST) {
          const uint2 R = ((const uint2 *)recA)[owner];
          bx = R.x;
          vo[r] = (Val)R.y;
        } else {
          const uint4 R = recA[owner];
          bx = R.x;
          vo[r] = (Val)(((unsigned long long)R.w << 32) | R.z);
        }
        lim[r] = lim1;
        qo[r] = 0;
        sbo[r] = 0;
      }
      const int32_t arc = (int32_t)(bx + min(ai, total - 1u));
      w[r] = (uint32_t)a.tgt[arc];
      wt[r] = (KIND == KIND_SSSP) ? a.wgt[arc] : 0u;
    }
    Val cur[NP];
#pragma unroll
    for (int r = 0; r < NP; r++) cur[r] = TF ? *(const Val *)&state[sbo[r] + w[r]] : (Val)0;
    Rx x[NP];
#pragma unroll
    for (int r = 0; r < NP; r++) x[r] = relax_issue(okl[r], sbo[r], w[r], wt[r], vo[r], cur[r]);
    uint32_t ns = 0;
#pragma unroll
    for (int r = 0; r < NP; r++) {
      Val nv = 0;
      const bool ok = okl[r] && relax_finish(x[r], (uint32_t)sbo[r] + w[r], vo[r], nv);
      ns += __popcll(__ballot(ok));
      if (IMPL && impl_on && ok) {
        // new bits reached w: if w is a source's vertex, record them
        uint32_t h = src_slot(w[r]);
        for (int t = 0; t < SRC_SLOTS; t++) {
          const int32_t key = shk[h];
          if (key == (int32_t)w[r]) {
            unsigned long long bits = shv[h];
            while (bits) {
              or_ag(&a.imp[__builtin_ctzll(bits)], (unsigned long long)nv);
              bits &= bits - 1;
            }
            break;
          }
          if (key < 0) break;
          h = (h + 1) & (SRC_SLOTS - 1);
        }
      }
      push_lim(ok, w[r], qo[r], nv, lim[r], ring_ok, x[r].nb, x[r].ne);
    }
    return ns;
  }

  // Expand the active lanes' entries: scan out-arcs, relax, push successes.
  // Returns the number of entries expanded (not stale). Every vertex's arcs
  // are dealt out across the wavefront 64 at a time (consecutive lanes take
  // consecutive arcs, so one memory instruction touches few cache lines).
  __device__ __forceinline__ uint32_t expand(bool act, uint32_t v, uint32_t q, Val val, bool ring_ok, int32_t b = 0,
                                             int32_t e = 0, bool have_range = false, bool check_stale = true) {
    const int64_t sb = MULTI ? sbase_of(act ? q : 0u) : 0;
    if (!have_range) {  // inactive lanes read row 0, so the loads need no branch
      b = a.off[act ? v : 0u];
      e = a.off[(act ? v : 0u) + 1];
    }
    if (DIST && act && check_stale) {
      // a smaller distance is already known: another entry carries it
      const uint32_t cur = ld_ag((uint32_t *)&state[sb + v]);
      if (cur < (uint32_t)val) act = false;
    }
    const unsigned long long actb = __ballot(act);
    const uint32_t nexp = __popcll(actb);
    st_expand += nexp;
    if (slice_ok) cut_heavy(act, v, q, val, b, e);
    const uint32_t deg = act ? (uint32_t)(e - b) : 0u;
    // scans by DPP row shifts: no LDS round trip on the step's critical path
    const uint32_t incl = wave_incl_sum_dpp(deg, ln);
    const uint32_t total = lane_read(incl, 63);
    if (total == 0) return nexp;
    const uint32_t excl = incl - deg;
    if (deg != 0u) {
      const uint32_t bx = (uint32_t)b - excl;
      if (MULTI) {
        if (DIST)
          recA[ln] = make_uint4(bx, (uint32_t)val, a.window ? limit_of(q) : 0xFFFFFFFFu, q);
        else
          recA[ln] = make_uint4(bx, q, (uint32_t)val, (uint32_t)((unsigned long long)val >> 32));
        recB[ln] = make_uint2((uint32_t)sb, (uint32_t)((unsigned long long)sb >> 32));
      } else if (DIST) {
        ((uint2 *)recA)[ln] = make_uint2(bx, (uint32_t)val);
      } else {
        unsigned long long m = (unsigned long long)val;
        if (IMPL && impl_on) {
          // the closure of the entry's bits: a bit already covered needs no
          // lookup (the table is transitively closed)
          unsigned long long M = 0, rem = m;
          while (rem) {
            M |= simp[__builtin_ctzll(rem)];
            rem &= ~M;
          }
          if (M != m) {  // the implied bits hold at v too
            or_ag((unsigned long long *)&state[v], M);
            m = M;
          }
        }
        recA[ln] = make_uint4(bx, 0u, (uint32_t)m, (uint32_t)(m >> 32));
      }
    }
    wave_sync();
    // one query: the round's limit is the same for every entry
    const uint32_t lim1 = (!MULTI && DIST && a.window) ? limit_of(0) : 0xFFFFFFFFu;
    uint32_t nsucc = 0;
    for (uint32_t j0 = 0; j0 < total;) {  // wave-uniform
      const uint32_t left = (total - j0 + 63u) >> 6;
      if (RB >= 5 && left >= 5) {
        nsucc += passes<(RB >= 5 ? 5 : 1)>(j0, total, excl, deg, lim1, ring_ok);
        j0 += 320;
      } else if (RB >= 4 && left >= 4) {
        nsucc += passes<(RB >= 4 ? 4 : 1)>(j0, total, excl, deg, lim1, ring_ok);
        j0 += 256;
      } else if (TAIL3 && left == 3) {
        nsucc += passes<(RB >= 3 ? 3 : 1)>(j0, total, excl, deg, lim1, ring_ok);
        j0 += 192;
      } else if (RB >= 2 && left >= 2) {
        nsucc += passes<(RB >= 2 ? 2 : 1)>(j0, total, excl, deg, lim1, ring_ok);
        j0 += 128;
      } else {
        nsucc += passes<1>(j0, total, excl, deg, lim1, ring_ok);
        j0 += 64;
      }
    }
    wave_sync();
    st_success += nsucc;
    st_arcs += total;
    return nexp;
  }

  // Pop up to 64 entries from the local queue and expand them.
  __device__ __forceinline__ uint32_t step(bool ring_ok) {
    const uint32_t avail = tail - head;
    const uint32_t k = min(avail, 64u);
    const uint32_t idx = FIFO ? (head + ln) : (tail - k + ln);
    const bool act = ln < k;
    uint32_t v = 0, q = 0;
    Val val = 0;
    int32_t b = 0, e = 0;
    if (act) {
      const uint32_t s = idx & (Q - 1);
      v = rv[s];
      val = rval[s];
      if (MULTI) q = rq[s];
      if (PF) {
        b = rb[s];
        e = re[s];
      }
    }
    wave_sync();
    if (FIFO)
      head += k;
    else
      tail -= k;
    // With the window, entries pushed by this very search are rarely stale;
    // the coherent re-read of the distance is kept for roots and for the
    // windowless schedule, where overlapping searches make staleness common.
    const bool chk = (a.window == 0) || (idx < root_end);
    st_steps += k ? 1u : 0u;
    const uint32_t ne = expand(act, v, q, val, ring_ok, b, e, PF, chk);
    st_stale += (uint32_t)__popcll(__ballot(act)) - ne;
    return ne;
  }

  // Move whatever is left in the local queue to the staging buffer.
  __device__ __forceinline__ void spill_ring() {
    while (tail != head) {
      const uint32_t k = min(tail - head, 64u);
      const bool act = ln < k;
      uint32_t v = 0, q = 0;
      Val val = 0;
      if (act) {
        const uint32_t s = (head + ln) & (Q - 1);
        v = rv[s];
        val = rval[s];
        if (MULTI) q = rq[s];
      }
      wave_sync();
      head += k;
      push(act, v, q, val, false);
    }
    head = tail = 0;
  }

  // One local search: the ring holds the roots; expand until the budget of
  // expanded vertices is spent or nothing is left, then publish the rest.
  __device__ __forceinline__ void local_search(uint32_t budget) {
    uint32_t expanded = 0;
    while (tail != head) {
      if (expanded >= budget) {
        spill_ring();
        break;
      }
      expanded += step(true);
    }
    head = tail = 0;
  }

  // Append the lanes' roots to the (not yet wrapped) local queue.
  __device__ __forceinline__ void append_roots(bool has, uint32_t v, uint32_t q, Val val) {
    const unsigned long long bal = __ballot(has);
    const uint32_t pos = tail + mbcnt64(bal);
    if (has) {
      rv[pos] = v;
      rval[pos] = val;
      if (MULTI) rq[pos] = q;
      if (PF) {
        rb[pos] = a.off[v];
        re[pos] = a.off[v + 1];
      }
    }
    wave_sync();
    tail += __popcll(bal);
  }

  __device__ __forceinline__ void load_roots(bool has, uint32_t v, uint32_t q, Val val) {
    const unsigned long long bal = __ballot(has);
    const uint32_t pos = mbcnt64(bal);
    if (has) {
      rv[pos] = v;
      rval[pos] = val;
      if (MULTI) rq[pos] = q;
      if (PF) {
        rb[pos] = a.off[v];
        re[pos] = a.off[v + 1];
      }
    }
    wave_sync();
    head = 0;
    tail = __popcll(bal);
  }

  // Frontier entries are dealt out in chunks of `chunk` consecutive entries.
  // Consecutive entries were published together by one local search, so a
  // wavefront's roots are close in the graph; a chunk may hold more roots than
  // lanes (up to half the ring): they all start one local search, which then
  // advances a wide front per step. The chunks are split into 8 contiguous
  // ranges, one per XCD (gw numbers wavefronts so that each XCD holds a
  // contiguous range of them). A wavefront first takes chunk lo + i of its
  // XCD's range (i = its index inside the XCD), then claims further chunks
  // of that range from the XCD's counter until the range is used up, so
  // wavefronts whose searches end early take over the remaining work.
  __device__ __forceinline__ void run_chunk(uint32_t cbuf, uint32_t nproc, uint32_t chunk, uint32_t c) {
    const uint32_t base = c * chunk;
    const uint32_t cnt = min(chunk, nproc - base);
    head = tail = 0;
    for (uint32_t j = 0; j < cnt; j += 64) {
      bool has = j + ln < cnt;
      uint32_t v = 0, q = 0;
      Val val = 0;
      if (has) {
        v = ld_ag(&a.fr.v[cbuf][base + j + ln]);
        if (MULTI) q = ld_ag(&a.fr.q[cbuf][base + j + ln]);
        val = (Val)ld_ag(&a.fr.val[cbuf][base + j + ln]);
      }
      if (DIST && a.window) {  // roots beyond the window wait for a later round
        const bool defer = has && (uint32_t)val >= limit_of(q);
        push_stage(defer, v, q, val);
        has = has && !defer;
      }
      append_roots(has, v, q, val);
    }
    const uint32_t nroots = tail - head;
    if (nroots == 0) return;
    root_end = tail;
    local_search(a.tau * nroots);
  }

  __device__ __forceinline__ void process_frontier(uint32_t cbuf, uint32_t nproc, uint32_t chunk, uint32_t gw,
                                                   uint32_t total, uint32_t cslot) {
    const uint32_t nchunks = (nproc + chunk - 1) / chunk;
    const uint32_t groups = (total % 8u == 0) ? 8u : 1u;
    const uint32_t per = total / groups;
    const uint32_t x = gw / per, i = gw % per;
    const uint32_t lo = (uint32_t)((uint64_t)nchunks * x / groups);
    const uint32_t hi = (uint32_t)((uint64_t)nchunks * (x + 1) / groups);
    uint32_t c = lo + i;
    while (c < hi) {
      run_chunk(cbuf, nproc, chunk, c);
      if (hi - lo <= per) break;  // every chunk of the range was dealt statically
      uint32_t k = 0;
      if (ln == 0) k = add_ag(&a.ctl->claim[cslot][x], 1u);
      k = __shfl(k, 0);
      c = lo + per + k;
    }
  }

  // Re-expand vertices whose frontier entries overflowed last round.
  __device__ __forceinline__ void process_dirty(uint32_t gw, uint32_t total) {
    for (int64_t base = (int64_t)gw * 64; base < a.dirty_words; base += (int64_t)total * 64) {
      // virtual word index -> (query, word of that query's bitmap)
      const int64_t widx = (int64_t)base + ln;
      uint32_t q = 0;
      int64_t lw = widx;
      if (MULTI && widx < a.dirty_words) {
        int32_t lo = 0, hi = a.nq - 1;  // last q with qword[q] <= widx
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if (a.qword[mid] <= widx) lo = mid;
          else hi = mid - 1;
        }
        q = (uint32_t)lo;
        lw = widx - a.qword[q];
      }
      uint32_t word = 0;
      if (widx < a.dirty_words) {
        uint32_t *wp = &a.dirty[(MULTI ? a.qi[q].dbase : 0) + lw];
        word = ld_ag(wp);
        if (word) word = xchg_ag(wp, 0u);
      }
      while (__ballot(word != 0)) {
        const bool has = word != 0;
        uint32_t v = 0;
        Val val = 0;
        if (has) {
          const uint32_t bit = __builtin_ctz(word);
          word &= word - 1;
          int32_t vbase = 0;
          int64_t sb = 0;
          if (MULTI) {
            vbase = a.qi[q].vbase;
            sb = a.qi[q].sbase;
          }
          v = (uint32_t)vbase + (uint32_t)(lw * 32 + bit);
          val = ld_ag(&state[sb + v]);
        }
        bool go = has;
        if (DIST && a.window) {
          const bool defer = has && (uint32_t)val >= limit_of(q);
          push_stage(defer, v, q, val);
          go = has && !defer;
        }
        const uint32_t c = __popcll(__ballot(go));
        if (c == 0) continue;
        load_roots(go, v, q, val);
        root_end = tail;
        local_search(a.tau * c);
      }
    }
  }

  __device__ __forceinline__ void flush_stats() {
    unsigned long long st_filtered = st_filt_lane;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) st_filtered += shfl64(st_filtered, ln ^ (uint32_t)d);
    if (ln == 0) {
      const unsigned long long vals[ST_COUNT] = {st_expand,   st_arcs,  st_success, st_publish,
                                                 st_overflow, st_stale, st_steps,   st_filtered};
#pragma clang loop unroll(full)
      for (int i = 0; i < ST_COUNT; i++)
        if (vals[i]) add_ag(&a.ctl->stats[i], vals[i]);
    }
  }
};

template <int KIND, bool MULTI, bool PF, bool TF>
__global__ void __launch_bounds__(1024) vgc_kernel(VgcArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ RoundHdr hdr;
  __shared__ uint32_t s_cnt[17];
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t wid = threadIdx.x >> 6;
  const size_t per_wave = vgc_lds_bytes(KIND, MULTI, PF, 1, a.ring_cap, a.stage_cap, a.filt);
  Wave<KIND, MULTI, PF, TF> wv(a, smem + per_wave * wid);
  __shared__ QLite qlite[MULTI ? QLITE : 1];
  constexpr bool IMPL = Wave<KIND, MULTI, PF, TF>::IMPL;
  __shared__ unsigned long long s_imp[IMPL ? 64 : 1];
  __shared__ int32_t s_hk[IMPL ? SRC_SLOTS : 1];
  __shared__ unsigned long long s_hv[IMPL ? SRC_SLOTS : 1];
  const bool impl = IMPL && a.imp != nullptr;
  if (impl) {
    if (threadIdx.x < SRC_SLOTS) s_hk[threadIdx.x] = -1;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int j = 0; j < 64; j++) {
        const int32_t v = a.srcv[j];
        if (v < 0) continue;
        uint32_t h = src_slot((uint32_t)v);
        while (s_hk[h] >= 0 && s_hk[h] != v) h = (h + 1) & (SRC_SLOTS - 1);
        if (s_hk[h] < 0) {
          s_hk[h] = v;
          s_hv[h] = 0ull;
        }
        s_hv[h] |= 1ull << j;
      }
    }
    wv.simp = (const LdsU64 *)s_imp;
    wv.shk = (const LdsI32 *)s_hk;
    wv.shv = (const LdsU64 *)s_hv;
    wv.impl_on = true;
  }
  if (MULTI && a.nq <= QLITE) {
    for (int i = threadIdx.x; i < a.nq; i += blockDim.x) {
      qlite[i].sbase = a.qi[i].sbase;
      qlite[i].r0 = a.qi[i].r0;
      qlite[i].pad = 0;
    }
    wv.qlite = (const LdsQLite *)qlite;
    wv.qlite_ok = true;
  }
  const uint32_t total_waves = gridDim.x * nw;
  // XCD-aware numbering: workgroups are dispatched round-robin over the 8
  // XCDs; give each XCD a contiguous range of logical workgroups.
  uint32_t lblock = blockIdx.x;
  if ((gridDim.x & 7u) == 0) lblock = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const uint32_t gw = lblock * nw + wid;
  const long long deadline = wall_clock64() + a.timeout_ticks;
  uint32_t epoch = 0;
  uint32_t cbuf = a.start_buf;
  if (threadIdx.x == 0) {
    hdr.ncur = ld_ag(&a.ctl->cnt[0]);
    hdr.ovf = ld_ag(&a.ctl->ovf[0]);
    hdr.abort = 0;
  }
  __syncthreads();
  uint32_t ncur = hdr.ncur, ovf = hdr.ovf;
  uint32_t maxf = 0;
  uint32_t r = 0;
  uint32_t nheavy = 0;
  bool yielded = false;  // the previous round saw a yield request (the same in every workgroup)
  uint32_t ysnap = 0;    // workgroup 0, thread 0: the yield word as read at the start of the round
  for (; r < a.max_rounds; ++r) {
    if (ncur == 0 && ovf == 0 && nheavy == 0) break;
    // a yield ends the launch here unless slices cut last round are pending
    if (yielded && nheavy == 0) break;
    maxf = max(maxf, ncur);
    const uint32_t nslot = (r + 1) % 3, fslot = (r + 2) % 3;
    if (blockIdx.x == 0 && threadIdx.x < 8) st_ag(&a.ctl->claim[fslot][threadIdx.x], 0u);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st_ag(&a.ctl->cnt[fslot], 0u);
      st_ag(&a.ctl->ovf[fslot], 0u);
      st_ag(&a.ctl->hcnt[fslot], 0u);
      st_ag(&a.ctl->yld[fslot], 0u);
      // issued now, used before the barrier: the host read overlaps the round
      if (a.yield) ysnap = __hip_atomic_load(a.yield, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (impl) {
      // implications recorded so far, closed transitively (Warshall, one row
      // per lane of the first wavefront, rows exchanged by lane reads)
      if (threadIdx.x < 64) {
        unsigned long long x = ld_ag(&a.imp[threadIdx.x]) | (1ull << threadIdx.x);
        for (int k = 0; k < 64; k++) {
          const unsigned long long yk = ((unsigned long long)lane_read((uint32_t)(x >> 32), k) << 32) |
                                        lane_read((uint32_t)x, k);
          if ((x >> k) & 1ull) x |= yk;
        }
        s_imp[threadIdx.x] = x;
      }
      __syncthreads();
    }
    wv.nslot = nslot;
    wv.nbuf = cbuf ^ 1u;
    wv.rabs = a.round_base + r;
    // no slices in a launch's last allowed round: nothing may be left in the
    // slice buffer when the launch returns
    wv.slice_ok = (a.heavy != 0 && r + 1 < a.max_rounds) ? 1u : 0u;
    if (nheavy) wv.process_heavy(cbuf, min(nheavy, a.hcap), gw, total_waves);
    if (ovf) wv.process_dirty(gw, total_waves);
    const uint32_t nproc = min(ncur, a.fr.cap);
    const uint64_t slots = (uint64_t)total_waves * max(a.chunks_per_wave, 1u);
    uint32_t chunk = (uint32_t)((nproc + slots - 1) / slots);
    chunk = min(max(chunk, max(a.min_chunk, 1u)), a.ring_cap / 2);
    wv.process_frontier(cbuf, nproc, chunk, gw, total_waves, r % 3);
    wv.flush_stage_block(s_cnt, wid, nw);
    if (a.yield && blockIdx.x == 0 && threadIdx.x == 0 && ysnap != a.yield_base) st_ag(&a.ctl->yld[nslot], 1u);
    grid_barrier(a.ctl, epoch, deadline, nslot, &hdr);
    if (hdr.abort) break;
    ncur = hdr.ncur;
    ovf = hdr.ovf;
    nheavy = hdr.nheavy;
    yielded = a.yield != nullptr && hdr.yld != 0u;
    cbuf ^= 1u;
  }
  wv.flush_stats();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st_ag(&a.ctl->rounds, r);
    st_ag(&a.ctl->final_cnt, ncur);
    st_ag(&a.ctl->final_ovf, ovf);
    st_ag(&a.ctl->final_buf, cbuf);
    max_ag(&a.ctl->max_frontier, maxf);
  }
}

template <int KIND>
__global__ void seed_kernel(VgcArgs a, const SeedEnt *seeds, uint32_t nseed, uint32_t start_cnt, uint32_t start_ovf) {
  using Val = typename ValT<KIND>::T;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t base = min(start_cnt, a.fr.cap);
  if (i == 0) {
    st_ag(&a.ctl->cnt[0], base + nseed);
    if (start_ovf) or_ag(&a.ctl->ovf[0], 1u);
  }
  if (i < nseed) {
    const SeedEnt s = seeds[i];
    const QInfo qi = a.qi[s.q];
    Val *state = (Val *)a.state;
    if (KIND != KIND_REACH)
      min_ag((uint32_t *)&state[qi.sbase + s.v], (uint32_t)s.val);
    else
      or_ag((unsigned long long *)&state[qi.sbase + s.v], (unsigned long long)s.val);
    const uint32_t pos = base + i;
    if (pos < a.fr.cap) {
      st_ag(&a.fr.v[a.start_buf][pos], s.v);
      if (a.fr.q[a.start_buf]) st_ag(&a.fr.q[a.start_buf][pos], s.q);
      st_ag(&a.fr.val[a.start_buf][pos], s.val);
    } else {
      const uint32_t local = s.v - (uint32_t)qi.vbase;
      or_ag(&a.dirty[qi.dbase + (local >> 5)], 1u << (local & 31));
      or_ag(&a.ctl->ovf[0], 1u);
    }
  }
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t val) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t n4 = n / 4;
  uint4 *p4 = (uint4 *)p;
  const bool aligned = (((uintptr_t)p) & 15) == 0;
  if (aligned) {
    const uint4 v = make_uint4(val, val, val, val);
    for (uint64_t j = i; j < n4; j += stride) p4[j] = v;
    for (uint64_t j = n4 * 4 + i; j < n; j += stride) p[j] = val;
  } else {
    for (uint64_t j = i; j < n; j += stride) p[j] = val;
  }
}

__global__ void fill_u64_kernel(unsigned long long *p, uint64_t n, unsigned long long val) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) p[j] = val;
}

static int fill_grid(uint64_t n) {
  uint64_t blocks = (n / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  return (int)blocks;
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t val, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, val);
  return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long val, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(fill_grid(4 * n)), dim3(256), 0, s, p, n, val);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) sum_u32_kernel(const uint32_t *p, uint64_t n, unsigned long long *out) {
  unsigned long long s = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) s += p[i];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += shfl64(s, (int)(lane_id() ^ (uint32_t)d));
  if (lane_id() == 0 && s) add_ag(out, s);
}

hipError_t launch_sum_u32(const uint32_t *p, uint64_t n, unsigned long long *out, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(sum_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, out);
  return hipGetLastError();
}

hipError_t launch_seed(int kind, const VgcArgs &a, const SeedEnt *seeds, uint32_t nseed, uint32_t start_cnt,
                       uint32_t start_ovf, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  const int grid = (int)((nseed + 255) / 256) > 0 ? (int)((nseed + 255) / 256) : 1;
  if (kind == KIND_BFS)
    hipLaunchKernelGGL(seed_kernel<KIND_BFS>, dim3(grid), dim3(256), 0, s, a, seeds, nseed, start_cnt, start_ovf);
  else if (kind == KIND_SSSP)
    hipLaunchKernelGGL(seed_kernel<KIND_SSSP>, dim3(grid), dim3(256), 0, s, a, seeds, nseed, start_cnt, start_ovf);
  else
    hipLaunchKernelGGL(seed_kernel<KIND_REACH>, dim3(grid), dim3(256), 0, s, a, seeds, nseed, start_cnt, start_ovf);
  return hipGetLastError();
}

template <int KIND, bool MULTI>
static const void *vgc_variant(bool pf, bool tf) {
  if (pf) return tf ? (const void *)vgc_kernel<KIND, MULTI, true, true> : (const void *)vgc_kernel<KIND, MULTI, true, false>;
  return tf ? (const void *)vgc_kernel<KIND, MULTI, false, true> : (const void *)vgc_kernel<KIND, MULTI, false, false>;
}

const void *vgc_kernel_ptr(int kind, bool multi, bool pf, bool tf) {
  if (kind == KIND_SSSP) {  // one query per launch
    if (multi) return nullptr;
    return vgc_variant<KIND_SSSP, false>(pf, tf);
  }
  if (kind == KIND_BFS) return multi ? vgc_variant<KIND_BFS, true>(pf, tf) : vgc_variant<KIND_BFS, false>(pf, tf);
  return multi ? vgc_variant<KIND_REACH, true>(pf, tf) : vgc_variant<KIND_REACH, false>(pf, tf);
}

hipError_t launch_vgc(int kind, bool multi, bool pf, const VgcArgs &a, int grid, int block, size_t lds,
                      bool cooperative, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  const void *fn = vgc_kernel_ptr(kind, multi, pf, a.test_first != 0);
  if (!fn) return hipErrorInvalidDeviceFunction;
  VgcArgs copy = a;
  void *args[] = {&copy};
  if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, (unsigned)lds, s);
  return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, s);
}

// ------------------------------------------------------ plain (VGC off) --
// One BFS level per launch: wavefronts take 64 frontier vertices each and
// deal their arcs out over the lanes; atomicCAS from "unreached" to level+1
// admits each vertex exactly once (the standard parallel BFS condition of
// the frontier framework).

template <int KIND>
__global__ void __launch_bounds__(256) plain_level_kernel(const int32_t *off, const int32_t *tgt, void *statev,
                                                          uint32_t *stamp, const uint32_t *cur, uint32_t ncur,
                                                          uint32_t *nxt, uint32_t *cnt, uint32_t level, Ctl *ctl) {
  __shared__ uint32_t scan_s[4][64];
  const uint32_t ln = lane_id();
  const uint32_t wid = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * (blockDim.x >> 6) + wid;
  const uint32_t nw = gridDim.x * (blockDim.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[(level + 2) % 3] = 0;
  uint32_t *nxt_cnt = &cnt[(level + 1) % 3];
  unsigned long long arcs = 0, succ = 0;
  for (uint32_t base = gw * 64; base < ncur; base += nw * 64) {
    const bool act = base + ln < ncur;
    uint32_t v = 0;
    int32_t b = 0, e = 0;
    unsigned long long m = 0;
    if (act) {
      v = cur[base + ln];
      b = off[v];
      e = off[v + 1];
      if (KIND == KIND_REACH) m = ld_ag(&((unsigned long long *)statev)[v]);
    }
    const uint32_t deg = act ? (uint32_t)(e - b) : 0u;
    const uint32_t incl = wave_incl_sum_dpp(deg, ln);
    const uint32_t total = lane_read(incl, 63);
    const uint32_t excl = incl - deg;
    arcs += total;
    for (uint32_t j = 0; j < total; j += 64) {
      const uint32_t ai = j + ln;
      // the lane that owns arc ai, and its first arc minus its first dealt position
      const int owner = (int)wave_arc_owner(excl, deg, j, scan_s[wid], ln);
      const uint32_t bx = (uint32_t)__shfl((int)((uint32_t)b - excl), owner);
      const unsigned long long mo = (KIND == KIND_REACH) ? shfl64(m, owner) : 0ull;
      bool ok = false;
      uint32_t w = 0;
      if (ai < total) {
        w = (uint32_t)tgt[(int32_t)(bx + ai)];
        if (KIND == KIND_BFS) {
          ok = cas_ag(&((uint32_t *)statev)[w], INF32, level + 1) == INF32;
        } else {
          const unsigned long long old = or_ag(&((unsigned long long *)statev)[w], mo);
          if ((old | mo) != old) ok = xchg_ag(&stamp[w], level + 1) != level + 1;
        }
      }
      const unsigned long long bal = __ballot(ok);
      if (bal) {
        uint32_t at = 0;
        if (ln == 0) at = add_ag(nxt_cnt, (uint32_t)__popcll(bal));
        at = __shfl(at, 0);
        if (ok) nxt[at + mbcnt64(bal)] = w;
        succ += __popcll(bal);
      }
    }
    wave_sync();
  }
  if (ln == 0) {
    if (arcs) add_ag(&ctl->stats[ST_ARCS], arcs);
    if (succ) add_ag(&ctl->stats[ST_SUCCESS], succ);
  }
}

hipError_t launch_plain_bfs_level(const int32_t *off, const int32_t *tgt, uint32_t *dist, const uint32_t *cur,
                                  uint32_t ncur, uint32_t *nxt, uint32_t *cnt, uint32_t level, Ctl *ctl,
                                  hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  uint32_t waves = (ncur + 63) / 64;
  uint32_t blocks = (waves + 3) / 4;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(plain_level_kernel<KIND_BFS>, dim3(blocks), dim3(256), 0, s, off, tgt, (void *)dist,
                     (uint32_t *)nullptr, cur, ncur, nxt, cnt, level, ctl);
  return hipGetLastError();
}

hipError_t launch_plain_reach_level(const int32_t *off, const int32_t *tgt, unsigned long long *mask,
                                    uint32_t *stamp, const uint32_t *cur, uint32_t ncur, uint32_t *nxt,
                                    uint32_t *cnt, uint32_t level, Ctl *ctl, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  uint32_t waves = (ncur + 63) / 64;
  uint32_t blocks = (waves + 3) / 4;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(plain_level_kernel<KIND_REACH>, dim3(blocks), dim3(256), 0, s, off, tgt, (void *)mask, stamp,
                     cur, ncur, nxt, cnt, level, ctl);
  return hipGetLastError();
}

// Level-0 frontier: BFS sets dist[src] = 0; reach ORs bit i into
// mask[srcs[i]]. A vertex enters the frontier once (stamp 0 for reach).
__global__ void plain_seed_kernel(int kind, void *state, uint32_t *frontier, uint32_t *cnt, uint32_t *stamp,
                                  const uint32_t *srcs, const unsigned long long *vals, uint32_t nsrc) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsrc) return;
  const uint32_t v = srcs[i];
  bool push;
  if (kind == KIND_BFS) {
    push = cas_ag(&((uint32_t *)state)[v], INF32, 0u) == INF32;
  } else {
    or_ag(&((unsigned long long *)state)[v], vals[i]);
    push = xchg_ag(&stamp[v], 0u) != 0u;
  }
  if (push) frontier[add_ag(&cnt[0], 1u)] = v;
}

hipError_t launch_plain_seed(int kind, void *state, uint32_t *frontier, uint32_t *cnt_slots, uint32_t *stamp,
                             const uint32_t *srcs, const unsigned long long *vals, uint32_t nsrc, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  hipLaunchKernelGGL(plain_seed_kernel, dim3((nsrc + 255) / 256), dim3(256), 0, s, kind, state, frontier, cnt_slots,
                     stamp, srcs, vals, nsrc);
  return hipGetLastError();
}

// -------------------------------------------------------------- transpose --
// G^T by counting sort on the target: histogram, exclusive scan, scatter.

__global__ void hist_kernel(const int32_t *tgt, int32_t m, int32_t *cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride)
    add_ag(&cnt[tgt[e]], 1);
}

constexpr int SCAN_TILE = 1024;  // elements per block (256 threads x 4)

// tile sums of in[0..len)
__global__ void scan_tiles_kernel(const int32_t *in, int64_t len, int32_t *sums) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 4;
  int32_t s = 0;
  for (int k = 0; k < 4; k++)
    if (base + k < len) s += in[base + k];
  int32_t tot;
  block_excl_scan_256(s, tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// exclusive scan of sums[0..nt) in place, one block
__global__ void scan_sums_kernel(int32_t *sums, int64_t nt) {
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nt; base += 256) {
    const int64_t i = base + threadIdx.x;
    const int32_t x = (i < nt) ? sums[i] : 0;
    int32_t tot;
    const int32_t ex = block_excl_scan_256(x, tot);
    const int32_t c = carry;
    if (i < nt) sums[i] = c + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + tot;
    __syncthreads();
  }
}

// out[i] = exclusive prefix of in over [0..len); out has len+1 entries
__global__ void scan_apply_kernel(const int32_t *in, int64_t len, const int32_t *sums, int32_t *out) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 4;
  int32_t v[4];
  int32_t s = 0;
  for (int k = 0; k < 4; k++) {
    v[k] = (base + k < len) ? in[base + k] : 0;
    s += v[k];
  }
  int32_t tot;
  int32_t ex = block_excl_scan_256(s, tot) + sums[blockIdx.x];
  for (int k = 0; k < 4; k++) {
    if (base + k <= len) out[base + k] = ex;
    ex += v[k];
  }
}

__global__ void __launch_bounds__(256) scatter_kernel(const int32_t *off, const int32_t *tgt, int32_t n,
                                                      int32_t *cursor, int32_t *t_tgt) {
  __shared__ uint32_t scan_s[4][64];
  const uint32_t ln = lane_id();
  const uint32_t wid = threadIdx.x >> 6;
  const uint32_t gw = blockIdx.x * 4 + wid;
  const uint32_t nw = gridDim.x * 4;
  for (uint32_t base = gw * 64; base < (uint32_t)n; base += nw * 64) {
    const bool act = base + ln < (uint32_t)n;
    const uint32_t u = base + ln;
    int32_t b = 0, e = 0;
    if (act) {
      b = off[u];
      e = off[u + 1];
    }
    const uint32_t deg = act ? (uint32_t)(e - b) : 0u;
    const uint32_t incl = wave_incl_scan(deg, ln);
    const uint32_t total = __shfl(incl, 63);
    const uint32_t excl = incl - deg;
    scan_s[wid][ln] = incl;
    wave_sync();
    for (uint32_t j = 0; j < total; j += 64) {
      const uint32_t ai = j + ln;
      uint32_t pos = 0;
#pragma unroll
      for (uint32_t step = 32; step >= 1; step >>= 1)
        if (scan_s[wid][pos + step - 1] <= ai) pos += step;
      const int owner = (int)min(pos, 63u);
      const int32_t bo = __shfl(b, owner);
      const uint32_t eo = __shfl(excl, owner);
      if (ai < total) {
        const int32_t w = tgt[bo + (int32_t)(ai - eo)];
        const int32_t at = add_ag(&cursor[w], 1);
        t_tgt[at] = (int32_t)(base + (uint32_t)owner);
      }
    }
    wave_sync();
  }
}

int64_t excl_scan_tiles(int64_t len) { return (len + 1 + SCAN_TILE - 1) / SCAN_TILE; }

hipError_t launch_excl_scan(const int32_t *in, int64_t len, int32_t *sums, int32_t *out, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  const int64_t tiles = excl_scan_tiles(len);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)tiles), dim3(256), 0, s, in, len, sums);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, s, sums, tiles);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)tiles), dim3(256), 0, s, in, len, sums, out);
  return hipGetLastError();
}

size_t transpose_scratch_elems(int32_t n) {
  const int64_t tiles = ((int64_t)n + 1 + SCAN_TILE - 1) / SCAN_TILE;
  return (size_t)n + 1 + (size_t)tiles + 16;
}

hipError_t launch_transpose(const int32_t *off, const int32_t *tgt, int32_t n, int32_t m, int32_t *t_off,
                            int32_t *t_tgt, int32_t *scratch, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  int32_t *cnt = scratch;                 // n+1 (histogram, then cursor)
  const int64_t len = (int64_t)n + 1;
  int32_t *sums = scratch + n + 1;        // scan tiles
  hipError_t e = launch_fill_u32((uint32_t *)cnt, (uint64_t)len, 0u, s);
  if (e != hipSuccess) return e;
  if (m > 0) {
    int g = (int)((m + 255) / 256);
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(hist_kernel, dim3(g), dim3(256), 0, s, tgt, m, cnt);
  }
  // counts live at cnt[0..n); scan them into t_off[0..n]
  if ((e = launch_excl_scan(cnt, (int64_t)n, sums, t_off, s)) != hipSuccess) return e;
  e = hipMemcpyAsync(cnt, t_off, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  if (m > 0) {
    int g = (int)(((int64_t)n + 255) / 256);
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(scatter_kernel, dim3(g), dim3(256), 0, s, off, tgt, n, cnt, t_tgt);
  }
  return hipGetLastError();
}

// --------------------------------------------------------------- validate --

__global__ void validate_kernel(const int32_t *off, const int32_t *tgt, int32_t n, int32_t m, Ctl *ctl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (tid == 0) bad = (off[0] != 0) || (off[n] != m);
  for (int64_t v = tid; v < n; v += stride) bad |= off[v] > off[v + 1];
  if (!bad) {
    for (int64_t e = tid; e < m; e += stride) {
      const int32_t w = tgt[e];
      bad |= (w < 0) || (w >= n);
    }
  }
  if (bad) or_ag(&ctl->bad_csr, 1u);
}

hipError_t launch_validate(const int32_t *off, const int32_t *tgt, int32_t n, int32_t m, Ctl *ctl, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  int64_t work = (int64_t)n > (int64_t)m ? (int64_t)n : (int64_t)m;
  int g = (int)((work + 255) / 256);
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(validate_kernel, dim3(g), dim3(256), 0, s, off, tgt, n, m, ctl);
  return hipGetLastError();
}

// ----------------------------------------------------------------- census --

// The frontier that a launch left behind is read from its control block
// (exit record) on the device, so the census follows the launch on the
// stream with no host round trip. A query only needs "has work left": a flag.
__global__ void census_kernel(const uint32_t *fq0, const uint32_t *fq1, const Ctl *ctl, uint32_t cap,
                              uint32_t *active, const QInfo *qi, const int64_t *qword, const uint32_t *dirty,
                              int32_t nq) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t buf = ld_ag((uint32_t *)&ctl->final_buf);
  const uint32_t cnt = min(ld_ag((uint32_t *)&ctl->final_cnt), cap);
  const uint32_t *fq = buf ? fq1 : fq0;
  for (int64_t i = tid; i < cnt; i += stride) {
    const uint32_t q = fq[i];
    if (ld_ag(&active[q]) == 0u) st_ag(&active[q], 1u);
  }
  if (ld_ag((uint32_t *)&ctl->final_ovf)) {
    const int64_t words = qword[nq];
    for (int64_t w = tid; w < words; w += stride) {
      int32_t lo = 0, hi = nq - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (qword[mid] <= w) lo = mid;
        else hi = mid - 1;
      }
      if (dirty[qi[lo].dbase + (w - qword[lo])] && ld_ag(&active[lo]) == 0u) st_ag(&active[lo], 1u);
    }
  }
}

hipError_t launch_census(const uint32_t *fq0, const uint32_t *fq1, const Ctl *ctl, uint32_t cap, uint32_t *active,
                         const QInfo *qi, const int64_t *qword, const uint32_t *dirty, int32_t nq, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  hipLaunchKernelGGL(census_kernel, dim3(1024), dim3(256), 0, s, fq0, fq1, ctl, cap, active, qi, qword, dirty, nq);
  return hipGetLastError();
}

// ------------------------------------------------------------ small utils --

__global__ void strided_u64_kernel(unsigned long long *dst, int stride, int word, const unsigned long long *src,
                                   uint64_t n) {
  const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += st)
    dst[v * (uint64_t)stride + (uint64_t)word] = src[v];
}

hipError_t launch_strided_u64(unsigned long long *dst, int stride, int word, const unsigned long long *src,
                              uint64_t n, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  hipLaunchKernelGGL(strided_u64_kernel, dim3(fill_grid(4 * n)), dim3(256), 0, s, dst, stride, word, src, n);
  return hipGetLastError();
}

// Segments are [seg_off[i], seg_off[i] + seg_len[i]) of base; `per` blocks
// share each segment (block b fills part b % per of segment b / per), so a
// few long segments still spread over the whole device.
template <class T>
__global__ void fill_segments_kernel(T *base, const int64_t *seg_off, const int64_t *seg_len, int32_t nseg, T val,
                                     int32_t per) {
  const int64_t nblk = (int64_t)nseg * per;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int32_t sgi = (int32_t)(b / per), part = (int32_t)(b % per);
    T *p = base + seg_off[sgi];
    const int64_t len = seg_len[sgi];
    for (int64_t j = (int64_t)part * blockDim.x + threadIdx.x; j < len; j += (int64_t)per * blockDim.x) p[j] = val;
  }
}

static int32_t fill_segments_per(int32_t nseg) { return nseg >= 4096 ? 1 : 4096 / nseg; }

hipError_t launch_fill_segments_u32(uint32_t *base, const int64_t *seg_off, const int64_t *seg_len, int32_t nseg,
                                    uint32_t val, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  if (nseg <= 0) return hipSuccess;
  const int32_t per = fill_segments_per(nseg);
  const int64_t blocks = std::min<int64_t>((int64_t)nseg * per, 65536);
  hipLaunchKernelGGL(fill_segments_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, base, seg_off, seg_len,
                     nseg, val, per);
  return hipGetLastError();
}
hipError_t launch_fill_segments_u64(unsigned long long *base, const int64_t *seg_off, const int64_t *seg_len,
                                    int32_t nseg, unsigned long long val, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  if (nseg <= 0) return hipSuccess;
  const int32_t per = fill_segments_per(nseg);
  const int64_t blocks = std::min<int64_t>((int64_t)nseg * per, 65536);
  hipLaunchKernelGGL(fill_segments_kernel<unsigned long long>, dim3((unsigned)blocks), dim3(256), 0, s, base, seg_off,
                     seg_len, nseg, val, per);
  return hipGetLastError();
}

__global__ void add_const_kernel(int32_t *dst, const int32_t *src, int64_t n, int32_t c) {
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += st) dst[i] = src[i] + c;
}

hipError_t launch_add_const(int32_t *dst, const int32_t *src, int64_t n, int32_t c, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's error
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_const_kernel, dim3(fill_grid(4 * (uint64_t)n)), dim3(256), 0, s, dst, src, n, c);
  return hipGetLastError();
}

}  // namespace pg
