// kern.h -- types shared by the host engine and the gfx950 kernels.
//
// Device data layout (all in HBM):
//   CSR        offsets int32[n+1], targets int32[m] (caller's, read-only)
//   state      BFS: uint32 dist[v] (0xFFFFFFFF = unreached = -1 as int32)
//              SSSP: uint32 dist[v], weighted (0xFFFFFFFF = unreached)
//              REACH: uint64 mask[v] (bit i = source i of the request)
//              A launch serves several queries: query q's value of global
//              vertex v lives at state[qi[q].sbase + v].
//   dirty      uint32 bitmap words per query, qi[q].dbase + local/32; a bit is
//              set for a vertex whose frontier entry did not fit.
//   frontier   two buffers (current / next) of entries {v, q, val}, SoA:
//              v uint32, q uint32, val uint64 (dist or mask), capacity cap.
//   slices     two buffers of heavy-row slices {v, q, val, first arc}, SoA,
//              capacity hcap (see VgcArgs::heavy).
//   ctl        control block: barrier counter, abort flag, frontier tails,
//              claim counters, overflow flags and slice counts rotating over
//              3 rounds, exit record and 64-bit statistics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pg {

enum Kind : int { KIND_BFS = 0, KIND_REACH = 1, KIND_SSSP = 2 };

struct QInfo {
  int64_t sbase;  // state index of global vertex v is sbase + v
  int64_t dbase;  // dirty word of local vertex l is dbase + l/32
  int32_t vbase;  // first global vertex of the query's graph
  int32_t nv;     // vertices of the query's graph
  uint32_t r0;    // absolute round in which the query was seeded (BFS window)
  uint32_t pad;
};

enum StatIdx {
  ST_EXPAND = 0,
  ST_ARCS,
  ST_SUCCESS,
  ST_PUBLISH,
  ST_OVERFLOW,
  ST_STALE,
  ST_STEPS,     // local-search steps (one pop of up to 64 entries)
  ST_FILTERED,  // relaxations skipped by the LDS filter or the test-first load
  ST_COUNT
};

struct Ctl {
  // Words that many waiters poll sit on 128-byte lines of their own (the
  // buffer is 256-byte aligned), away from the frontier tails that every
  // flush updates atomically.
  uint32_t bar;       // grid-barrier arrivals within one launch
  uint32_t pad_bar[31];
  uint32_t abort;     // set when a bounded wait expired
  uint32_t pad_abort[31];
  uint32_t cnt[3];    // frontier tails: round r reads cnt[r%3], appends to cnt[(r+1)%3]
  uint32_t ovf[3];    // ovf[(r+1)%3] != 0: round r+1 must rescan the dirty bitmaps
  uint32_t rounds;    // rounds run by the launch (exit record)
  uint32_t final_cnt; // entries left in the last next-frontier
  uint32_t final_ovf; // dirty bits pending at exit
  uint32_t final_buf; // frontier buffer holding the leftover entries
  uint32_t max_frontier;
  uint32_t bad_csr;   // validation result
  uint32_t hcnt[3];   // heavy-row slices: round r reads hcnt[r%3], appends to hcnt[(r+1)%3]
  uint32_t claim[3][8];  // frontier chunks claimed in round r, per XCD: claim[r%3][xcd]
  uint32_t yld[3];    // yld[(r+1)%3] != 0: a yield request was seen in round r (launches with a yield word)
  unsigned long long stats[8];
};

struct Frontier {
  uint32_t *v[2];
  uint32_t *q[2];
  unsigned long long *val[2];
  uint32_t cap;
};

struct VgcArgs {
  const int32_t *off;
  const int32_t *tgt;
  const uint32_t *wgt;    // SSSP: weight of each arc (parallel to tgt); unused otherwise
  void *state;
  uint32_t *dirty;
  const QInfo *qi;
  const int64_t *qword;   // nq+1 prefix of dirty words per query (dirty scan)
  int64_t dirty_words;    // qword[nq]
  int32_t nq;
  Frontier fr;
  uint32_t start_buf;
  uint32_t tau;
  uint32_t max_rounds;
  uint32_t ring_cap;      // LDS ring entries per wave (power of two)
  uint32_t stage_cap;     // LDS staging entries per wave
  uint32_t min_chunk;     // frontier entries a wavefront takes at least per local search
  uint32_t chunks_per_wave; // frontier chunks per wavefront and round: 1 deals them statically; more
                            // makes chunks smaller, deals the first per wavefront statically and lets
                            // wavefronts that finish early claim the rest of their XCD's range
  uint32_t window;        // BFS / SSSP: round r of query q expands only distances below
                          // (round_base + r + 1 - qi[q].r0) * window; 0 = no limit
  uint32_t round_base;    // absolute number of the launch's first round
  uint32_t test_first;    // plain load before each atomic to skip relaxations that cannot succeed (selects
                          // the kernel variant)
  uint32_t filt;          // BFS / SSSP: entries of each wavefront's LDS filter of values it wrote (power of
                          // two; 0 = off). Keys are 32-bit state indices, so the state must hold < 2^32 values
  long long timeout_ticks;
  Ctl *ctl;
  // Reach with one query, source implications: srcv[j] is the vertex of
  // source j (bit j of the mask word), -1 for an unused bit; imp[j] collects
  // the bits of the sources found to reach srcv[j], which then reach every
  // vertex that source j reaches. Null imp: not used.
  unsigned long long *imp;
  const int32_t *srcv;
  // Heavy rows: an expanded vertex with more than `heavy` out-arcs (0 = never)
  // is cut into slices of `heavy` arcs {v, q, val, first arc}, written to
  // slice buffer (round parity ^ 1) and dealt one per wavefront next round.
  uint32_t heavy;
  uint32_t hcap;          // slices per buffer; slices that do not fit are expanded in place
  uint32_t *hv[2];
  uint32_t *hq[2];
  unsigned long long *hval[2];
  int32_t *hb[2];
  // Yield word (null: none): a host-written word in coherent host memory.
  // When it differs from yield_base the launch ends at the next round
  // boundary with no heavy-row slices pending, with its exit record written
  // as if max_rounds had been reached, so that the caller can add work and
  // continue from the frontier it left.
  const uint32_t *yield;
  uint32_t yield_base;
};

// Initial frontier entries for a launch (host-built, uploaded).
struct SeedEnt {
  uint32_t v;  // global vertex
  uint32_t q;
  unsigned long long val;
};

// LDS of a persistent launch: per wavefront a ring (local queue) of ring_cap
// entries and a staging buffer of stage_cap entries ({v, val[, q]} each, SoA),
// 64 words of arc-owner marks, 64 per-step entry records (16 bytes, plus 8
// with several queries) and a filter of filt 8-byte entries, 16-byte
// aligned.
__host__ __device__ inline size_t vgc_lds_bytes(int kind, bool multi, bool pf, int waves, uint32_t ring_cap,
                                                uint32_t stage_cap, uint32_t filt) {
  const size_t vsz = (kind == KIND_REACH) ? 8 : 4;
  size_t per = (size_t)(ring_cap + stage_cap) * (vsz + 4 + (multi ? 4 : 0)) + (pf ? 8 * (size_t)ring_cap : 0) +
               64 * 4 + 64 * (multi ? 24 : 16) + 8 * (size_t)filt;
  per = (per + 15) & ~(size_t)15;
  return per * (size_t)waves;
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t val, hipStream_t s);
// *out += sum of p[0..n) (64-bit; *out is not cleared).
hipError_t launch_sum_u32(const uint32_t *p, uint64_t n, unsigned long long *out, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long val, hipStream_t s);
// Zero the control block, set cnt[0] = start_cnt + nseed and ovf[0]; write the
// seed entries into frontier buffer start_buf after start_cnt and apply them
// to the state (BFS: store val; REACH: OR val).
hipError_t launch_seed(int kind, const VgcArgs &a, const SeedEnt *seeds, uint32_t nseed, uint32_t start_cnt,
                       uint32_t start_ovf, hipStream_t s);
hipError_t launch_vgc(int kind, bool multi, bool pf, const VgcArgs &a, int grid, int block, size_t lds,
                      bool cooperative, hipStream_t s);
// tf: the test-first variant (VgcArgs::test_first != 0)
const void *vgc_kernel_ptr(int kind, bool multi, bool pf, bool tf);

// Plain level-synchronous rounds (one launch per BFS level).
hipError_t launch_plain_bfs_level(const int32_t *off, const int32_t *tgt, uint32_t *dist, const uint32_t *cur,
                                  uint32_t ncur, uint32_t *nxt, uint32_t *cnt, uint32_t level, Ctl *ctl,
                                  hipStream_t s);
hipError_t launch_plain_reach_level(const int32_t *off, const int32_t *tgt, unsigned long long *mask,
                                    uint32_t *stamp, const uint32_t *cur, uint32_t ncur, uint32_t *nxt,
                                    uint32_t *cnt, uint32_t level, Ctl *ctl, hipStream_t s);
hipError_t launch_plain_seed(int kind, void *state, uint32_t *frontier, uint32_t *cnt_slots, uint32_t *stamp,
                             const uint32_t *srcs, const unsigned long long *vals, uint32_t nsrc, hipStream_t s);

// Exclusive prefix sum: out[i] = in[0] + ... + in[i-1] for i in [0, len], so
// out has len+1 entries. sums needs excl_scan_tiles(len) entries of scratch.
int64_t excl_scan_tiles(int64_t len);
hipError_t launch_excl_scan(const int32_t *in, int64_t len, int32_t *sums, int32_t *out, hipStream_t s);

// Transpose (counting sort by target).
hipError_t launch_transpose(const int32_t *off, const int32_t *tgt, int32_t n, int32_t m, int32_t *t_off,
                            int32_t *t_tgt, int32_t *scratch /* n+1 + block sums */, hipStream_t s);
size_t transpose_scratch_elems(int32_t n);

hipError_t launch_validate(const int32_t *off, const int32_t *tgt, int32_t n, int32_t m, Ctl *ctl, hipStream_t s);

// Per-query census (served form), after a launch: active[q] = 1 when query q
// has entries in the frontier the launch left (buffer and count read from the
// control block's exit record on the device) or, when an overflow is
// pending, dirty bits. active must be zeroed before.
hipError_t launch_census(const uint32_t *fq0, const uint32_t *fq1, const Ctl *ctl, uint32_t cap, uint32_t *active,
                         const QInfo *qi, const int64_t *qword, const uint32_t *dirty, int32_t nq, hipStream_t s);

}  // namespace pg
