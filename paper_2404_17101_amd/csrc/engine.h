// engine.h -- host-side helpers shared by engine.hip, batch.hip and server.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "kern.h"
#include "pasgal.h"

namespace pg {

struct DevInfo {
  int device = 0;
  int cus = 0;
  size_t lds_per_cu = 0;
  size_t lds_per_block = 0;
  int wall_khz = 100000;
  int coop = 0;
};

// grow-only device buffer
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
};
// grow-only pinned host buffer
struct HBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Slice buffers for heavy rows (VgcArgs::heavy): two of `cap` entries each.
struct SliceBufs {
  DBuf v[2], q[2], val[2], b[2];
  uint64_t cap = 0;
  int ensure(uint64_t entries, bool multi);
  // Point a's slice fields at these buffers; hcap 0 (or heavy 0) turns cutting off.
  void apply(VgcArgs &a, uint32_t heavy, uint32_t hcap, bool multi) const;
  ~SliceBufs();
};
// Slice capacity for a graph of m arcs: room for every arc twice over, at
// most the frontier capacity (0 when heavy is 0).
uint32_t slice_capacity(uint64_t m, uint32_t heavy, uint64_t frontier_cap);

// Library-owned scratch of one stream: frontier buffers, dirty bitmap,
// control block, query tables, plain-mode frontiers, pinned staging.
struct Workspace {
  std::mutex mu;
  hipStream_t stream = nullptr;
  DBuf ctl, fv[2], fq[2], fval[2], dirty, qi, qword, seeds, pf[2], stamp, tmp_state, tscratch, plain_src, aux, imp;
  uint32_t cap = 0;
  HBuf h_ctl, h_stage, h_aux, h_src;
  // An asynchronous launch (PASGAL_FLAG_ASYNC) returned before its control
  // block was read: the next call on this stream, or pasgal_wait, reads it.
  bool async_pending = false;
  SliceBufs slices;
  hipEvent_t ev0 = nullptr, evk = nullptr, ev1 = nullptr;
  void *ext = nullptr;                   // buffers of a larger driver (SCC), freed by ext_free
  void (*ext_free)(void *) = nullptr;
  ~Workspace();
};

struct Opts {
  int mode = PASGAL_MODE_VGC;
  uint32_t tau = 1024;
  int wg = 1024;
  int bpc = 1;
  int64_t cap = 0;
  uint32_t flags = 0;
  int timeout_ms = 20000;
  hipStream_t stream = nullptr;
  uint32_t window = 32;
  uint32_t min_chunk = 1;
  bool prefetch = false;
  bool test_first = false;
  uint32_t heavy = 512;  // 0 = never cut heavy rows
  uint32_t filt = 256;   // LDS filter entries per wavefront wanted (0 = none)
  uint32_t cpw = 1;      // frontier chunks per wavefront and round
  int share = 0;         // percent of every CU for a launch beside another (PASGAL_FLAG_HALF_DEVICE: 50);
                         // 0 = the whole device
};

// Persistent launches are cooperative where the device supports it, except
// half-device launches, which must be able to run beside another one.
bool coop_launch(const Opts &o);

struct LaunchGeom {
  int grid = 0, block = 0;
  size_t lds = 0;
  uint32_t ring = 0, stage = 0;
  uint32_t filt = 0;  // LDS filter entries per wavefront (distance kinds)
  bool pf = false;
};

extern thread_local int g_last_hip;
int hip_fail(hipError_t e);
const DevInfo &dev_info();
int grow(DBuf &b, size_t bytes);
int grow_host(HBuf &b, size_t bytes);
void free_buf(DBuf &b);
void free_hbuf(HBuf &b);
Workspace *workspace_for(hipStream_t s);

// A caller's gate around each burst of device work of a host-driven
// traversal (one level of the direction-optimizing BFS, enqueued and waited
// for): enter() before its first launch, leave() once the stream is idle. The
// served form uses it to keep such kernels off the device while a persistent
// launch, which needs every one of its workgroups resident, is in flight.
struct LevelGate {
  virtual void enter() = 0;
  virtual void leave() = 0;
  virtual ~LevelGate() = default;
};
// One source of a multi-source direction-optimizing BFS and where its result
// goes (device pointers, either may be null): dist[n] its hop distances (-1
// where it does not arrive), mask1[n] a reach word with bit 0 set where it
// arrives.
struct MsQuery {
  int32_t *dist;
  unsigned long long *mask1;
};
// Direction-optimizing BFS from k <= 64 sources at once (host array src),
// with per-source outputs qs (host array of k); visited_out (device, n words,
// may be null) receives bit q where source q arrives. Synchronous on
// opts->stream; gate as for bfs_do_gated.
int ms_bfs_do_gated(const pasgal_csr *g, const pasgal_csr *gt, int32_t k, const int32_t *src, const MsQuery *qs,
                    unsigned long long *visited_out, int32_t alpha, int32_t beta, const pasgal_opts *opts,
                    pasgal_stats *stats, LevelGate *gate);
// pasgal_bfs_do with a gate (nullptr: none).
int bfs_do_gated(const pasgal_csr *g, const pasgal_csr *gt, int32_t src, int32_t *dist_out, int32_t alpha,
                 int32_t beta, const pasgal_opts *opts, pasgal_stats *stats, LevelGate *gate);
Opts resolve_opts(const pasgal_opts *o);
bool opts_valid(const pasgal_opts *o);
bool csr_valid(const pasgal_csr *g);
int vgc_geometry(int kind, bool multi, const Opts &o, LaunchGeom &lg);
uint64_t default_cap(int64_t requested, uint64_t nvert);
int ensure_frontier(Workspace &w, uint64_t cap, bool multi);
void fill_stats_from_ctl(const Ctl &c, pasgal_stats *st, bool add);
int validate_csr_device(Workspace &w, const pasgal_csr *g, hipStream_t s);
// Under w.mu, first thing in every entry point that uses a workspace: when an
// asynchronous launch on this stream has not been checked yet, wait for it
// and return PASGAL_ETIMEOUT if its bounded waits expired (its results are
// then invalid), else PASGAL_OK.
int collect_async(Workspace &w);

hipError_t launch_strided_u64(unsigned long long *dst, int stride, int word, const unsigned long long *src,
                              uint64_t n, hipStream_t s);
hipError_t launch_add_const(int32_t *dst, const int32_t *src, int64_t n, int32_t c, hipStream_t s);
hipError_t launch_fill_segments_u32(uint32_t *base, const int64_t *seg_off, const int64_t *seg_len, int32_t nseg,
                                    uint32_t val, hipStream_t s);
hipError_t launch_fill_segments_u64(unsigned long long *base, const int64_t *seg_off, const int64_t *seg_len,
                                    int32_t nseg, unsigned long long val, hipStream_t s);

}  // namespace pg
