// noalloc.hip -- pasgal_bfs_noalloc: the VGC BFS of pasgal_bfs_ex with every
// library-side buffer (control block, query table, seed entry, dirty bitmap,
// heavy-row slice buffers, frontier buffers) carved from one fixed device
// array instead of the grow-only workspace, so that the call allocates
// nothing.
//
// The array is a file-scope __device__ array. Its name is a host-side stand-in
// in host code: the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress, and only that address is handed to
// kernels and fills.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "engine.h"
#include "kern.h"
#include "pasgal.h"

namespace pg {

static __device__ __align__(256) unsigned char scratch[PASGAL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;                       // one call at a time: every call on a GPU uses that GPU's array
unsigned char *g_ptr[kMaxDevices] = {};  // device address of each GPU's copy (set up once per device)

// One thread writes the single query's table, the dirty-word prefix and the
// seed entry into the array (no host staging buffer).
__global__ void noalloc_init_kernel(QInfo *qi, int64_t *qword, SeedEnt *seed, int32_t n, int64_t words,
                                    uint32_t src) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  QInfo q;
  q.sbase = 0;
  q.dbase = 0;
  q.vbase = 0;
  q.nv = n;
  q.r0 = 0;
  q.pad = 0;
  *qi = q;
  qword[0] = 0;
  qword[1] = words;
  SeedEnt e;
  e.v = src;
  e.q = 0;
  e.val = 0ull;
  *seed = e;
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Set-up, once per device, with that device current.
int scratch_for_device(int dev, unsigned char **out) {
  if (dev < 0 || dev >= kMaxDevices) return PASGAL_EINVAL;
  if (!g_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
    (void)dev_info();  // device properties cached here, not inside a later call
    g_ptr[dev] = (unsigned char *)p;
  }
  *out = g_ptr[dev];
  return PASGAL_OK;
}

}  // namespace
}  // namespace pg

using namespace pg;

extern "C" int pasgal_bfs_noalloc(const pasgal_csr *g, int32_t src, int32_t *dist_out, const pasgal_opts *opts,
                                  pasgal_stats *stats) {
  if (!csr_valid(g) || !dist_out || src < 0 || src >= g->n || !opts_valid(opts)) return PASGAL_EINVAL;
  Opts o = resolve_opts(opts);
  if (o.mode != PASGAL_MODE_VGC || (o.flags & (PASGAL_FLAG_ASYNC | PASGAL_FLAG_VALIDATE))) return PASGAL_EINVAL;
  if ((int64_t)g->n > PASGAL_NOALLOC_MAX_VERTICES) return PASGAL_ECAPACITY;
  // the same defaults as pasgal_bfs_ex
  if (!(o.flags & PASGAL_FLAG_NO_PREFETCH) && o.tau > 1) o.prefetch = true;
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  unsigned char *base = nullptr;
  if (int rc = scratch_for_device(dev, &base)) return rc;

  // layout of the array
  const uint64_t n = (uint64_t)g->n;
  const uint64_t words = (n + 31) / 32;
  size_t off = 0;
  Ctl *ctl = (Ctl *)(base + off);
  off += up256(sizeof(Ctl));
  QInfo *qi = (QInfo *)(base + off);
  off += up256(sizeof(QInfo));
  int64_t *qword = (int64_t *)(base + off);
  off += up256(2 * sizeof(int64_t));
  SeedEnt *seed = (SeedEnt *)(base + off);
  off += up256(sizeof(SeedEnt));
  uint32_t *dirty = (uint32_t *)(base + off);
  off += up256(4 * words);
  // heavy-row slices: a bounded buffer (slices that do not fit are expanded
  // in place by the wavefront that cut them)
  const uint32_t hcap = std::min<uint32_t>(slice_capacity((uint64_t)g->m, o.heavy, 1u << 30), 16384u);
  unsigned char *slices = base + off;
  off += 2 * up256(16ull * hcap);
  if (off + 24ull * 64 > (size_t)PASGAL_NOALLOC_SCRATCH_BYTES) return PASGAL_ECAPACITY;
  const uint64_t fit = ((size_t)PASGAL_NOALLOC_SCRATCH_BYTES - off - 2 * 256) / 24;
  const uint64_t cap = std::min<uint64_t>(default_cap(o.cap, n), fit);
  uint32_t *fv[2];
  unsigned long long *fval[2];
  for (int i = 0; i < 2; i++) {
    fv[i] = (uint32_t *)(base + off);
    off += up256(4 * cap);
  }
  for (int i = 0; i < 2; i++) {
    fval[i] = (unsigned long long *)(base + off);
    off += up256(8 * cap);
  }
  if (off > (size_t)PASGAL_NOALLOC_SCRATCH_BYTES) return PASGAL_EINTERNAL;

  LaunchGeom lg;
  if (int rc = vgc_geometry(KIND_BFS, false, o, lg)) return rc;
  hipStream_t s = o.stream;
  VgcArgs a{};
  a.off = g->offsets;
  a.tgt = g->targets;
  a.state = dist_out;
  a.dirty = dirty;
  a.qi = qi;
  a.qword = qword;
  a.dirty_words = (int64_t)words;
  a.nq = 1;
  for (int i = 0; i < 2; i++) {
    a.fr.v[i] = fv[i];
    a.fr.q[i] = nullptr;
    a.fr.val[i] = fval[i];
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
  a.filt = lg.filt;
  a.ctl = ctl;
  a.heavy = hcap ? o.heavy : 0u;
  a.hcap = a.heavy ? hcap : 0u;
  for (int i = 0; i < 2; i++) {
    unsigned char *sb = slices + i * up256(16ull * hcap);
    a.hv[i] = (uint32_t *)sb;
    a.hq[i] = nullptr;
    a.hb[i] = (int32_t *)(sb + 4ull * hcap);
    a.hval[i] = (unsigned long long *)(sb + 8ull * hcap);
  }

  // everything that must start at zero is cleared with fill kernels: the
  // array keeps the previous call's contents
  (void)hipGetLastError();
  hipLaunchKernelGGL(noalloc_init_kernel, dim3(1), dim3(64), 0, s, qi, qword, seed, g->n, (int64_t)words,
                     (uint32_t)src);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e);
  if ((e = launch_fill_u32((uint32_t *)dist_out, n, 0xFFFFFFFFu, s)) != hipSuccess) return hip_fail(e);
  if ((e = launch_fill_u32(dirty, words, 0u, s)) != hipSuccess) return hip_fail(e);
  if ((e = launch_fill_u32((uint32_t *)ctl, sizeof(Ctl) / 4, 0u, s)) != hipSuccess) return hip_fail(e);
  if ((e = launch_seed(KIND_BFS, a, seed, 1, 0, 0, s)) != hipSuccess) return hip_fail(e);
  if ((e = launch_vgc(KIND_BFS, false, lg.pf, a, lg.grid, lg.block, lg.lds, coop_launch(o), s)) != hipSuccess)
    return hip_fail(e);
  // the control block (abort flag, counters) comes back through a stack copy
  Ctl c;
  if ((e = hipMemcpyAsync(&c, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
  if (c.abort) return PASGAL_ETIMEOUT;
  if (stats) fill_stats_from_ctl(c, stats, false);
  return PASGAL_OK;
}
