// scc.hip -- strongly connected components by batched reachability searches
// (Parallel SCC section of the paper; the algorithm it adopts runs forward
// and backward reachability from batches of pivots, settles every vertex
// found both ways from a pivot into that pivot's component, and splits the
// rest into subproblems that later searches never leave).
//
// GPU form:
//  * G and G^T are packed into one CSR of 2n vertices: v is the forward copy
//    of vertex v, n+v its backward copy. The packed CSR keeps only arcs
//    between unsettled vertices of the same subproblem, so one persistent
//    VGC reach launch runs every pivot's forward and backward search at once
//    and no search leaves its subproblem.
//  * Subproblems are named by labels in [0, H), H = 2^k >= n. A pivot takes
//    bit i of a 64-bit mask from its subproblem's counter, so bits are
//    numbered per subproblem and a batch may hold any number of pivots, at
//    most 64 per subproblem (the rest wait for a repeat of the batch).
//    Because arcs never cross subproblems, bit i seen at a vertex always
//    means the pivot of the vertex's own subproblem that drew bit i.
//  * After a batch a vertex v with F(v) & B(v) != 0 joins the component of
//    the pivot of the lowest common bit; any other vertex reached either way
//    gets the label hash(label, F, B) mod H. Vertices of one component have
//    equal (label, F, B), so components are never split. Two subproblems
//    whose labels collide merge: a union of whole components is still a valid
//    subproblem, so the result stays exact and only the work grows.
//  * Pivots come from a random order of the vertices (a keyed Feistel
//    permutation walked into [0, n)), in batches of 1, 2, 4, ... positions;
//    a position whose vertex is already settled is skipped.
//  * Trimming (an addition, not in the paper's description): a vertex with
//    no in-arc or no out-arc left in the packed CSR is a component by itself.
//  * Weak-connectivity split (an addition, not in the paper's description):
//    after every batch each subproblem is cut into the weakly connected
//    pieces of its packed arcs (a component never spans two pieces) and each
//    piece is named by its smallest vertex. Tendrils left around a removed
//    giant component become many small subproblems, each with its own 64
//    pivot bits, instead of one subproblem that gets 64 pivots per repeat.
//  * The output names each component by its smallest vertex, which makes it
//    unique whatever the pivots were.
//  * Active-vertex renumbering: the unsettled vertices, in ascending order,
//    are numbered 0..na-1 (act[j] = global id, loc[v] = local id). After
//    every refinement and trimming pass a stable compaction drops the
//    settled ones, and the packed CSR (2*na rows, local ids), the masks, the
//    labels (per local row) and every per-vertex pass cover only the active
//    vertices. Pivots still come from the random order of all vertex ids.
//    Because the order is kept, the smallest local id of a set of active
//    vertices is also its smallest global id.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "devutil.h"
#include "engine.h"
#include "kern.h"
#include "pasgal.h"

namespace pg {

namespace {

// counters[] slots (device; read back once per batch)
enum : int { C_NPIV = 0, C_DEFER, C_POOL, C_TRIM, C_COMPS, C_UNSETTLED, C_COUNT = 8 };

// Source of a pack: the arcs of the rows to keep, in the numbering of the
// previous pack (or the caller's G and G^T, numbered by global id, before the
// first pack). Forward rows are (offA, tgtA), backward rows (offB, tgtB),
// both indexed by the old local id; a target t names old local id t, or
// t - na_old for a backward copy.
struct PackSrc {
  const int32_t *offA, *tgtA;
  const int32_t *offB, *tgtB;
  uint32_t na_old;
};

// ------------------------------------------------------------ permutation --
// Keyed bijection of [0, 2^(2h)) from four Feistel rounds; walking it from a
// position below n until the value is below n is a bijection of [0, n)
// (the walk stays on the position's cycle, which contains a value < n).
__device__ __forceinline__ uint32_t feistel_f(uint32_t x, uint32_t key) {
  x ^= key;
  x *= 0x9E3779B1u;
  x ^= x >> 15;
  x *= 0x85EBCA77u;
  x ^= x >> 13;
  return x;
}

__device__ __forceinline__ uint32_t perm_at(uint32_t pos, uint32_t n, uint32_t h, uint32_t seed) {
  const uint32_t hm = (1u << h) - 1u;  // h <= 15
  uint32_t x = pos;
  do {
    uint32_t l = x >> h, r = x & hm;
#pragma unroll
    for (uint32_t k = 0; k < 4; k++) {
      const uint32_t t = l ^ (feistel_f(r, seed + k * 0x6A09E667u) & hm);
      l = r;
      r = t;
    }
    x = (l << h) | r;
  } while (x >= n);
  return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += (uint32_t)__shfl_xor(x, d);
  return x;
}

// Label of the subproblem of vertices reached by forward set f and backward
// set b from subproblem lab (64-bit mix, folded to [0, hmask]).
__device__ __forceinline__ uint32_t refine_label(uint32_t lab, unsigned long long f, unsigned long long b,
                                                 uint32_t hmask) {
  unsigned long long x = (unsigned long long)lab * 0x9E3779B97F4A7C15ull;
  x ^= f + 0xBF58476D1CE4E5B9ull + (x << 6) + (x >> 2);
  x ^= (b * 0x94D049BB133111EBull) + (x << 6) + (x >> 2);
  x ^= x >> 31;
  x *= 0xD6E8FEB86659FD93ull;
  x ^= x >> 32;
  return (uint32_t)x & hmask;
}

// Work of every kernel below is walked in whole wavefronts: each wave takes
// 64 consecutive items per step, so ballots and shuffles see all 64 lanes.
__device__ __forceinline__ uint64_t wave_first(uint64_t lo) {
  return lo + (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
}
__device__ __forceinline__ uint64_t grid_step() { return (uint64_t)gridDim.x * blockDim.x; }

// ------------------------------------------------------------ pack kernels --
// One wavefront handles 64 consecutive rows of the new packed graph (row r <
// na_new: forward copy of new local vertex r; row na_new + r: its backward
// copy): their source arcs are dealt out across the lanes (consecutive lanes
// take consecutive arcs, owner row by binary search over the degree scan).
// An arc is kept iff its target is still active (remap >= 0), is not the row's
// own vertex and carries the same label. The count pass writes the kept arcs
// of each row; the scatter pass writes them at off_new[first row] + (kept
// arcs of the 64 rows before it), which is their packed position because the
// rows are consecutive.
template <bool SCATTER>
__global__ void __launch_bounds__(256) pack_kernel(PackSrc in, uint32_t na_new, const uint32_t *__restrict__ old_of,
                                                   const int32_t *__restrict__ remap,
                                                   const uint32_t *__restrict__ label_old, int32_t *__restrict__ cnt,
                                                   const int32_t *__restrict__ off_new,
                                                   int32_t *__restrict__ tgt_new) {
  __shared__ uint32_t scan_s[4][64];
  __shared__ uint32_t keep_s[4][64];
  const uint32_t ln = lane_id(), wid = threadIdx.x >> 6;
  const uint64_t rows = 2ull * na_new;
  const uint32_t na_old = in.na_old;
  for (uint64_t base = wave_first(0); base < rows; base += grid_step()) {
    const uint64_t u = base + ln;
    const bool fwd = u < na_new;
    int32_t b = 0, e = 0;
    uint32_t lab = 0, src = 0;
    if (u < rows) {
      src = old_of[fwd ? u : u - na_new];
      const int32_t *o = fwd ? in.offA : in.offB;
      b = o[src];
      e = o[src + 1];
      lab = label_old[src];
    }
    const uint32_t deg = (uint32_t)(e - b);
    const uint32_t incl = wave_incl_scan(deg, ln);
    const uint32_t total = __shfl(incl, 63);
    const uint32_t excl = incl - deg;
    scan_s[wid][ln] = incl;
    keep_s[wid][ln] = 0;
    const int32_t dst = SCATTER ? off_new[base] : 0;
    uint32_t run = 0;
    wave_sync();
    for (uint32_t j = 0; j < total; j += 64) {
      const uint32_t ai = j + ln;
      uint32_t pos = 0;
#pragma unroll
      for (uint32_t s = 32; s >= 1; s >>= 1)
        if (scan_s[wid][pos + s - 1] <= ai) pos += s;
      const int owner = (int)min(pos, 63u);
      const int32_t bo = __shfl(b, owner);
      const uint32_t eo = __shfl(excl, owner);
      const uint32_t lo = __shfl(lab, owner);
      const uint32_t so = __shfl(src, owner);
      bool keep = false;
      uint32_t t_out = 0;
      if (ai < total) {
        const bool f = base + (uint64_t)owner < na_new;
        const uint32_t t = (uint32_t)(f ? in.tgtA : in.tgtB)[bo + (int32_t)(ai - eo)];
        const uint32_t bw = t >= na_old ? t - na_old : t;
        const int32_t nw = remap[bw];
        keep = bw != so && nw >= 0 && label_old[bw] == lo;
        t_out = f ? (uint32_t)nw : (uint32_t)nw + na_new;
      }
      const unsigned long long bal = __ballot(keep);
      if (SCATTER) {
        if (keep) tgt_new[dst + (int32_t)(run + mbcnt64(bal))] = (int32_t)t_out;
      } else if (keep) {
        atomicAdd(&keep_s[wid][owner], 1u);
      }
      run += (uint32_t)__popcll(bal);
    }
    wave_sync();
    if (!SCATTER && u < rows) cnt[u] = (int32_t)keep_s[wid][ln];
    wave_sync();
  }
}

// Active-vertex compaction, step 1: keep[j] = 1 iff act[j] is unsettled.
__global__ void __launch_bounds__(256) keep_kernel(uint32_t na, const uint32_t *__restrict__ act,
                                                   const int32_t *__restrict__ comp, int32_t *__restrict__ keep) {
  const uint64_t stride = grid_step();
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < na; j += stride)
    keep[j] = comp[act[j]] < 0 ? 1 : 0;
}

// Step 2 (after the exclusive scan pos of keep): the kept vertices move to
// their new local ids in order; remap[old] = new id or -1.
__global__ void __launch_bounds__(256) compact_kernel(uint32_t na, const uint32_t *__restrict__ act_old,
                                                      const uint32_t *__restrict__ label_old,
                                                      const int32_t *__restrict__ keep,
                                                      const int32_t *__restrict__ pos, uint32_t *__restrict__ act_new,
                                                      uint32_t *__restrict__ label_new, uint32_t *__restrict__ old_of,
                                                      int32_t *__restrict__ remap, uint32_t *__restrict__ loc) {
  const uint64_t stride = grid_step();
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < na; j += stride) {
    if (keep[j]) {
      const uint32_t jn = (uint32_t)pos[j], v = act_old[j];
      act_new[jn] = v;
      label_new[jn] = label_old[j];
      old_of[jn] = (uint32_t)j;
      remap[j] = (int32_t)jn;
      loc[v] = jn;
    } else {
      remap[j] = -1;
    }
  }
}

__global__ void iota_kernel(uint32_t n, uint32_t *__restrict__ out) {
  const uint64_t stride = grid_step();
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) out[v] = (uint32_t)v;
}

// The reach launch's query record: one query over the 2*na packed vertices.
__global__ void set_query_kernel(QInfo *qi, int64_t *qword, uint32_t nv) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    qi->sbase = 0;
    qi->dbase = 0;
    qi->vbase = 0;
    qi->nv = (int32_t)nv;
    qi->r0 = 0;
    qi->pad = 0;
    qword[0] = 0;
    qword[1] = ((int64_t)nv + 31) / 32;
  }
}

// A vertex with no out-arc or no in-arc left in the packed CSR is a
// component by itself.
__global__ void __launch_bounds__(256) trim_kernel(const int32_t *__restrict__ off2, uint32_t na,
                                                   const uint32_t *__restrict__ act, int32_t *__restrict__ comp,
                                                   uint32_t *__restrict__ counters) {
  uint32_t mine = 0;
  for (uint64_t base = wave_first(0); base < na; base += grid_step()) {
    const uint64_t j = base + lane_id();
    if (j < na) {
      const uint32_t v = act[j];
      if (comp[v] < 0) {
        const bool no_out = off2[j + 1] == off2[j];
        const bool no_in = off2[na + j + 1] == off2[na + j];
        if (no_out || no_in) {
          comp[v] = (int32_t)v;
          mine++;
        }
      }
    }
  }
  mine = wave_sum(mine);
  if (lane_id() == 0 && mine) add_ag(&counters[C_TRIM], mine);
}

// Pivots of positions [lo, hi) of the random order: each unsettled vertex
// draws the next bit of its subproblem's counter; draws >= 64 wait for a
// repeat of the batch. act != null: the batch covers every remaining position
// (hi = n), and the active vertices act[0, hi) are walked instead of the
// positions (fewer once most vertices are settled).
__global__ void __launch_bounds__(256) select_kernel(uint32_t lo, uint32_t hi, uint32_t n, uint32_t h,
                                                     uint32_t seed, const uint32_t *__restrict__ act,
                                                     const int32_t *__restrict__ comp,
                                                     const uint32_t *__restrict__ loc,
                                                     const uint32_t *__restrict__ label,
                                                     uint32_t *__restrict__ slot_cnt, uint32_t *__restrict__ piv_v,
                                                     uint32_t *__restrict__ piv_bit,
                                                     uint32_t *__restrict__ counters) {
  const uint32_t ln = lane_id();
  uint32_t deferred = 0;
  for (uint64_t base = wave_first(lo); base < hi; base += grid_step()) {
    const uint64_t pos = base + ln;
    uint32_t v = 0, bit = 64;
    bool draw = false;
    if (pos < hi) {
      v = act ? act[pos] : perm_at((uint32_t)pos, n, h, seed);
      if (comp[v] < 0) {
        bit = add_ag(&slot_cnt[label[loc[v]]], 1u);
        draw = true;
      }
    }
    const bool isp = draw && bit < 64;
    deferred += (draw && !isp) ? 1u : 0u;
    const unsigned long long bp = __ballot(isp);
    uint32_t k0 = 0;
    if (ln == 0 && bp) k0 = add_ag(&counters[C_NPIV], (uint32_t)__popcll(bp));
    k0 = __shfl(k0, 0);
    if (isp) {
      const uint32_t k = k0 + mbcnt64(bp);
      piv_v[k] = v;
      piv_bit[k] = bit;
    }
  }
  deferred = wave_sum(deferred);
  if (ln == 0 && deferred) add_ag(&counters[C_DEFER], deferred);
}

// The pivot that drew bit 0 of a subproblem reserves min(draws, 64) entries
// of the pivot table for it.
__global__ void __launch_bounds__(256) reserve_kernel(uint32_t npiv, const uint32_t *__restrict__ piv_v,
                                                      const uint32_t *__restrict__ piv_bit,
                                                      const uint32_t *__restrict__ loc,
                                                      const uint32_t *__restrict__ label,
                                                      const uint32_t *__restrict__ slot_cnt,
                                                      uint32_t *__restrict__ slot_base,
                                                      uint32_t *__restrict__ counters) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npiv || piv_bit[k] != 0) return;
  const uint32_t lab = label[loc[piv_v[k]]];
  slot_base[lab] = add_ag(&counters[C_POOL], min(slot_cnt[lab], 64u));
}

// Record each pivot (global id) in the table and seed its forward copy j =
// loc[v] and backward copy na + j with its bit: mask state and frontier
// entries 2k, 2k+1 (entries past the frontier capacity go to the dirty
// bitmap). The masks and the control block were zeroed before.
__global__ void __launch_bounds__(256) seed_pivots_kernel(VgcArgs a, uint32_t na, uint32_t npiv,
                                                          const uint32_t *__restrict__ piv_v,
                                                          const uint32_t *__restrict__ piv_bit,
                                                          const uint32_t *__restrict__ loc,
                                                          const uint32_t *__restrict__ label,
                                                          const uint32_t *__restrict__ slot_base,
                                                          int32_t *__restrict__ pivtab) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) st_ag(&a.ctl->cnt[0], 2u * npiv);
  if (k >= npiv) return;
  const uint32_t v = piv_v[k], bit = piv_bit[k], j = loc[v];
  pivtab[slot_base[label[j]] + bit] = (int32_t)v;
  const unsigned long long m = 1ull << bit;
  unsigned long long *mask = (unsigned long long *)a.state;
  const uint32_t vv[2] = {j, na + j};
  for (int d = 0; d < 2; d++) {
    mask[vv[d]] = m;
    const uint64_t pos = 2ull * k + (uint64_t)d;
    if (pos < a.fr.cap) {
      a.fr.v[0][pos] = vv[d];
      a.fr.val[0][pos] = m;
    } else {
      or_ag(&a.dirty[vv[d] >> 5], 1u << (vv[d] & 31));
      or_ag(&a.ctl->ovf[0], 1u);
    }
  }
}

// Settle or refine every unsettled active vertex from its forward mask
// F = mask[j] and backward mask B = mask[na + j].
__global__ void __launch_bounds__(256) refine_kernel(uint32_t na, uint32_t hmask,
                                                     const unsigned long long *__restrict__ mask,
                                                     const uint32_t *__restrict__ act, int32_t *__restrict__ comp,
                                                     uint32_t *__restrict__ label,
                                                     const uint32_t *__restrict__ slot_base,
                                                     const int32_t *__restrict__ pivtab) {
  const uint64_t stride = grid_step();
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < na; j += stride) {
    const uint32_t v = act[j];
    if (comp[v] >= 0) continue;
    const unsigned long long f = mask[j], b = mask[na + j];
    const unsigned long long c = f & b;
    const uint32_t lab = label[j];
    if (c)
      comp[v] = pivtab[slot_base[lab] + (uint32_t)__builtin_ctzll(c)];
    else if (f | b)
      label[j] = refine_label(lab, f, b, hmask);
  }
}

// Pivots are settled and keep their label: their subproblem counters go back
// to zero for the next batch.
__global__ void __launch_bounds__(256) clear_slots_kernel(uint32_t npiv, const uint32_t *__restrict__ piv_v,
                                                          const uint32_t *__restrict__ loc,
                                                          const uint32_t *__restrict__ label,
                                                          uint32_t *__restrict__ slot_cnt) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < npiv) slot_cnt[label[loc[piv_v[k]]]] = 0;
}

// minv[c] = smallest vertex whose component record is c. A giant component
// sends millions of vertices to one record, so lanes that share the
// wavefront's first record reduce among themselves first, and an atomic is
// issued only when a plain read shows it can still lower the record.
__global__ void __launch_bounds__(256) min_member_kernel(uint32_t n, const int32_t *__restrict__ comp,
                                                         int32_t *minv) {
  const uint32_t ln = lane_id();
  for (uint64_t base = wave_first(0); base < n; base += grid_step()) {
    const uint64_t v = base + ln;
    const int32_t c = v < n ? comp[v] : -1;
    const int32_t c0 = __shfl(c, 0);  // lane 0 holds the wave's smallest vertex
    const bool same = c >= 0 && c == c0;
    const uint32_t vmin = wave_min(same ? (uint32_t)v : 0xFFFFFFFFu);
    if (ln == 0 && c0 >= 0 && (int32_t)vmin < ld_ag(&minv[c0])) min_ag(&minv[c0], (int32_t)vmin);
    if (c >= 0 && !same && (int32_t)v < ld_ag(&minv[c])) min_ag(&minv[c], (int32_t)v);
  }
}

// comp[v] <- smallest vertex of its component; counts the components (and,
// as a consistency check, vertices left unsettled, which must be none).
__global__ void __launch_bounds__(256) relabel_kernel(uint32_t n, int32_t *__restrict__ comp,
                                                      const int32_t *__restrict__ minv,
                                                      uint32_t *__restrict__ counters) {
  uint32_t roots = 0, unsettled = 0;
  for (uint64_t base = wave_first(0); base < n; base += grid_step()) {
    const uint64_t v = base + lane_id();
    if (v < n) {
      const int32_t r = comp[v];
      if (r >= 0) {
        const int32_t c = minv[r];
        comp[v] = c;
        roots += (c == (int32_t)v) ? 1u : 0u;
      } else {
        unsettled++;
      }
    }
  }
  roots = wave_sum(roots);
  unsettled = wave_sum(unsettled);
  if (lane_id() == 0 && roots) add_ag(&counters[C_COMPS], roots);
  if (lane_id() == 0 && unsettled) add_ag(&counters[C_UNSETTLED], unsettled);
}

// ------------------------------------------------------ weak connectivity --
// Lock-free union-find over the packed arcs: parent pointers only ever point
// to a smaller vertex, so the root of a piece ends as its smallest vertex.
// find() halves paths as it walks (a vertex is re-pointed to an ancestor,
// which stays an ancestor); unite() hooks the larger root under the smaller
// one with a compare-and-swap and retries from the new roots when another
// thread hooked first (each failure means a root was hooked, so the retries
// end).
__device__ __forceinline__ uint32_t uf_find(uint32_t *parent, uint32_t v) {
  uint32_t p = ld_ag(&parent[v]);
  while (p != v) {
    const uint32_t gp = ld_ag(&parent[p]);
    if (gp != p) st_ag(&parent[v], gp);
    v = p;
    p = gp;
  }
  return v;
}

__device__ __forceinline__ void uf_unite(uint32_t *parent, uint32_t a, uint32_t b) {
  a = uf_find(parent, a);
  b = uf_find(parent, b);
  while (a != b) {
    if (a < b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    const uint32_t old = cas_ag(&parent[a], a, b);
    if (old == a) return;
    a = uf_find(parent, old);
    b = uf_find(parent, b);
  }
}

// Unite the endpoints of every forward arc of the packed CSR between
// unsettled vertices (local ids; the backward rows hold the same arcs
// reversed). The arcs of 64 consecutive rows are dealt out across a
// wavefront as in the pack.
__global__ void __launch_bounds__(256) union_kernel(const int32_t *__restrict__ off2,
                                                    const int32_t *__restrict__ tgt2, uint32_t na,
                                                    const uint32_t *__restrict__ act,
                                                    const int32_t *__restrict__ comp, uint32_t *parent) {
  __shared__ uint32_t scan_s[4][64];
  const uint32_t ln = lane_id(), wid = threadIdx.x >> 6;
  for (uint64_t base = wave_first(0); base < na; base += grid_step()) {
    const uint64_t u = base + ln;
    int32_t b = 0, e = 0;
    if (u < na && comp[act[u]] < 0) {
      b = off2[u];
      e = off2[u + 1];
    }
    const uint32_t deg = (uint32_t)(e - b);
    const uint32_t incl = wave_incl_scan(deg, ln);
    const uint32_t total = __shfl(incl, 63);
    const uint32_t excl = incl - deg;
    scan_s[wid][ln] = incl;
    wave_sync();
    for (uint32_t j = 0; j < total; j += 64) {
      const uint32_t ai = j + ln;
      uint32_t pos = 0;
#pragma unroll
      for (uint32_t s = 32; s >= 1; s >>= 1)
        if (scan_s[wid][pos + s - 1] <= ai) pos += s;
      const int owner = (int)min(pos, 63u);
      const int32_t bo = __shfl(b, owner);
      const uint32_t eo = __shfl(excl, owner);
      if (ai < total) {
        const uint32_t w = (uint32_t)tgt2[bo + (int32_t)(ai - eo)];
        if (comp[act[w]] < 0) uf_unite(parent, (uint32_t)base + (uint32_t)owner, w);
      }
    }
    wave_sync();
  }
}

// Every unsettled active vertex takes its piece's root as label, named by
// the root's global id (the smallest vertex of the piece, since local ids
// keep the order of global ids).
__global__ void __launch_bounds__(256) piece_label_kernel(uint32_t na, const uint32_t *__restrict__ act,
                                                          const int32_t *__restrict__ comp, uint32_t *parent,
                                                          uint32_t *__restrict__ label) {
  const uint64_t stride = grid_step();
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < na; j += stride)
    if (comp[act[j]] < 0) label[j] = act[uf_find(parent, (uint32_t)j)];
}

int grid_for(uint64_t items, int cap = 8192) {
  uint64_t g = (items + 255) / 256;
  if (g < 1) g = 1;
  if (g > (uint64_t)cap) g = (uint64_t)cap;
  return (int)g;
}

// ------------------------------------------------------------ host driver --

// Grow-only buffers of the SCC driver, one set per stream workspace.
struct SccBufs {
  DBuf off2[2], tgt2[2], mask, lab[2], act[2], loc, remap, old_of, keep, pos, slot_cnt, slot_base, pivtab, piv_v,
      piv_bit, cnt, sums, counters, minv, t_off, t_tgt, tscratch, parent;
  HBuf h_read;  // counters, control block and the active count, read back per batch
  ~SccBufs() {
    for (DBuf *b : {&off2[0], &off2[1], &tgt2[0], &tgt2[1], &mask, &lab[0], &lab[1], &act[0], &act[1], &loc, &remap,
                    &old_of, &keep, &pos, &slot_cnt, &slot_base, &pivtab, &piv_v, &piv_bit, &cnt, &sums, &counters,
                    &minv, &t_off, &t_tgt, &tscratch, &parent})
      free_buf(*b);
    free_hbuf(h_read);
  }
};

std::mutex g_scc_mu;

void free_scc_bufs(void *p) { delete (SccBufs *)p; }

SccBufs *scc_bufs(Workspace *w) {
  std::lock_guard<std::mutex> lk(g_scc_mu);
  if (!w->ext) {
    w->ext = new (std::nothrow) SccBufs();
    if (w->ext) w->ext_free = free_scc_bufs;
  }
  return (SccBufs *)w->ext;
}

struct SccRun {
  SccBufs &b;
  hipStream_t s;
  uint32_t n;
  uint32_t *h_na;  // pinned: the active count read back after a compaction
  int cur = 0;     // packed CSR buffer holding the current graph
  int ab = 0;      // act / label buffers of the current numbering
  uint32_t na = 0;  // active vertices in the current numbering

  int32_t *off2(int i) { return (int32_t *)b.off2[i].p; }
  int32_t *tgt2(int i) { return (int32_t *)b.tgt2[i].p; }
  uint32_t *counters() { return (uint32_t *)b.counters.p; }
  uint32_t *act() { return (uint32_t *)b.act[ab].p; }
  uint32_t *label() { return (uint32_t *)b.lab[ab].p; }
  uint32_t *loc() { return (uint32_t *)b.loc.p; }

  // Drop the settled vertices from the numbering (stable compaction) and
  // rebuild the packed CSR from `src`, numbered by the numbering before this
  // call, into buffer dst.
  hipError_t compact_and_pack(const PackSrc &src, int dst, const int32_t *comp) {
    (void)hipGetLastError();
    const uint32_t na_old = na;
    const int old = ab, nw = ab ^ 1;
    int32_t *keep = (int32_t *)b.keep.p, *pos = (int32_t *)b.pos.p;
    hipLaunchKernelGGL(keep_kernel, dim3(grid_for(na_old)), dim3(256), 0, s, na_old, (const uint32_t *)b.act[old].p,
                       comp, keep);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_excl_scan(keep, (int64_t)na_old, (int32_t *)b.sums.p, pos, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(h_na, pos + na_old, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const uint32_t na_new = *h_na;
    hipLaunchKernelGGL(compact_kernel, dim3(grid_for(na_old)), dim3(256), 0, s, na_old,
                       (const uint32_t *)b.act[old].p, (const uint32_t *)b.lab[old].p, (const int32_t *)keep,
                       (const int32_t *)pos, (uint32_t *)b.act[nw].p, (uint32_t *)b.lab[nw].p,
                       (uint32_t *)b.old_of.p, (int32_t *)b.remap.p, loc());
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const uint64_t rows = 2ull * na_new;
    const int grid = grid_for(rows, 16384);  // 256 rows per block and step (4 waves x 64 rows)
    int32_t *cnt = (int32_t *)b.cnt.p;
    hipLaunchKernelGGL(pack_kernel<false>, dim3(grid), dim3(256), 0, s, src, na_new, (const uint32_t *)b.old_of.p,
                       (const int32_t *)b.remap.p, (const uint32_t *)b.lab[old].p, cnt, (const int32_t *)nullptr,
                       (int32_t *)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_excl_scan(cnt, (int64_t)rows, (int32_t *)b.sums.p, off2(dst), s)) != hipSuccess) return e;
    hipLaunchKernelGGL(pack_kernel<true>, dim3(grid), dim3(256), 0, s, src, na_new, (const uint32_t *)b.old_of.p,
                       (const int32_t *)b.remap.p, (const uint32_t *)b.lab[old].p, (int32_t *)nullptr,
                       (const int32_t *)off2(dst), tgt2(dst));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ab = nw;
    na = na_new;
    return hipSuccess;
  }
  // Relabel every unsettled active vertex by its weakly connected piece of
  // the current packed CSR.
  hipError_t split_pieces(const int32_t *comp) {
    (void)hipGetLastError();
    if (na == 0) return hipSuccess;
    uint32_t *parent = (uint32_t *)b.parent.p;
    hipLaunchKernelGGL(iota_kernel, dim3(grid_for(na)), dim3(256), 0, s, na, parent);
    hipLaunchKernelGGL(union_kernel, dim3(grid_for(na, 16384)), dim3(256), 0, s, (const int32_t *)b.off2[cur].p,
                       (const int32_t *)b.tgt2[cur].p, na, (const uint32_t *)act(), comp, parent);
    hipLaunchKernelGGL(piece_label_kernel, dim3(grid_for(na)), dim3(256), 0, s, na, (const uint32_t *)act(), comp,
                       parent, label());
    return hipGetLastError();
  }
  PackSrc packed_src() const {
    PackSrc p;
    p.offA = (const int32_t *)b.off2[cur].p;
    p.tgtA = (const int32_t *)b.tgt2[cur].p;
    p.offB = (const int32_t *)b.off2[cur].p + na;
    p.tgtB = (const int32_t *)b.tgt2[cur].p;
    p.na_old = na;
    return p;
  }
};

}  // namespace

}  // namespace pg

using namespace pg;

extern "C" int pasgal_scc(const pasgal_csr *g, const pasgal_csr *gt, int32_t *comp_out,
                          const pasgal_scc_opts *scc_opts, const pasgal_opts *opts, pasgal_scc_stats *stats) {
  if (!csr_valid(g) || !comp_out || !opts_valid(opts)) return PASGAL_EINVAL;
  if (scc_opts && (scc_opts->flags & ~PASGAL_SCC_NO_SPLIT)) return PASGAL_EINVAL;
  int32_t trim_rounds = scc_opts ? scc_opts->trim_rounds : -1;
  const bool split = !(scc_opts && (scc_opts->flags & PASGAL_SCC_NO_SPLIT));
  const uint32_t seed = (scc_opts && scc_opts->seed) ? scc_opts->seed : 0x5CC0FFEEu;
  if (gt && (!csr_valid(gt) || gt->n != g->n || gt->m != g->m)) return PASGAL_EINVAL;
  if (g->n >= (1 << 30) || g->m >= (1 << 30)) return PASGAL_EINVAL;
  Opts o = resolve_opts(opts);
  if (o.flags & PASGAL_FLAG_ASYNC) return PASGAL_EINVAL;
  // default tau by mean out-degree, as for SSSP: on dense low-diameter graphs
  // the searches reach everything in a few levels anyway
  if (!opts || opts->tau <= 0) o.tau = (int64_t)g->m > 8 * (int64_t)g->n ? 1u : 1024u;
  // and a plain read before each OR there (most arcs offer bits already present)
  if ((int64_t)g->m > 8 * (int64_t)g->n && !(o.flags & PASGAL_FLAG_NO_TEST_FIRST)) o.test_first = true;
  if (o.mode == PASGAL_MODE_PLAIN) o.tau = 1;
  // arc ranges carried in the local queue, as for pasgal_reach_ex (4-5% faster on road and k-NN
  // graphs); at tau 1 no carried range is used
  if (!(o.flags & PASGAL_FLAG_NO_PREFETCH) && o.tau > 1) o.prefetch = true;
  if (trim_rounds < 0) trim_rounds = 1;  // later passes run after every batch anyway
  Workspace *w = workspace_for(o.stream);
  if (!w) return PASGAL_ENOMEM;
  std::lock_guard<std::mutex> lk(w->mu);
  if (int arc = collect_async(*w)) return arc;
  SccBufs *bp = scc_bufs(w);
  if (!bp) return PASGAL_ENOMEM;
  SccBufs &B = *bp;
  hipStream_t s = o.stream;
  int rc;
  hipError_t e;
  if (o.flags & PASGAL_FLAG_VALIDATE) {
    if ((rc = validate_csr_device(*w, g, s))) return rc;
    if (gt && (rc = validate_csr_device(*w, gt, s))) return rc;
  }
  if (stats) memset(stats, 0, sizeof(*stats));
  const uint32_t n = (uint32_t)g->n;
  const uint64_t n2 = 2ull * n, m2 = 2ull * (uint64_t)g->m;
  uint32_t hbits = 1;
  while ((1ull << hbits) < n) hbits++;
  const uint64_t H = 1ull << hbits;  // label space
  const uint32_t hmask = (uint32_t)(H - 1);
  uint32_t fh = 1;  // Feistel half width: 2^(2 fh) >= n
  while ((1ull << (2 * fh)) < n) fh++;
  const uint64_t cap = default_cap(o.cap, n2);
  const uint64_t dwords = (n2 + 31) / 32;
  LaunchGeom lg;
  if ((rc = vgc_geometry(KIND_REACH, false, o, lg))) return rc;
  if ((rc = ensure_frontier(*w, cap, false))) return rc;
  struct {
    DBuf *b;
    size_t bytes;
  } need[] = {{&B.off2[0], 4 * (n2 + 1)}, {&B.off2[1], 4 * (n2 + 1)}, {&B.tgt2[0], 4 * m2 + 4},
              {&B.tgt2[1], 4 * m2 + 4}, {&B.mask, 8 * n2}, {&B.lab[0], 4 * (size_t)n}, {&B.lab[1], 4 * (size_t)n},
              {&B.act[0], 4 * (size_t)n}, {&B.act[1], 4 * (size_t)n}, {&B.loc, 4 * (size_t)n},
              {&B.remap, 4 * (size_t)n}, {&B.old_of, 4 * (size_t)n}, {&B.keep, 4 * ((size_t)n + 1)},
              {&B.pos, 4 * ((size_t)n + 1)}, {&B.slot_cnt, 4 * H},
              {&B.slot_base, 4 * H}, {&B.pivtab, 4 * (size_t)n}, {&B.piv_v, 4 * (size_t)n},
              {&B.piv_bit, 4 * (size_t)n}, {&B.cnt, 4 * (n2 + 1)}, {&B.sums, 4 * (size_t)excl_scan_tiles(n2) + 64},
              {&B.counters, 4 * C_COUNT}, {&B.minv, 4 * (size_t)n}, {&B.parent, 4 * (size_t)n},
              {&w->dirty, 4 * dwords},
              {&w->ctl, sizeof(Ctl)}, {&w->qi, sizeof(QInfo)}, {&w->qword, 2 * sizeof(int64_t)}};
  for (auto &x : need)
    if ((rc = grow(*x.b, x.bytes))) return rc;
  if ((rc = grow_host(B.h_read, 4 * C_COUNT + sizeof(Ctl) + 16))) return rc;
  pasgal_csr t{};
  if (gt) {
    t = *gt;
  } else {
    if ((rc = grow(B.t_off, 4 * ((size_t)n + 1))) || (rc = grow(B.t_tgt, 4 * (size_t)g->m + 4)) ||
        (rc = grow(B.tscratch, 4 * transpose_scratch_elems(g->n))))
      return rc;
    if ((e = launch_transpose(g->offsets, g->targets, g->n, g->m, (int32_t *)B.t_off.p, (int32_t *)B.t_tgt.p,
                              (int32_t *)B.tscratch.p, s)) != hipSuccess)
      return hip_fail(e);
    t.n = g->n;
    t.m = g->m;
    t.offsets = (const int32_t *)B.t_off.p;
    t.targets = (const int32_t *)B.t_tgt.p;
  }
  int32_t *comp = comp_out;
  uint32_t *slot_cnt = (uint32_t *)B.slot_cnt.p;
  uint32_t *slot_base = (uint32_t *)B.slot_base.p;
  uint32_t *piv_v = (uint32_t *)B.piv_v.p, *piv_bit = (uint32_t *)B.piv_bit.p;
  int32_t *pivtab = (int32_t *)B.pivtab.p;
  uint32_t *h_ctr = (uint32_t *)B.h_read.p;
  Ctl *h_ctl = (Ctl *)((uint8_t *)B.h_read.p + 4 * C_COUNT);
  SccRun R{B, s, n, (uint32_t *)((uint8_t *)B.h_read.p + 4 * C_COUNT + sizeof(Ctl))};
  uint32_t *ctr = R.counters();

  VgcArgs a{};
  a.tgt = nullptr;
  a.state = B.mask.p;
  a.dirty = (uint32_t *)w->dirty.p;
  a.qi = (const QInfo *)w->qi.p;
  a.qword = (const int64_t *)w->qword.p;
  a.dirty_words = (int64_t)dwords;
  a.nq = 1;
  for (int i = 0; i < 2; i++) {
    a.fr.v[i] = (uint32_t *)w->fv[i].p;
    a.fr.q[i] = nullptr;
    a.fr.val[i] = (unsigned long long *)w->fval[i].p;
  }
  a.fr.cap = (uint32_t)cap;
  a.start_buf = 0;
  a.tau = o.tau;
  a.max_rounds = 0xFFFFFFFFu;
  a.ring_cap = lg.ring;
  a.stage_cap = lg.stage;
  a.min_chunk = o.min_chunk;
  a.chunks_per_wave = o.cpw;
  a.window = 0;
  a.round_base = 0;
  a.test_first = o.test_first ? 1u : 0u;
  a.timeout_ticks = (long long)o.timeout_ms * (long long)dev_info().wall_khz;
  a.ctl = (Ctl *)w->ctl.p;
  const uint32_t hcap = slice_capacity(m2, o.heavy, cap);
  if ((rc = w->slices.ensure(hcap, false))) return rc;
  w->slices.apply(a, o.heavy, hcap, false);

  auto fail = [&](hipError_t err) { return hip_fail(err); };
  auto read_counters = [&]() -> hipError_t {
    hipError_t x = hipMemcpyAsync(h_ctr, ctr, 4 * C_COUNT, hipMemcpyDeviceToHost, s);
    if (x != hipSuccess) return x;
    return hipStreamSynchronize(s);
  };

  if ((e = hipEventRecord(w->ev0, s)) != hipSuccess) return fail(e);
  if ((e = launch_fill_u32((uint32_t *)comp, n, 0xFFFFFFFFu, s)) != hipSuccess) return fail(e);
  if ((e = launch_fill_u32(R.label(), n, 0u, s)) != hipSuccess) return fail(e);
  hipLaunchKernelGGL(iota_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, R.act());  // every vertex active
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  if ((e = launch_fill_u32(slot_cnt, H, 0u, s)) != hipSuccess) return fail(e);
  if ((e = launch_fill_u32(ctr, C_COUNT, 0u, s)) != hipSuccess) return fail(e);
  // first numbering: every vertex (the caller's G and G^T are numbered by global id)
  R.na = n;
  R.cur = 0;
  if ((e = R.compact_and_pack(PackSrc{g->offsets, g->targets, t.offsets, t.targets, n}, 0, comp)) != hipSuccess)
    return fail(e);

  int64_t trimmed = 0;
  for (int tr = 0; tr < trim_rounds && R.na > 0; tr++) {
    hipLaunchKernelGGL(trim_kernel, dim3(grid_for(R.na)), dim3(256), 0, s, (const int32_t *)R.off2(R.cur), R.na,
                       (const uint32_t *)R.act(), comp, ctr);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    if ((e = read_counters()) != hipSuccess) return fail(e);
    const int64_t now = h_ctr[C_TRIM];
    const int64_t got = now - trimmed;
    trimmed = now;
    // A pass that settles under 1/32 of the vertices is not worth a full
    // repack (nor another pass: the pass after every batch picks up what is
    // left; on the 10M-point 5-NN graph the first pass settles 0.1%). The searches
    // step over the settled vertices left in the packed graph, since a
    // trimmed vertex has no in-arc or no out-arc inside its subproblem and so
    // lies on no path between two others; the first batch's compaction then
    // drops them.
    if (got < std::max<int64_t>(1, (int64_t)n / 32)) break;
    if ((e = R.compact_and_pack(R.packed_src(), R.cur ^ 1, comp)) != hipSuccess) return fail(e);
    R.cur ^= 1;
  }
  // no weak-connectivity split yet: most inputs are one piece until the
  // first batch removes their giant component

  int64_t batches = 0, pivots = 0, rounds = 0, arcs = 0;
  double reach_ms = 0;
  bool pending_reach = false;  // a reach launch whose control block and events are not read yet
  auto collect = [&]() -> bool {  // false if the collected reach launch hit its time limit
    if (!pending_reach) return true;
    pending_reach = false;
    rounds += h_ctl->rounds;
    arcs += (int64_t)h_ctl->stats[ST_ARCS];
    float ms = 0;
    if (hipEventElapsedTime(&ms, w->evk, w->ev1) == hipSuccess) reach_ms += ms;
    (void)hipGetLastError();
    return h_ctl->abort == 0;
  };
  for (uint64_t lo = 0, len = 1; lo < n && R.na > 0; lo += len, len *= 2) {
    uint32_t hi = (uint32_t)std::min<uint64_t>(n, lo + len);
    // with the split on, once the next range of positions is more than twice
    // the number of unsettled vertices, the batch takes every remaining
    // position and walks the active vertices instead (the result does not
    // depend on the order); without the split the few large subproblems left
    // would give at most 64 pivots each per repeat over a range of every
    // unsettled vertex, so the doubling ranges stay
    const bool from_active = split && (uint64_t)hi - lo > 2ull * R.na;
    if (from_active) {
      hi = (uint32_t)n;
      len = n;  // the loop ends after this batch and its repeats
    }
    // every repeat settles at least one vertex of the range (each drawn
    // subproblem's bit-0 pivot), so more repeats than positions is a bug
    for (uint64_t rep = 0;; rep++) {
      if (rep > (uint64_t)(hi - lo)) return PASGAL_EINTERNAL;
      if ((e = launch_fill_u32(ctr, 3, 0u, s)) != hipSuccess) return fail(e);  // NPIV, DEFER, POOL
      if (from_active)
        hipLaunchKernelGGL(select_kernel, dim3(grid_for(R.na)), dim3(256), 0, s, 0u, R.na, n, fh, seed,
                           (const uint32_t *)R.act(), (const int32_t *)comp, (const uint32_t *)R.loc(),
                           (const uint32_t *)R.label(), slot_cnt, piv_v, piv_bit, ctr);
      else
        hipLaunchKernelGGL(select_kernel, dim3(grid_for(hi - lo)), dim3(256), 0, s, (uint32_t)lo, hi, n, fh, seed,
                           (const uint32_t *)nullptr, (const int32_t *)comp, (const uint32_t *)R.loc(),
                           (const uint32_t *)R.label(), slot_cnt, piv_v, piv_bit, ctr);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      if ((e = read_counters()) != hipSuccess) return fail(e);
      if (!collect()) return PASGAL_ETIMEOUT;
      const uint32_t npiv = h_ctr[C_NPIV], ndefer = h_ctr[C_DEFER];
      if (npiv == 0) break;
      batches++;
      pivots += npiv;
      const int pg_grid = (int)((npiv + 255) / 256);
      hipLaunchKernelGGL(reserve_kernel, dim3(pg_grid), dim3(256), 0, s, npiv, (const uint32_t *)piv_v,
                         (const uint32_t *)piv_bit, (const uint32_t *)R.loc(), (const uint32_t *)R.label(),
                         (const uint32_t *)slot_cnt, slot_base, ctr);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      // the searches run on the packed graph of the 2 * na active copies
      const uint64_t nv2 = 2ull * R.na, dw2 = (nv2 + 31) / 32;
      if ((e = launch_fill_u64((unsigned long long *)B.mask.p, nv2, 0ull, s)) != hipSuccess) return fail(e);
      if ((e = launch_fill_u32((uint32_t *)w->dirty.p, dw2, 0u, s)) != hipSuccess) return fail(e);
      if ((e = launch_fill_u32((uint32_t *)w->ctl.p, sizeof(Ctl) / 4, 0u, s)) != hipSuccess) return fail(e);
      hipLaunchKernelGGL(set_query_kernel, dim3(1), dim3(64), 0, s, (QInfo *)w->qi.p, (int64_t *)w->qword.p,
                         (uint32_t)nv2);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      a.off = R.off2(R.cur);
      a.tgt = R.tgt2(R.cur);
      a.dirty_words = (int64_t)dw2;
      hipLaunchKernelGGL(seed_pivots_kernel, dim3(pg_grid), dim3(256), 0, s, a, R.na, npiv, (const uint32_t *)piv_v,
                         (const uint32_t *)piv_bit, (const uint32_t *)R.loc(), (const uint32_t *)R.label(),
                         (const uint32_t *)slot_base, pivtab);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      if ((e = hipEventRecord(w->evk, s)) != hipSuccess) return fail(e);
      if ((e = launch_vgc(KIND_REACH, false, lg.pf, a, lg.grid, lg.block, lg.lds, coop_launch(o), s)) !=
          hipSuccess)
        return fail(e);
      if ((e = hipEventRecord(w->ev1, s)) != hipSuccess) return fail(e);
      if ((e = hipMemcpyAsync(h_ctl, w->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return fail(e);
      pending_reach = true;
      hipLaunchKernelGGL(refine_kernel, dim3(grid_for(R.na)), dim3(256), 0, s, R.na, hmask,
                         (const unsigned long long *)B.mask.p, (const uint32_t *)R.act(), comp, R.label(),
                         (const uint32_t *)slot_base, (const int32_t *)pivtab);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      hipLaunchKernelGGL(clear_slots_kernel, dim3(pg_grid), dim3(256), 0, s, npiv, (const uint32_t *)piv_v,
                         (const uint32_t *)R.loc(), (const uint32_t *)R.label(), slot_cnt);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      if ((e = R.compact_and_pack(R.packed_src(), R.cur ^ 1, comp)) != hipSuccess) return fail(e);
      R.cur ^= 1;
      if (R.na == 0) break;  // every vertex is settled
      if (trim_rounds > 0) {
        hipLaunchKernelGGL(trim_kernel, dim3(grid_for(R.na)), dim3(256), 0, s, (const int32_t *)R.off2(R.cur), R.na,
                           (const uint32_t *)R.act(), comp, ctr);
        if ((e = hipGetLastError()) != hipSuccess) return fail(e);
      }
      if (split && (e = R.split_pieces(comp)) != hipSuccess) return fail(e);
      if (ndefer == 0) break;
    }
  }
  if ((e = read_counters()) != hipSuccess) return fail(e);
  if (!collect()) return PASGAL_ETIMEOUT;
  trimmed = h_ctr[C_TRIM];
  // name each component by its smallest vertex
  int32_t *minv = (int32_t *)B.minv.p;
  if ((e = launch_fill_u32((uint32_t *)minv, n, 0x7FFFFFFFu, s)) != hipSuccess) return fail(e);
  hipLaunchKernelGGL(min_member_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, (const int32_t *)comp, minv);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  hipLaunchKernelGGL(relabel_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, comp, (const int32_t *)minv, ctr);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  if ((e = hipEventRecord(w->ev1, s)) != hipSuccess) return fail(e);
  if ((e = read_counters()) != hipSuccess) return fail(e);
  if (h_ctr[C_UNSETTLED]) return PASGAL_EINTERNAL;
  if (stats) {
    stats->components = h_ctr[C_COMPS];
    stats->trimmed = trimmed;
    stats->pivots = pivots;
    stats->batches = batches;
    stats->rounds = rounds;
    stats->arcs_scanned = arcs;
    float ms = 0;
    if (hipEventElapsedTime(&ms, w->ev0, w->ev1) == hipSuccess) stats->device_ms = ms;
    (void)hipGetLastError();
    stats->reach_ms = reach_ms;
  }
  return PASGAL_OK;
}
