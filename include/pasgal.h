/*
 * pasgal.h -- C ABI of libpasgal.so: frontier-based graph traversal with
 * vertical granularity control (VGC) on one AMD Instinct MI355X (gfx950).
 *
 * Operations (PASGAL, SPAA'24 brief announcement):
 *   - BFS: hop distance of every vertex from one source (Parallel BFS,
 *     Other Algorithms section; frontier framework of Algorithm 1). VGC lets
 *     each frontier vertex run a local search that may visit a vertex more
 *     than once; a vertex is kept for later rounds whenever its hop distance
 *     was lowered, so the result is still the exact hop distance.
 *   - Reachability: for a set of sources, every vertex reachable from each
 *     (reachability search, Parallel SCC section). Visit order is free, so
 *     the local search of VGC (Vertical Granularity Control paragraph) may go
 *     deep. Backward reachability is forward reachability on G^T.
 *   Built on the same kernel: strongly connected components (pasgal_scc),
 *   direction-optimizing BFS (pasgal_bfs_do), single-source shortest paths
 *   (pasgal_sssp), a batched form for many BFS queries over many graphs
 *   (pasgal_batch_*) and a served form with continuous batching
 *   (pasgal_server_*); pasgal_probe_latency measures the dependent-access
 *   time behind a traversal's latency floor.
 *
 * Graph: int32 CSR, G = (V, E), n = |V|, m arcs (Preliminaries). offsets[n+1]
 * with offsets[0] = 0 and offsets[n] = m, targets[m] in [0, n). Self-loops and
 * duplicate arcs are allowed and do not change any result. Rows need not be
 * sorted. All graph and output arrays are DEVICE pointers owned by the caller
 * (typically torch tensors); the library never frees them and keeps no
 * pointer to them after a call returns (server-resident graphs are copied).
 *
 * Errors: every int-returning call returns PASGAL_OK (0) or a negative code.
 * No C++ exception crosses this interface. On PASGAL_EINVAL nothing is
 * written. After any other error the outputs are unspecified but every
 * pointer stayed in bounds, and the library remains usable.
 *
 * Threads: calls on different streams may run concurrently from different
 * host threads; each stream has its own workspace. A persistent traversal
 * launch assumes it has the GPU's compute units to itself (its grid barrier
 * needs every workgroup resident), so two such launches must not overlap,
 * except launches whose pasgal_opts.device_share values add up to at most 100
 * (PASGAL_FLAG_HALF_DEVICE is a share of 50), which are sized to share every
 * compute unit. A launch that cannot become resident ends in PASGAL_ETIMEOUT
 * when its barrier deadline passes; it does not hang.
 */
#ifndef PASGAL_H
#define PASGAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PASGAL_VERSION 1

#define PASGAL_OK 0
#define PASGAL_EINVAL (-1)    /* bad argument: null pointer, n <= 0, m < 0, src or a source out of range, k <= 0 */
#define PASGAL_ENOMEM (-2)    /* device or host allocation failed */
#define PASGAL_EHIP (-3)      /* a HIP runtime call failed; see pasgal_last_hip_error() */
#define PASGAL_ECSR (-4)      /* malformed CSR (only detected with PASGAL_FLAG_VALIDATE) */
#define PASGAL_ECAPACITY (-5) /* a fixed-size structure was too small (never for traversals) */
#define PASGAL_EAGAIN (-6)    /* server: no room for the request right now (non-blocking submit) */
#define PASGAL_ETIMEOUT (-7)  /* a device-side bounded wait expired (e.g. grid barrier); results invalid */
#define PASGAL_ENOTFOUND (-8) /* server: unknown request or graph id */
#define PASGAL_EINTERNAL (-9) /* an internal consistency check failed (a library bug); outputs invalid */

/* Graph in device memory. */
typedef struct pasgal_csr {
  int32_t n;
  int32_t m;
  const int32_t *offsets; /* device, n+1 */
  const int32_t *targets; /* device, m */
} pasgal_csr;

/* Traversal engine. */
#define PASGAL_MODE_VGC 0   /* persistent kernel, rounds of VGC local searches (default) */
#define PASGAL_MODE_PLAIN 1 /* level-synchronous frontier rounds, one launch per round (Algorithm 1, VGC off) */

#define PASGAL_FLAG_VALIDATE 1u /* check the CSR on the device first (O(n+m)) */
#define PASGAL_FLAG_ASYNC 2u    /* do not synchronize the stream before returning (VGC mode only). The
                                   launch's timeout status is read later: by pasgal_wait on the same
                                   stream, or else by the next call on that stream, which then returns
                                   PASGAL_ETIMEOUT (and does nothing else) if the asynchronous launch
                                   timed out */
#define PASGAL_FLAG_PREFETCH 4u   /* VGC: local-queue entries carry their vertex's arc range, loaded while the
                                      relaxing atomic is in flight, instead of when the entry is expanded.
                                      On by default for pasgal_bfs_ex, pasgal_sssp, pasgal_reach_ex and
                                      pasgal_scc when their tau is above 1 (1-8% faster there; at tau 1
                                      no carried range is used) and for the served form's launches
                                      (a lone 8192^2 grid BFS request: 31 against 33.5 ms); off by
                                      default for the batched form, where it measured neutral */
#define PASGAL_FLAG_TEST_FIRST 8u  /* VGC: read a target's state before the atomic and skip the atomic when
                                      the relaxation cannot change it. On by default for pasgal_reach_ex
                                      with k >= 2 sources on graphs with m >= 4n and for pasgal_scc on
                                      graphs with m > 8n (most arcs there offer bits the target already
                                      has); off by default elsewhere, where it measured slower */
#define PASGAL_FLAG_NO_TEST_FIRST 64u /* VGC: never read before the atomic (overrides those defaults) */
#define PASGAL_FLAG_NO_PREFETCH 128u  /* VGC: never carry arc ranges in the local queue (overrides those
                                         defaults and PASGAL_FLAG_PREFETCH) */
#define PASGAL_FLAG_NO_IMPLICATIONS 256u /* reach, VGC: do not use source implications. By default, when new
                                            bits reach the vertex of source j, the sources behind them reach
                                            everything source j reaches, so bit j implies them, and every
                                            expansion propagates the closure of its mask under the
                                            implications known so far (only true reachability facts): the
                                            bits of sources that reach each other then travel together
                                            instead of re-expanding each vertex once per bit */
#define PASGAL_FLAG_HALF_DEVICE 32u /* VGC: size the persistent launch to half of every compute unit (LDS and
                                       wave slots for 2 x blocks_per_cu workgroups per CU; PASGAL_EINVAL if
                                       that many do not fit) and launch it as an ordinary kernel, so that a
                                       second such call on another stream runs beside it: the two grids always
                                       fit the device together. A grid that cannot become resident (a third
                                       launch holding the CUs) ends in PASGAL_ETIMEOUT, never a hang. The same
                                       as pasgal_opts.device_share = 50; two launches whose shares add up to
                                       at most 100 fit the device together in the same way. */

typedef struct pasgal_opts {
  int32_t mode;              /* PASGAL_MODE_VGC or PASGAL_MODE_PLAIN */
  int32_t tau;               /* VGC: vertices a local search expands per frontier vertex before it
                                publishes what is left (the paper's tau); <= 0 selects the entry
                                point's default: 1024, except pasgal_sssp and pasgal_scc on a graph of
                                mean out-degree above 8, where it selects 1. tau = 1 makes every round
                                one BFS level inside the persistent kernel. */
  int32_t wg_size;           /* threads per workgroup: 64..1024, multiple of 64; <= 0 selects 1024 */
  int32_t blocks_per_cu;     /* persistent workgroups per compute unit; <= 0 selects 1 */
  int64_t frontier_capacity; /* entries per frontier buffer; <= 0 selects max(2n, 65536). Smaller values
                                are legal: overflowing entries go to a per-vertex dirty bitmap and are
                                rescanned next round, never dropped. */
  uint32_t flags;            /* PASGAL_FLAG_* */
  int32_t timeout_ms;        /* bound on any device-side wait; <= 0 selects 20000 */
  void *stream;              /* hipStream_t to run on; NULL = the null stream */
  int32_t window;            /* BFS, VGC: round r expands only distances below (r + 1) * window; larger
                                ones wait in the frontier for their round (the paper's remedy of keeping
                                unready vertices out of the current round). 0 selects 32; < 0 = no window. */
  int32_t min_chunk;         /* VGC: frontier entries one wavefront takes at least per local search
                                (1..64; <= 0 selects 1) */
  int32_t heavy_arcs;        /* VGC: a vertex with more out-arcs than this is not scanned by the one
                                wavefront that expands it: its arcs are cut into slices of this many and
                                dealt one per wavefront in the next round (skewed degrees, e.g. RMAT).
                                0 selects 512; < 0 never cuts. */
  int32_t filter_slots;      /* BFS / SSSP, VGC: entries of each wavefront's LDS filter (rounded down to a
                                power of two, at most 4096). It remembers values the wavefront saw in the
                                state and skips a relaxation whose value cannot beat one of them (values
                                only go down, so this never skips a winning relaxation). 0 selects 256,
                                < 0 turns it off. The filter gets at most half of the LDS ring. */
  int32_t chunks_per_wave;   /* VGC: the frontier of a round is cut into this many chunks per wavefront;
                                each wavefront takes one, then claims more from its XCD's share as it
                                finishes, so early finishers take over work. 0 selects 1 (purely
                                static): on the 5-NN graph smaller chunks thin the local searches more
                                than the balancing gains (batched 16-source BFS: 29.6 ms at 1, 42.8 ms
                                at 4). */
  int32_t device_share;      /* VGC: percent (1..99) of every compute unit the persistent launch may take,
                                so that another launch sized to the rest runs beside it on another stream:
                                its workgroups get that share of a CU's LDS and its waves at most that
                                share of the wave slots its registers allow (PASGAL_EINVAL if they do
                                not fit, or if wg_size is not a multiple of 256, i.e. its waves do not
                                spread evenly over a CU's four SIMDs), and it is launched as an ordinary
                                kernel. 0 = the whole device (a cooperative launch), or 50 with
                                PASGAL_FLAG_HALF_DEVICE. */
} pasgal_opts;

/* Counters of one call (schedule dependent, never part of the result). */
typedef struct pasgal_stats {
  int64_t rounds;         /* frontier rounds (VGC) or BFS levels (plain) */
  int64_t expansions;     /* frontier/local entries whose out-arcs were scanned */
  int64_t arcs_scanned;   /* arcs relaxed */
  int64_t relax_success;  /* relaxations that changed the state (lowered a distance / added bits) */
  int64_t published;      /* entries written to a global frontier */
  int64_t overflow;       /* entries that went to the dirty bitmap instead */
  int64_t stale;          /* popped entries skipped because a better value was already known */
  int64_t max_frontier;   /* largest global frontier */
  double device_ms;       /* time on the stream from the state fill to the end of the traversal */
  double kernel_ms;       /* time of the traversal launches alone (VGC: the persistent kernel) */
  int64_t steps;          /* VGC: local-search steps (each pops up to 64 entries; expansions / steps is
                             the average width) */
  int64_t filtered;       /* VGC: relaxations skipped without an atomic (LDS filter, test-first load) */
} pasgal_stats;

void pasgal_opts_default(pasgal_opts *opts);
const char *pasgal_strerror(int code);
int pasgal_last_hip_error(void); /* hipError_t of the last EHIP in this thread */
int pasgal_version(void);

/* Waits for the work the library enqueued on `stream` (a hipStream_t; NULL =
 * the null stream) and reports the status of asynchronous launches there:
 * PASGAL_ETIMEOUT if one of them ended because a bounded device-side wait
 * expired (its results are invalid), else PASGAL_OK. */
int pasgal_wait(void *stream);

/* Releases everything the library owns outside batches and servers: the
 * per-stream workspaces (frontier buffers, bitmaps, control blocks, pinned
 * staging buffers) and their events, on every device, after waiting for each
 * device. Destroy batches and servers first; call from one thread, with no
 * other call in flight. The library stays usable: workspaces are re-created
 * on demand. The Python binding calls it at interpreter exit. */
void pasgal_shutdown(void);

/* BFS from src (Parallel BFS paragraph of the Other Algorithms section: hop
 * distances by the frontier framework of Algorithm 1, here with VGC local
 * searches). dist_out[v] = hop distance from src along out-arcs, or -1 if v
 * is unreachable. dist_out: device, n int32, written entirely. Synchronous on
 * the null stream. PASGAL_EINVAL (nothing written): null pointer, n <= 0,
 * m < 0, src outside [0, n). */
int pasgal_bfs(const pasgal_csr *g, int32_t src, int32_t *dist_out);
/* Same with options and optional counters (stats may be NULL). Runs on
 * opts->stream; returns after the stream is synchronized unless
 * PASGAL_FLAG_ASYNC is set (VGC mode only; stats->device_ms is then 0). */
int pasgal_bfs_ex(const pasgal_csr *g, int32_t src, int32_t *dist_out, const pasgal_opts *opts,
                  pasgal_stats *stats);

/* For callers that cannot allocate memory (code that must not call hipMalloc
 * or an allocator, tight serving loops, harnesses that forbid it): the VGC BFS
 * of pasgal_bfs_ex, bit for bit the same distances, with every library-side
 * buffer (control block, query table, dirty bitmap, slice and frontier
 * buffers) carved from one fixed device array of
 * PASGAL_NOALLOC_SCRATCH_BYTES that each GPU holds until the process ends.
 * The call allocates nothing (no hipMalloc, hipFree, pinned or other
 * allocation); the caller passes dist_out as for pasgal_bfs_ex. Limits:
 * n <= PASGAL_NOALLOC_MAX_VERTICES, else PASGAL_ECAPACITY before anything
 * runs; the frontier capacity is whatever the array holds beside the dirty
 * bitmap (overflow goes to the bitmap, so results stay exact). Every call on a
 * GPU shares that GPU's array and clears what must start at zero: calls are
 * serialized inside the process, and calls that overlap on one GPU from
 * elsewhere would race. Synchronous on opts->stream (PASGAL_FLAG_ASYNC,
 * PASGAL_FLAG_VALIDATE and PASGAL_MODE_PLAIN are rejected with PASGAL_EINVAL);
 * stats->device_ms and kernel_ms are 0. */
#define PASGAL_NOALLOC_SCRATCH_BYTES (64u << 20)
#define PASGAL_NOALLOC_MAX_VERTICES (1 << 28)
int pasgal_bfs_noalloc(const pasgal_csr *g, int32_t src, int32_t *dist_out, const pasgal_opts *opts,
                       pasgal_stats *stats);

/* Single-source shortest paths with non-negative integer arc weights
 * (Parallel SSSP paragraph: the stepping framework with VGC local searches).
 * Round r of the persistent kernel expands only tentative distances below
 * (r + 1) * delta (delta-stepping's buckets over rounds); inside a round each
 * frontier vertex runs a local search of up to tau expansions, relaxing
 * dist[w] = min(dist[w], dist[u] + weight) with atomicMin and re-queueing a
 * vertex whenever its distance drops, so the fixpoint is the exact distance.
 * weights: device, m uint32, weights[e] belongs to arc e (parallel to
 * targets). dist_out: device, n uint32, written entirely; 0xFFFFFFFF marks an
 * unreachable vertex. The caller must keep every shortest distance below
 * 0xFFFFFFFF (larger sums saturate at 0xFFFFFFFE). opts->window is delta:
 * > 0 as given, 0 selects 8 times the mean arc weight (computed on the
 * device), < 0 no buckets (every tentative distance may be expanded at once).
 * PASGAL_MODE_PLAIN runs tau = 1 (one expansion per local search, VGC off) in
 * the same kernel. opts->tau <= 0 selects 1
 * when m > 8n and 1024 otherwise: on dense low-diameter graphs a deep local
 * search mostly lowers distances that a later search lowers again (RMAT-22:
 * 7-8 expansions per vertex and 44-48 ms at tau 1024, 3.8 and 21-23 ms at
 * tau 1), while on sparse high-diameter graphs the bucket bounds the search
 * anyway and tau 1024 is 5-12x faster than tau 1. */
int pasgal_sssp(const pasgal_csr *g, const uint32_t *weights, int32_t src, uint32_t *dist_out,
                const pasgal_opts *opts, pasgal_stats *stats);

/* Direction-optimizing BFS (Parallel BFS paragraph: the paper's BFS also uses
 * the direction optimization of Beamer et al.). Level-synchronous: a level is
 * expanded top-down (frontier vertices relax their out-arcs) while the
 * frontier is small, and bottom-up (every unreached vertex scans its in-arcs
 * and stops at the first in-neighbour in the frontier) while it is large.
 * Suited to low-diameter graphs; on high-diameter graphs use pasgal_bfs_ex.
 * gt: G^T (device CSR of the in-arcs, as pasgal_transpose builds it), or NULL
 * when g is symmetric (every arc u->v has its reverse v->u), in which case g
 * serves as its own transpose; a NULL gt with a directed g gives wrong
 * distances. alpha: go bottom-up when the arcs out of the frontier exceed
 * 1/alpha of the arcs out of unreached vertices (0 selects 100, < 0 never);
 * beta: go back top-down when the frontier holds fewer than n/beta vertices
 * (0 selects 24, < 0 never). Output exactly as pasgal_bfs. Synchronous on
 * opts->stream (PASGAL_FLAG_ASYNC is rejected); opts->mode, tau and window are
 * ignored; opts and stats may be NULL. stats->rounds counts levels. */
int pasgal_bfs_do(const pasgal_csr *g, const pasgal_csr *gt, int32_t src, int32_t *dist_out, int32_t alpha,
                  int32_t beta, const pasgal_opts *opts, pasgal_stats *stats);

/* Direction-optimizing BFS from k sources at once, 1 <= k <= 64 (the served
 * form's batches of BFS and single-source reach requests on low-diameter
 * graphs; not in the paper, which runs one BFS at a time). Every vertex
 * carries one bit per source in 64-bit words (reached so far, reached in the
 * current level, in the next); a top-down level ORs the frontier bits of each
 * frontier vertex into its targets (an atomicOr decides which lane owns each
 * new bit), a bottom-up level has every vertex still missing some bit OR the
 * frontier bits of its in-neighbours until it has them all. The switching
 * rule is pasgal_bfs_do's on the union of the frontiers, with alpha 0
 * selecting 14 for k > 1 (such a bottom-up scan stops only once every
 * missing bit is found; 100 for k = 1). sources: HOST array
 * of k vertex ids (repeats allowed). dist_out: device, k * n int32, row q =
 * hop distances from sources[q] exactly as pasgal_bfs, or NULL. reach_out:
 * device, n uint64, bit q set iff sources[q] reaches v, or NULL. gt, alpha,
 * beta, opts, stats as for pasgal_bfs_do. PASGAL_EINVAL (nothing written): k
 * outside [1, 64], a source outside [0, n), a null graph pointer. */
int pasgal_bfs_do_multi(const pasgal_csr *g, const pasgal_csr *gt, int32_t k, const int32_t *sources,
                        int32_t *dist_out, uint64_t *reach_out, int32_t alpha, int32_t beta, const pasgal_opts *opts,
                        pasgal_stats *stats);

/* Multi-source reachability (Parallel SCC section: a reachability search from
 * a vertex finds every vertex it reaches; the sources form the initial
 * frontier F0 of Algorithm 1). sources: DEVICE array of k int32 vertex ids
 * (repeats allowed), k >= 1; the call reads it on its stream, after the
 * stream's earlier work, with one small device-to-host copy and a wait, and
 * checks it before anything is written. label_out: device, n * W uint64 with
 * W = ceil(k/64); bit (i % 64) of label_out[v*W + i/64] is set iff
 * sources[i] reaches v (v = sources[i] included). Written entirely.
 * PASGAL_EINVAL (nothing written): null pointer, k <= 0, a source outside
 * [0, n). Synchronous on the null stream. */
int pasgal_reach(const pasgal_csr *g, const int32_t *sources, int32_t k, uint64_t *label_out);
/* Same with options and optional counters, on opts->stream; with k > 64 the
 * mask words are computed one after the other (PASGAL_FLAG_ASYNC is then
 * rejected). */
int pasgal_reach_ex(const pasgal_csr *g, const int32_t *sources, int32_t k, uint64_t *label_out,
                    const pasgal_opts *opts, pasgal_stats *stats);

/* G^T (Parallel SCC section: the backward search from a pivot follows
 * in-arcs, i.e. it is a forward search on G^T). t_offsets device n+1,
 * t_targets device m, owned by the caller. Row v of G^T lists every u with an
 * arc u->v, once per arc; the order inside a row is unspecified. Synchronous
 * on opts->stream (opts may be NULL). PASGAL_EINVAL (nothing written): null
 * pointer, n <= 0, m < 0. */
int pasgal_transpose(const pasgal_csr *g, int32_t *t_offsets, int32_t *t_targets, const pasgal_opts *opts);

/* Device-side CSR check (monotone offsets, offsets[0]=0, offsets[n]=m,
 * targets in range). Returns PASGAL_OK or PASGAL_ECSR. */
int pasgal_validate(const pasgal_csr *g, const pasgal_opts *opts);

/* Memory-latency probe (measurement support; Experimental Results: a
 * traversal's rounds follow the diameter, so its time has a floor of one
 * dependent memory access per level): the mean time of one dependent access.
 * One lane follows a random single cycle through a device buffer of
 * 2^floor(log2(bytes / 4)) uint32 slots (built on the device; each slot holds
 * the next slot's index), `steps` times, timed by the device wall clock. A
 * traversal from a source of eccentricity e makes at least e such accesses
 * one after the other, so it takes at least e * ns_per_hop.
 * kind: PASGAL_PROBE_LOAD plain load (cached), PASGAL_PROBE_COHERENT
 * agent-scope relaxed atomic load (how the kernels read data other
 * workgroups write), PASGAL_PROBE_ATOMIC agent-scope atomic add of 0 (a
 * relaxation's round trip). bytes in [4096, 2^32], steps in [1, 2^24].
 * The buffer is allocated and freed inside the call. Synchronous on
 * opts->stream (opts may be NULL). PASGAL_EINVAL: null ns_per_hop or an
 * argument out of range (nothing is run). */
#define PASGAL_PROBE_LOAD 0
#define PASGAL_PROBE_COHERENT 1
#define PASGAL_PROBE_ATOMIC 2
int pasgal_probe_latency(int64_t bytes, int32_t steps, int32_t kind, double *ns_per_hop, const pasgal_opts *opts);

/* --------------------------------------------------------------------- SCC --
 * Strongly connected components (Parallel SCC section): reachability searches
 * from batches of pivots. Pivots are taken in a random vertex order, in
 * batches of 1, 2, 4, ... positions (a settled vertex is skipped). For every
 * pivot p a forward search (along out-arcs) and a backward search (along
 * in-arcs) run; a vertex found both ways from p belongs to p's component.
 * Every other vertex moves to the subproblem named by its old subproblem and
 * the sets of pivots that reached it forward and backward; vertices of one
 * component always agree on these, and later searches stay inside one
 * subproblem. All forward and backward searches of a batch run together in
 * one persistent VGC reach launch (PASGAL_MODE_PLAIN: tau = 1, one BFS level
 * per round, in the same launch). Trimming, an addition to the paper's
 * description: a vertex with no in-arc or no out-arc left inside its
 * subproblem is a component by itself. After every batch the still
 * unsettled vertices are renumbered 0..na-1, and every later pass (packing,
 * searches, refinement, trimming, splitting) covers only them. */
typedef struct pasgal_scc_stats {
  int64_t components;   /* strongly connected components */
  int64_t trimmed;      /* vertices settled by trimming */
  int64_t pivots;       /* pivots whose forward and backward searches ran */
  int64_t batches;      /* reach launches (pivot batches, repeats included) */
  int64_t rounds;       /* VGC rounds summed over the reach launches */
  int64_t arcs_scanned; /* arcs relaxed by the searches */
  double device_ms;     /* whole call on the stream, transpose included when built here */
  double reach_ms;      /* inside the reach launches */
} pasgal_scc_stats;

#define PASGAL_SCC_NO_SPLIT 1u /* keep subproblems whole instead of cutting each into its weakly connected
                                  pieces after every batch (an addition to the paper's description: a
                                  component never spans two pieces, and small pieces each get their own
                                  64 pivots per batch) */

typedef struct pasgal_scc_opts {
  int32_t trim_rounds; /* trimming passes before the first batch (the loop stops after a pass that
                          settles fewer than n/1024 vertices), plus one pass after every batch; < 0
                          selects 1 (every pass before the first batch also renumbers and repacks,
                          and the pass after each batch catches what a second one would), 0
                          disables trimming */
  uint32_t flags;      /* PASGAL_SCC_* */
  uint32_t seed;       /* key of the random pivot order; 0 selects a fixed default. The result does not
                          depend on it. */
  int32_t reserved;    /* 0 */
} pasgal_scc_opts;

/* comp_out: device, n int32, written entirely: comp_out[v] = the smallest
 * vertex id of v's strongly connected component (so comp_out[v] <= v, and
 * comp_out[v] == v for exactly one vertex per component). gt: G^T as
 * pasgal_transpose builds it, or NULL to build it inside the call (4(n+1)+4m
 * bytes more). scc_opts, opts and stats may be NULL (defaults). Limits:
 * n < 2^30 and m < 2^30 (the forward and backward graphs are packed into one
 * CSR of 2n vertices). Device memory used: about 80n + 16m bytes plus the
 * frontier buffers (24 bytes per entry, 4n entries by default). Synchronous
 * on opts->stream (PASGAL_FLAG_ASYNC is rejected). */
int pasgal_scc(const pasgal_csr *g, const pasgal_csr *gt, int32_t *comp_out, const pasgal_scc_opts *scc_opts,
               const pasgal_opts *opts, pasgal_scc_stats *stats);

/* ------------------------------------------------------------ batched form --
 * Many BFS queries over many graphs in ONE persistent launch, captured once
 * in a hipGraph and replayed. The graphs are laid out as one packed CSR over
 * the disjoint union of their vertex sets (graph g owns global vertices
 * [vbase[g], vbase[g+1]); targets hold global ids). Query j runs on graph
 * q_graph[j] from local vertex q_source[j] and writes its n_g distances to
 * dist_out[q_out[j] .. q_out[j] + n_g). Output regions may not overlap. */
typedef struct pasgal_batch pasgal_batch;

typedef struct pasgal_batch_desc {
  pasgal_csr packed;       /* device CSR of the packed graphs */
  int32_t ngraphs;
  const int32_t *vbase;    /* HOST, ngraphs+1, vbase[0] = 0, vbase[ngraphs] = packed.n */
  int32_t nqueries;
  const int32_t *q_graph;  /* HOST, nqueries */
  const int32_t *q_source; /* HOST, nqueries, local ids */
  const int64_t *q_out;    /* HOST, nqueries, element offsets into dist_out */
  int32_t *dist_out;       /* device */
  int64_t dist_len;        /* elements in dist_out (bounds check) */
} pasgal_batch_desc;

#define PASGAL_BATCH_AUTOTUNE 1u /* choose tau, wg_size, blocks_per_cu, capacity by timed probes */

/* Builds the batch (uploads query tables, sizes the workspace, optionally
 * autotunes, captures the hipGraph). opts supplies the starting parameters and
 * the stream; flags may include PASGAL_BATCH_AUTOTUNE. */
int pasgal_batch_create(const pasgal_batch_desc *desc, const pasgal_opts *opts, uint32_t batch_flags,
                        pasgal_batch **out);
/* Replays the captured launch: every query's distances are rewritten. Returns
 * after the stream is synchronized. stats may be NULL. */
int pasgal_batch_run(pasgal_batch *b, pasgal_stats *stats);
/* The parameters the batch runs with (after autotuning). */
int pasgal_batch_config(const pasgal_batch *b, pasgal_opts *chosen);
void pasgal_batch_destroy(pasgal_batch *b);

/* ------------------------------------------------------------- served form --
 * A request loop over graphs kept resident in device memory. Requests (BFS
 * from one source, or reachability from up to 64 sources) are admitted while
 * the per-request state fits the memory budget and a slot is free, and join
 * the running traversal at the next round boundary (continuous batching): the
 * device advances every admitted request in shared persistent launches of a
 * bounded number of rounds, retiring finished ones and admitting new ones
 * between launches. Results are copied into the caller's device buffer. */
typedef struct pasgal_server pasgal_server;

typedef struct pasgal_server_opts {
  int64_t memory_budget;   /* bytes of request state (result slots + bitmaps); <= 0: 1/4 of free HBM */
  int32_t max_slots;       /* concurrent requests; <= 0 selects 256 */
  int32_t slice_rounds;    /* rounds per launch before re-admitting; <= 0 selects 32 */
  int32_t tau;             /* <= 0 selects 256 */
  int32_t wg_size;         /* <= 0 selects 1024 */
  int32_t blocks_per_cu;   /* <= 0 selects 1 */
  int64_t frontier_capacity; /* per kind; <= 0 selects 64M entries */
  int32_t timeout_ms;
  int32_t window;          /* BFS distance window per round (see pasgal_opts.window); < 0 selects none,
                              0 selects 32 */
  uint32_t flags;          /* PASGAL_FLAG_TEST_FIRST / PASGAL_FLAG_NO_TEST_FIRST: read a target's state
                              before each relaxing atomic in every launch. Default: on in a launch that
                              holds a request on a graph with mean out-degree above 8 (there most arcs
                              reach vertices that already have the value, and a plain read is cheaper
                              than the atomic), off otherwise. PASGAL_SERVER_FIXED_SLICES,
                              PASGAL_SERVER_NO_DIRECTION_OPT: see there. Other bits must be 0. */
  int32_t reserved;        /* 0 */
} pasgal_server_opts;

/* Server flag: every launch runs at most slice_rounds rounds. By default a launch made while exactly one
   request is resident and none is queued runs the single-query kernel until that request finishes or
   another request is submitted (the launch polls a word in coherent host memory once per round and ends
   at the next round boundary, handing its frontier back to the multi-query layout), so that a request
   served alone pays no per-slice host round trips and no multi-query overhead. */
#define PASGAL_SERVER_FIXED_SLICES 65536u
/* Server flag: every request goes through the batched VGC launches. By default a graph added with mean
   out-degree above 8 (m > 8n: low diameter, where top-down levels scan most arcs) gets a copy of itself
   and of its transpose in server memory (4(n+1) + 4m bytes each, built once by pasgal_server_add_graph),
   and its BFS requests and single-source reach requests are served in batches of up to 64 per graph
   by the multi-source direction-optimizing BFS (pasgal_bfs_do_multi, default alpha and beta) on a host
   thread and stream of the server's own; its levels and the batched launches take turns on the device.
   A reach request gets bit 0 set where its source arrives. Their completions report levels as rounds.
   Reach requests with several sources always use the batched launches. */
#define PASGAL_SERVER_NO_DIRECTION_OPT 131072u

#define PASGAL_REQ_BFS 0
#define PASGAL_REQ_REACH 1

typedef struct pasgal_request {
  int32_t graph;          /* id from pasgal_server_add_graph */
  int32_t kind;           /* PASGAL_REQ_BFS or PASGAL_REQ_REACH */
  int32_t nsources;       /* BFS: 1; REACH: 1..64 */
  int32_t sources[64];    /* local vertex ids */
  void *out;              /* device: int32[n] (BFS) or uint64[n] (REACH); may be NULL (result dropped) */
  uint64_t tag;           /* caller's cookie, echoed in the completion */
} pasgal_request;

typedef struct pasgal_completion {
  int64_t id;             /* from pasgal_server_submit */
  uint64_t tag;
  int32_t status;         /* PASGAL_OK or an error code */
  int32_t graph;
  double t_submit_ms;     /* host monotonic clock, ms */
  double t_admit_ms;
  double t_done_ms;
  int64_t rounds;         /* rounds the request was resident for */
} pasgal_completion;

/* Starts the server's host threads (the request loop and the direction-optimizing thread) and streams;
 * opts may be NULL (all defaults). PASGAL_EINVAL: unknown flag bits, reserved != 0, max_slots > 4096. */
int pasgal_server_create(const pasgal_server_opts *opts, pasgal_server **out);
/* Copies the graph into server-owned device memory; returns its id. */
int pasgal_server_add_graph(pasgal_server *s, const pasgal_csr *g, int32_t *graph_id);
/* Queues a request; id receives its number. Never blocks: PASGAL_EAGAIN when
 * the submission queue is full. */
int pasgal_server_submit(pasgal_server *s, const pasgal_request *req, int64_t *id);
/* Takes up to max finished requests; *count receives how many. */
int pasgal_server_poll(pasgal_server *s, pasgal_completion *out, int32_t max, int32_t *count);
/* Blocks until every submitted request has completed (or timeout_ms passes). */
int pasgal_server_drain(pasgal_server *s, int32_t timeout_ms);
/* Current queue depth, admitted requests and bytes of state in use. */
int pasgal_server_load(pasgal_server *s, int32_t *queued, int32_t *active, int64_t *bytes_in_use);
void pasgal_server_destroy(pasgal_server *s);

#ifdef __cplusplus
}
#endif

#endif /* PASGAL_H */
