/*
 * graphgen.c -- seeded synthetic graph generators emitting int32 CSR.
 *
 * Input tooling only: nothing here traverses a graph. Both the CPU oracle's
 * tests and the GPU path consume what these functions write, so this file
 * holds none of the traversal arithmetic (no distances, no reachability, no
 * transposition).
 *
 * CSR convention (matches the paper's G=(V,E), n=|V|, m arcs, Preliminaries):
 *   offsets[n+1] int32, offsets[0]=0, offsets[n]=m; targets[m] int32.
 *   Every generator here emits rows sorted ascending by target, without
 *   self-loops and without duplicate arcs. Undirected graphs are stored
 *   symmetrised (each edge as two arcs), as the paper's m counts them.
 *
 * Randomness: one counter-based stream per purpose. rng64(seed, stream, i)
 * applies the SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014) to a key
 * derived from (seed, stream) plus (i+1) times the golden-ratio increment, so
 * any element is reproducible without sequential state and results do not
 * depend on the thread count.
 *
 * Memory returned through gg_graph is malloc'ed here and released by gg_free.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct gg_graph {
  int64_t n;
  int64_t m;
  int32_t *offsets; /* n+1 */
  int32_t *targets; /* m */
} gg_graph;

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t gg_rng64(uint64_t seed, uint64_t stream, uint64_t i) {
  uint64_t key = mix64(seed * 0xD1B54A32D192ED03ULL + stream * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL);
  return mix64(key + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

/* uniform double in [0,1) with 53 random bits */
static double u01(uint64_t seed, uint64_t stream, uint64_t i) {
  return (double)(gg_rng64(seed, stream, i) >> 11) * (1.0 / 9007199254740992.0);
}

void gg_free(gg_graph *g) {
  if (!g) return;
  free(g->offsets);
  free(g->targets);
  g->offsets = NULL;
  g->targets = NULL;
  g->n = g->m = 0;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Sort each row, drop self-loops and duplicates, compact in place.
 * deg must hold the current row sizes inside the fixed slots start[v]. */
static int compact_rows(int64_t n, const int64_t *start, int64_t *deg, int32_t *buf, gg_graph *g) {
  int64_t v;
#pragma omp parallel for schedule(dynamic, 4096)
  for (v = 0; v < n; v++) {
    int32_t *row = buf + start[v];
    int64_t d = deg[v];
    if (d > 1) qsort(row, (size_t)d, sizeof(int32_t), cmp_i32);
    int64_t w = 0;
    for (int64_t i = 0; i < d; i++) {
      if (row[i] == (int32_t)v) continue;
      if (w > 0 && row[w - 1] == row[i]) continue;
      row[w++] = row[i];
    }
    deg[v] = w;
  }
  int64_t m = 0;
  for (v = 0; v < n; v++) m += deg[v];
  if (m > 2147483647LL) return -2;
  g->n = n;
  g->m = m;
  g->offsets = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  g->targets = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  if (!g->offsets || !g->targets) return -1;
  int64_t acc = 0;
  for (v = 0; v < n; v++) {
    g->offsets[v] = (int32_t)acc;
    acc += deg[v];
  }
  g->offsets[n] = (int32_t)acc;
#pragma omp parallel for schedule(dynamic, 4096)
  for (v = 0; v < n; v++) memcpy(g->targets + g->offsets[v], buf + start[v], sizeof(int32_t) * (size_t)deg[v]);
  return 0;
}

/* ---------------------------------------------------------------- grids -- */

/* a x b 4-neighbour grid, vertex id = r*b + c. torus!=0 wraps both axes.
 * Undirected (symmetrised). */
int gg_grid(int64_t a, int64_t b, int torus, gg_graph *g) {
  memset(g, 0, sizeof(*g));
  if (a <= 0 || b <= 0 || a * b > 2147483647LL) return -3;
  int64_t n = a * b;
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * n));
  if (!start || !deg || !buf) { free(start); free(deg); free(buf); return -1; }
  int64_t v;
#pragma omp parallel for schedule(static)
  for (v = 0; v < n; v++) {
    int64_t r = v / b, c = v % b, d = 0;
    int32_t *row = buf + 4 * v;
    start[v] = 4 * v;
    if (r > 0) row[d++] = (int32_t)(v - b);
    else if (torus) row[d++] = (int32_t)((a - 1) * b + c);
    if (c > 0) row[d++] = (int32_t)(v - 1);
    else if (torus) row[d++] = (int32_t)(r * b + (b - 1));
    if (c < b - 1) row[d++] = (int32_t)(v + 1);
    else if (torus) row[d++] = (int32_t)(r * b);
    if (r < a - 1) row[d++] = (int32_t)(v + b);
    else if (torus) row[d++] = (int32_t)c;
    deg[v] = d;
  }
  int rc = compact_rows(n, start, deg, buf, g);
  free(start); free(deg); free(buf);
  return rc;
}

/* ----------------------------------------------------- simple families -- */

/* kind: 0 = directed chain i->i+1, 1 = undirected chain, 2 = directed cycle,
 * 3 = undirected cycle, 4 = complete digraph, 5 = undirected star (centre 0),
 * 6 = no arcs */
int gg_simple(int32_t kind, int64_t n, gg_graph *g) {
  memset(g, 0, sizeof(*g));
  if (n <= 0 || n > 2147483647LL) return -3;
  int64_t cap = 0;
  switch (kind) {
    case 0: cap = 1; break;
    case 1: cap = 2; break;
    case 2: cap = 1; break;
    case 3: cap = 2; break;
    case 4: cap = n - 1; break;
    case 5: cap = 1; break;
    case 6: cap = 0; break;
    default: return -3;
  }
  if (kind == 4 && n * (n - 1) > 2147483647LL) return -3;
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *deg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int64_t total = (kind == 5) ? 2 * (n - 1) : cap * n;
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  if (!start || !deg || !buf) { free(start); free(deg); free(buf); return -1; }
  if (kind == 5) {
    start[0] = 0;
    for (int64_t v = 1; v < n; v++) start[v] = (n - 1) + (v - 1);
    for (int64_t v = 1; v < n; v++) {
      buf[start[0] + deg[0]++] = (int32_t)v;
      buf[start[v] + deg[v]++] = 0;
    }
  } else {
    for (int64_t v = 0; v < n; v++) {
      start[v] = cap * v;
      int32_t *row = buf + start[v];
      int64_t d = 0;
      if (kind == 0 || kind == 1) {
        if (kind == 1 && v > 0) row[d++] = (int32_t)(v - 1);
        if (v + 1 < n) row[d++] = (int32_t)(v + 1);
      } else if (kind == 2 || kind == 3) {
        if (n > 1) {
          row[d++] = (int32_t)((v + 1) % n);
          if (kind == 3) row[d++] = (int32_t)((v + n - 1) % n);
        }
      } else if (kind == 4) {
        for (int64_t w = 0; w < n; w++)
          if (w != v) row[d++] = (int32_t)w;
      }
      deg[v] = d;
    }
  }
  int rc = compact_rows(n, start, deg, buf, g);
  free(start); free(deg); free(buf);
  return rc;
}

/* Random digraph: m0 arcs with uniform endpoints (self-loops and repeats are
 * then removed, so m <= m0). symmetric!=0 stores both directions. */
int gg_random(int64_t n, int64_t m0, int symmetric, uint64_t seed, gg_graph *g) {
  memset(g, 0, sizeof(*g));
  if (n <= 0 || m0 < 0 || n > 2147483647LL) return -3;
  int64_t mult = symmetric ? 2 : 1;
  int64_t *deg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!deg || !start) { free(deg); free(start); return -1; }
  for (int64_t e = 0; e < m0; e++) {
    int64_t u = (int64_t)(gg_rng64(seed, 100, 2 * e) % (uint64_t)n);
    int64_t v = (int64_t)(gg_rng64(seed, 100, 2 * e + 1) % (uint64_t)n);
    deg[u]++;
    if (symmetric) deg[v]++;
  }
  int64_t acc = 0;
  for (int64_t v = 0; v < n; v++) { start[v] = acc; acc += deg[v]; deg[v] = 0; }
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(acc > 0 ? acc : 1));
  if (!buf) { free(deg); free(start); return -1; }
  (void)mult;
  for (int64_t e = 0; e < m0; e++) {
    int64_t u = (int64_t)(gg_rng64(seed, 100, 2 * e) % (uint64_t)n);
    int64_t v = (int64_t)(gg_rng64(seed, 100, 2 * e + 1) % (uint64_t)n);
    buf[start[u] + deg[u]++] = (int32_t)v;
    if (symmetric) buf[start[v] + deg[v]++] = (int32_t)u;
  }
  int rc = compact_rows(n, start, deg, buf, g);
  free(start); free(deg); free(buf);
  return rc;
}

/* ------------------------------------------------------------------ kNN -- */

/* Points: X_i = rng64(seed,0,2i)>>40 and Y_i = rng64(seed,0,2i+1)>>40, 24-bit
 * integers; the point is (X_i, Y_i) * 2^-24 in [0,1)^2. Squared distances are
 * computed exactly in int64 on the integer coordinates. */
void gg_points(int64_t n, uint64_t seed, int32_t *xy /* 2n */) {
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < n; i++) {
    xy[2 * i] = (int32_t)(gg_rng64(seed, 0, 2 * (uint64_t)i) >> 40);
    xy[2 * i + 1] = (int32_t)(gg_rng64(seed, 0, 2 * (uint64_t)i + 1) >> 40);
  }
}

/* Directed k-NN graph: arc i -> j for each of the k nearest other points j,
 * nearest by exact squared distance, ties to the smaller index. Exact search
 * through a uniform bucket grid, widening Chebyshev rings until no unvisited
 * cell can hold a closer (or equal-distance) point. Rows sorted by target. */
typedef struct { uint64_t key; int64_t idx; } zkey;
static int cmp_zkey(const void *a, const void *b) {
  const zkey *x = (const zkey *)a, *y = (const zkey *)b;
  if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
  return (x->idx > y->idx) - (x->idx < y->idx);
}
static uint64_t spread24(uint64_t v) { /* bit i -> bit 2i */
  uint64_t r = 0;
  for (int i = 0; i < 24; i++) r |= ((v >> i) & 1ULL) << (2 * i);
  return r;
}

/* Point layout of the k-NN generator. order 0: vertex i is the i-th drawn
 * point. order 1: the drawn points are renumbered along the Z-order (Morton)
 * curve of their 24-bit coordinates, ties by draw index -- the spatially
 * sorted layout point-cloud data is usually stored in. */
void gg_points_ordered(int64_t n, uint64_t seed, int order, int32_t *xy) {
  gg_points(n, seed, xy);
  if (order != 1) return;
  zkey *z = (zkey *)malloc(sizeof(zkey) * (size_t)n);
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * n));
  if (!z || !tmp) { free(z); free(tmp); return; }
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < n; i++) {
    z[i].key = spread24((uint64_t)xy[2 * i]) | (spread24((uint64_t)xy[2 * i + 1]) << 1);
    z[i].idx = i;
  }
  qsort(z, (size_t)n, sizeof(zkey), cmp_zkey);
  for (i = 0; i < n; i++) { tmp[2 * i] = xy[2 * z[i].idx]; tmp[2 * i + 1] = xy[2 * z[i].idx + 1]; }
  memcpy(xy, tmp, sizeof(int32_t) * (size_t)(2 * n));
  free(z); free(tmp);
}

int gg_knn(int64_t n, int32_t k, uint64_t seed, int layout, gg_graph *g) {
  memset(g, 0, sizeof(*g));
  if (n <= 0 || k <= 0 || k >= n || k > 64 || n * k > 2147483647LL) return -3;
  int32_t *xy = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * n));
  if (!xy) return -1;
  gg_points_ordered(n, seed, layout, xy);
  int64_t G = (int64_t)floor(sqrt((double)n / 2.0));
  if (G < 1) G = 1;
  if (G > 16384) G = 16384;
  int64_t ncell = G * G;
  int64_t *cstart = (int64_t *)calloc((size_t)(ncell + 1), sizeof(int64_t));
  int32_t *cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!cstart || !cell_of || !order) { free(xy); free(cstart); free(cell_of); free(order); return -1; }
  for (int64_t i = 0; i < n; i++) {
    int64_t cx = ((int64_t)xy[2 * i] * G) >> 24, cy = ((int64_t)xy[2 * i + 1] * G) >> 24;
    cell_of[i] = (int32_t)(cy * G + cx);
    cstart[cell_of[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; c++) cstart[c + 1] += cstart[c];
  {
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    if (!cur) { free(xy); free(cstart); free(cell_of); free(order); return -1; }
    memcpy(cur, cstart, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; i++) order[cur[cell_of[i]]++] = (int32_t)i; /* ascending ids per cell */
    free(cur);
  }
  /* a cell at Chebyshev ring distance >= r+1 from the home cell is at least
   * r * floor(2^24 / G) away along one axis */
  int64_t wmin = ((int64_t)1 << 24) / G;
  g->n = n;
  g->m = n * k;
  g->offsets = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  g->targets = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n * k));
  if (!g->offsets || !g->targets) { free(xy); free(cstart); free(cell_of); free(order); gg_free(g); return -1; }
  int failed = 0;
  int64_t i;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : failed)
  for (i = 0; i < n; i++) {
    int64_t bd[64];
    int32_t bi[64];
    int cnt = 0;
    int64_t X = xy[2 * i], Y = xy[2 * i + 1];
    int64_t hx = (X * G) >> 24, hy = (Y * G) >> 24;
    for (int64_t r = 0; r <= G; r++) {
      for (int64_t cy = hy - r; cy <= hy + r; cy++) {
        if (cy < 0 || cy >= G) continue;
        int64_t step = (cy == hy - r || cy == hy + r) ? 1 : 2 * r;
        if (step == 0) step = 1;
        for (int64_t cx = hx - r; cx <= hx + r; cx += step) {
          if (cx < 0 || cx >= G) continue;
          int64_t c = cy * G + cx;
          for (int64_t p = cstart[c]; p < cstart[c + 1]; p++) {
            int32_t j = order[p];
            if (j == (int32_t)i) continue;
            int64_t dx = (int64_t)xy[2 * j] - X, dy = (int64_t)xy[2 * j + 1] - Y;
            int64_t d = dx * dx + dy * dy;
            /* keep the k best by (d, j) in ascending order */
            if (cnt == k && (d > bd[k - 1] || (d == bd[k - 1] && j > bi[k - 1]))) continue;
            int pos = (cnt < k) ? cnt++ : k - 1;
            while (pos > 0 && (bd[pos - 1] > d || (bd[pos - 1] == d && bi[pos - 1] > j))) {
              bd[pos] = bd[pos - 1];
              bi[pos] = bi[pos - 1];
              pos--;
            }
            bd[pos] = d;
            bi[pos] = j;
          }
        }
      }
      int64_t bound = r * wmin;
      if (cnt == k && bd[k - 1] < bound * bound) break;
    }
    if (cnt < k) failed = 1;
    /* rows sorted by target id */
    for (int a = 1; a < cnt; a++) {
      int32_t t = bi[a];
      int b = a;
      while (b > 0 && bi[b - 1] > t) { bi[b] = bi[b - 1]; b--; }
      bi[b] = t;
    }
    for (int a = 0; a < k; a++) g->targets[i * k + a] = (a < cnt) ? bi[a] : 0;
  }
  for (int64_t v = 0; v <= n; v++) g->offsets[v] = (int32_t)(v * k);
  free(xy); free(cstart); free(cell_of); free(order);
  if (failed) { gg_free(g); return -4; }
  return 0;
}

/* ------------------------------------------------------------ road grid -- */

/* side x side road-like directed grid.
 *  - Undirected grid edges in canonical order: horizontal (r,c)-(r,c+1)
 *    row-major, then vertical (r,c)-(r+1,c) row-major; edge index e.
 *  - Edge e is deleted iff u01(seed,1,e) < p_del.
 *  - A survivor is kept both ways iff u01(seed,2,e) < p_both, otherwise one
 *    direction: low id -> high id iff bit 0 of rng64(seed,3,e) is 0.
 *  - Diagonal shortcut from vertex v=(r,c), r < side-1, iff u01(seed,4,v) <
 *    p_diag: to (r+1, c-1) if bit 0 of rng64(seed,5,v) is 0 else (r+1, c+1);
 *    the in-bounds one at the left/right border. Same direction rule with
 *    streams 6 (both ways) and 7 (which way).
 */
int gg_road(int64_t side, double p_del, double p_both, double p_diag, uint64_t seed, gg_graph *g) {
  memset(g, 0, sizeof(*g));
  if (side < 2 || side * side > 2147483647LL) return -3;
  int64_t n = side * side;
  int64_t nh = side * (side - 1); /* horizontal edges */
  int64_t ne = 2 * nh;
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *deg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(6 * n));
  if (!start || !deg || !buf) { free(start); free(deg); free(buf); return -1; }
  for (int64_t v = 0; v < n; v++) start[v] = 6 * v; /* <= 4 grid + 2 diagonal out-arcs */
  /* Each vertex collects its own out-arcs: iterate per vertex over incident
   * edges so the fill is race-free and thread-count independent. */
  int64_t v;
#pragma omp parallel for schedule(static)
  for (v = 0; v < n; v++) {
    int64_t r = v / side, c = v % side, d = 0;
    int32_t *row = buf + 6 * v;
    /* incident grid edges: (edge index, other endpoint) */
    int64_t eidx[4], oth[4];
    int ninc = 0;
    if (c > 0) { eidx[ninc] = r * (side - 1) + (c - 1); oth[ninc++] = v - 1; }
    if (c < side - 1) { eidx[ninc] = r * (side - 1) + c; oth[ninc++] = v + 1; }
    if (r > 0) { eidx[ninc] = nh + (r - 1) * side + c; oth[ninc++] = v - side; }
    if (r < side - 1) { eidx[ninc] = nh + r * side + c; oth[ninc++] = v + side; }
    for (int t = 0; t < ninc; t++) {
      int64_t e = eidx[t], w = oth[t];
      if (u01(seed, 1, (uint64_t)e) < p_del) continue;
      int out;
      if (u01(seed, 2, (uint64_t)e) < p_both) out = 1;
      else {
        int low_to_high = (gg_rng64(seed, 3, (uint64_t)e) & 1) == 0;
        out = (v < w) ? low_to_high : !low_to_high;
      }
      if (out) row[d++] = (int32_t)w;
    }
    /* diagonal shortcuts touching v: the one v originates, and those that
     * originate at the row above and land on v */
    int64_t cand[3];
    int nc = 0;
    if (r < side - 1) cand[nc++] = v;                 /* v as origin */
    if (r > 0) {
      if (c > 0) cand[nc++] = v - side - 1;           /* origin (r-1,c-1) */
      if (c < side - 1) cand[nc++] = v - side + 1;    /* origin (r-1,c+1) */
    }
    for (int t = 0; t < nc; t++) {
      int64_t o = cand[t];
      if (u01(seed, 4, (uint64_t)o) >= p_diag) continue;
      int64_t orr = o / side, oc = o % side, tc;
      int left = (gg_rng64(seed, 5, (uint64_t)o) & 1) == 0;
      if (oc == 0) left = 0;
      if (oc == side - 1) left = 1;
      tc = left ? oc - 1 : oc + 1;
      int64_t dst = (orr + 1) * side + tc;
      int64_t w;
      if (o == v) w = dst;
      else if (dst == v) w = o;
      else continue;
      int out;
      if (u01(seed, 6, (uint64_t)o) < p_both) out = 1;
      else {
        int low_to_high = (gg_rng64(seed, 7, (uint64_t)o) & 1) == 0;
        out = (v < w) ? low_to_high : !low_to_high;
      }
      if (out) row[d++] = (int32_t)w;
    }
    deg[v] = d;
  }
  (void)ne;
  int rc = compact_rows(n, start, deg, buf, g);
  free(start); free(deg); free(buf);
  return rc;
}

/* ----------------------------------------------------------------- RMAT -- */

/* RMAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): m0 = edge_factor * 2^scale
 * edges; at each of the scale levels an edge picks a quadrant with
 * probabilities (a, b, c, 1-a-b-c). Level l of edge e uses the 16-bit field
 * (l % 4) of rng64(seed, 10, e*ceil(scale/4) + l/4) as a uniform draw in
 * units of 2^-16. Self-loops dropped, symmetrised, duplicates removed, then
 * vertex ids relabelled by a seeded Fisher-Yates permutation (stream 11). */
static void rmat_edge(int32_t scale, uint32_t ta, uint32_t tb, uint32_t tc, uint64_t seed, int64_t e, int64_t *u,
                      int64_t *v) {
  int64_t uu = 0, vv = 0;
  const int64_t words = (scale + 3) / 4;
  uint64_t r = 0;
  for (int l = 0; l < scale; l++) {
    if ((l & 3) == 0) r = gg_rng64(seed, 10, (uint64_t)e * (uint64_t)words + (uint64_t)(l >> 2));
    const uint32_t p = (uint32_t)((r >> (16 * (l & 3))) & 0xFFFFu);
    int bu, bv;
    if (p < ta) { bu = 0; bv = 0; }
    else if (p < tb) { bu = 0; bv = 1; }
    else if (p < tc) { bu = 1; bv = 0; }
    else { bu = 1; bv = 1; }
    uu = (uu << 1) | bu;
    vv = (vv << 1) | bv;
  }
  *u = uu;
  *v = vv;
}

int gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, uint64_t seed, gg_graph *g) {
  memset(g, 0, sizeof(*g));
  if (scale < 1 || scale > 30 || edge_factor < 1 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -3;
  int64_t n = (int64_t)1 << scale;
  int64_t m0 = (int64_t)edge_factor * n;
  if (2 * m0 > ((int64_t)1 << 33)) return -3;
  const uint32_t ta = (uint32_t)(a * 65536.0 + 0.5), tb = (uint32_t)((a + b) * 65536.0 + 0.5),
                 tc = (uint32_t)((a + b + c) * 65536.0 + 0.5);
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int64_t *deg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int32_t *eu = (int32_t *)malloc(sizeof(int32_t) * (size_t)m0);
  int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)m0);
  if (!perm || !deg || !start || !eu || !ev) {
    free(perm); free(deg); free(start); free(eu); free(ev);
    return -1;
  }
  for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; i--) {
    int64_t j = (int64_t)(gg_rng64(seed, 11, (uint64_t)i) % (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
  /* per-thread degree histograms: thread t owns edge chunk t in both passes,
   * so arcs land at precomputed offsets without atomics */
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  int32_t *cnt = (int32_t *)calloc((size_t)nt * (size_t)n, sizeof(int32_t));
  if (!cnt) { free(perm); free(deg); free(start); free(eu); free(ev); return -1; }
#pragma omp parallel num_threads(nt)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    const int64_t lo = m0 * t / nt, hi = m0 * (t + 1) / nt;
    int32_t *ct = cnt + (size_t)t * (size_t)n;
    for (int64_t e = lo; e < hi; e++) {
      int64_t u, v;
      rmat_edge(scale, ta, tb, tc, seed, e, &u, &v);
      if (u == v) {
        eu[e] = -1;
        ev[e] = -1;
        continue;
      }
      eu[e] = perm[u];
      ev[e] = perm[v];
      ct[eu[e]]++;
      ct[ev[e]]++;
    }
  }
  int64_t v0;
#pragma omp parallel for schedule(static)
  for (v0 = 0; v0 < n; v0++) {
    int64_t acc = 0;
    for (int t = 0; t < nt; t++) {
      const int32_t c = cnt[(size_t)t * (size_t)n + v0];
      cnt[(size_t)t * (size_t)n + v0] = (int32_t)acc;
      acc += c;
    }
    deg[v0] = acc;
  }
  int64_t acc = 0;
  for (int64_t v = 0; v < n; v++) { start[v] = acc; acc += deg[v]; }
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(acc > 0 ? acc : 1));
  if (!buf) { free(perm); free(deg); free(start); free(eu); free(ev); free(cnt); return -1; }
#pragma omp parallel num_threads(nt)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    const int64_t lo = m0 * t / nt, hi = m0 * (t + 1) / nt;
    int32_t *ct = cnt + (size_t)t * (size_t)n;
    for (int64_t e = lo; e < hi; e++) {
      const int32_t u = eu[e], v = ev[e];
      if (u < 0) continue;
      buf[start[u] + ct[u]++] = v;
      buf[start[v] + ct[v]++] = u;
    }
  }
  free(cnt);
  free(eu);
  free(ev);
  int rc = compact_rows(n, start, deg, buf, g);
  free(perm); free(deg); free(start); free(buf);
  return rc;
}

/* Arc weights for weighted shortest paths: w[e] = lo + (draw of stream 70 at
 * counter e) mod (hi - lo + 1), independent per arc (modulo bias below
 * 2^-40 for hi - lo < 2^24). */
void gg_weights(int64_t m, uint64_t seed, uint32_t lo, uint32_t hi, uint32_t *w) {
  const uint64_t span = (uint64_t)(hi - lo) + 1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; e++) w[e] = lo + (uint32_t)(gg_rng64(seed, 70, (uint64_t)e) % span);
}

int gg_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
