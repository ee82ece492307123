/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the traversal
 * results. TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * benchmark's CPU-baseline leg call it; the GPU library never links, loads or
 * calls anything here, and nothing here uses GPU code.
 *
 * Every function is the plain definition of the result it returns, single
 * threaded, with no blocking, fusion or reordering:
 *
 *  oracle_bfs     hop distances from one source, by the standard sequential
 *                 algorithm that keeps visited vertices in a FIFO queue (the
 *                 paper's sequential BFS baseline, Experimental Results and
 *                 the BFS time table). Unreached vertices get -1.
 *  oracle_reach   for each source i, the set of vertices reachable from it
 *                 (reachability search, Parallel SCC section), by iterative
 *                 depth-first search with an explicit stack; the result is a
 *                 bit mask per vertex, bit i%64 of word i/64 set iff
 *                 sources[i] reaches the vertex (length-0 paths included).
 *  oracle_scc     strongly connected components by Tarjan's algorithm (the
 *                 paper's sequential SCC baseline), iterative; comp[v] is the
 *                 index of v's component in the order Tarjan completes them.
 *  oracle_transpose  G^T by a stable counting sort of the arcs by target, so
 *                 every row of G^T lists its sources in ascending order.
 *  oracle_sssp    single-source shortest-path distances with non-negative
 *                 integer arc weights (Parallel SSSP paragraph: the stepping
 *                 framework computes these exact distances), by Dijkstra's
 *                 algorithm with a binary heap and lazy deletion; int64
 *                 distances, -1 for unreached vertices.
 *
 * CSR input: offsets[n+1], targets[m], int32, targets in [0,n). Self-loops and
 * duplicate arcs are allowed and change nothing.
 * Return value: 0 on success (oracle_scc: the number of components), -1 on
 * allocation failure, -2 on bad arguments.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int oracle_bfs(int32_t n, const int32_t *offsets, const int32_t *targets, int32_t src, int32_t *dist) {
  if (n <= 0 || src < 0 || src >= n) return -2;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return -1;
  for (int32_t v = 0; v < n; v++) dist[v] = -1;
  int64_t head = 0, tail = 0;
  dist[src] = 0;
  queue[tail++] = src;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int32_t e = offsets[u]; e < offsets[u + 1]; e++) {
      int32_t w = targets[e];
      if (dist[w] == -1) {
        dist[w] = dist[u] + 1;
        queue[tail++] = w;
      }
    }
  }
  free(queue);
  return 0;
}

int oracle_reach(int32_t n, const int32_t *offsets, const int32_t *targets, int32_t k, const int32_t *sources,
                 int32_t words, uint64_t *mask) {
  if (n <= 0 || k <= 0 || words < (k + 63) / 64) return -2;
  for (int32_t i = 0; i < k; i++)
    if (sources[i] < 0 || sources[i] >= n) return -2;
  int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!stack) return -1;
  memset(mask, 0, sizeof(uint64_t) * (size_t)n * (size_t)words);
  for (int32_t i = 0; i < k; i++) {
    const int32_t word = i / 64;
    const uint64_t bit = 1ULL << (i % 64);
    int32_t s = sources[i];
    int64_t top = 0;
    mask[(size_t)s * words + word] |= bit;
    stack[top++] = s;
    while (top > 0) {
      int32_t u = stack[--top];
      for (int32_t e = offsets[u]; e < offsets[u + 1]; e++) {
        int32_t w = targets[e];
        uint64_t *mw = &mask[(size_t)w * words + word];
        if (!(*mw & bit)) {
          *mw |= bit;
          stack[top++] = w; /* each vertex is pushed at most once per source */
        }
      }
    }
  }
  free(stack);
  return 0;
}

/* Tarjan (1972). Iterative form: an explicit call stack of (vertex, next arc)
 * frames replaces recursion. index[v] = discovery order, low[v] = smallest
 * index reachable through the DFS subtree of v and one back/cross arc into the
 * current stack. A vertex with low == index roots a component, which is
 * popped from the component stack. */
int oracle_scc(int32_t n, const int32_t *offsets, const int32_t *targets, int32_t *comp) {
  if (n <= 0) return -2;
  int32_t *index = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *low = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  char *onstack = (char *)calloc((size_t)n, 1);
  int32_t *cstack = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *fv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *fe = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!index || !low || !onstack || !cstack || !fv || !fe) {
    free(index); free(low); free(onstack); free(cstack); free(fv); free(fe);
    return -1;
  }
  for (int32_t v = 0; v < n; v++) { index[v] = -1; comp[v] = -1; }
  int32_t counter = 0, ncomp = 0, ctop = 0;
  for (int32_t root = 0; root < n; root++) {
    if (index[root] != -1) continue;
    int32_t ftop = 0;
    fv[ftop] = root; fe[ftop] = offsets[root]; ftop++;
    index[root] = low[root] = counter++;
    cstack[ctop++] = root; onstack[root] = 1;
    while (ftop > 0) {
      int32_t u = fv[ftop - 1];
      if (fe[ftop - 1] < offsets[u + 1]) {
        int32_t w = targets[fe[ftop - 1]++];
        if (index[w] == -1) {
          index[w] = low[w] = counter++;
          cstack[ctop++] = w; onstack[w] = 1;
          fv[ftop] = w; fe[ftop] = offsets[w]; ftop++;
        } else if (onstack[w] && index[w] < low[u]) {
          low[u] = index[w];
        }
      } else {
        /* u finished */
        if (low[u] == index[u]) {
          int32_t x;
          do {
            x = cstack[--ctop];
            onstack[x] = 0;
            comp[x] = ncomp;
          } while (x != u);
          ncomp++;
        }
        ftop--;
        if (ftop > 0) {
          int32_t p = fv[ftop - 1];
          if (low[u] < low[p]) low[p] = low[u];
        }
      }
    }
  }
  free(index); free(low); free(onstack); free(cstack); free(fv); free(fe);
  return ncomp;
}

int oracle_transpose(int32_t n, const int32_t *offsets, const int32_t *targets, int32_t *t_offsets,
                     int32_t *t_targets) {
  if (n <= 0) return -2;
  int32_t m = offsets[n];
  int32_t *cursor = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!cursor) return -1;
  for (int32_t v = 0; v <= n; v++) t_offsets[v] = 0;
  for (int32_t e = 0; e < m; e++) t_offsets[targets[e] + 1]++;
  for (int32_t v = 0; v < n; v++) t_offsets[v + 1] += t_offsets[v];
  for (int32_t v = 0; v < n; v++) cursor[v] = t_offsets[v];
  for (int32_t u = 0; u < n; u++)
    for (int32_t e = offsets[u]; e < offsets[u + 1]; e++) t_targets[cursor[targets[e]]++] = u;
  free(cursor);
  return 0;
}

/* Binary min-heap of (distance, vertex) pairs for Dijkstra. */
typedef struct {
  int64_t key;
  int32_t v;
} heap_item;

static void heap_push(heap_item *h, int64_t *size, int64_t key, int32_t v) {
  int64_t i = (*size)++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].key <= key) break;
    h[i] = h[p];
    i = p;
  }
  h[i].key = key;
  h[i].v = v;
}

static heap_item heap_pop(heap_item *h, int64_t *size) {
  heap_item top = h[0];
  heap_item last = h[--(*size)];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= *size) break;
    if (c + 1 < *size && h[c + 1].key < h[c].key) c++;
    if (last.key <= h[c].key) break;
    h[i] = h[c];
    i = c;
  }
  if (*size > 0) h[i] = last;
  return top;
}

int oracle_sssp(int32_t n, const int32_t *offsets, const int32_t *targets, const uint32_t *weights, int32_t src,
                int64_t *dist) {
  if (n <= 0 || src < 0 || src >= n) return -2;
  const int64_t m = offsets[n];
  heap_item *heap = (heap_item *)malloc(sizeof(heap_item) * (size_t)(m + 1));
  if (!heap) return -1;
  for (int32_t v = 0; v < n; v++) dist[v] = -1;
  int64_t size = 0;
  dist[src] = 0;
  heap_push(heap, &size, 0, src);
  while (size > 0) {
    heap_item it = heap_pop(heap, &size);
    int32_t u = it.v;
    if (it.key != dist[u]) continue; /* a shorter distance was found after this push */
    for (int32_t e = offsets[u]; e < offsets[u + 1]; e++) {
      int32_t w = targets[e];
      int64_t nd = it.key + (int64_t)weights[e];
      if (dist[w] < 0 || nd < dist[w]) {
        dist[w] = nd;
        heap_push(heap, &size, nd, w);
      }
    }
  }
  free(heap);
  return 0;
}
