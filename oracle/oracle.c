/*
 * CPU oracle for direction-optimized BFS expressed as Boolean matvec.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the GPU library links, includes or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it. It shares no code, header or table with the GPU
 * path.
 *
 * Every routine is the plain definition of what it computes, written for a
 * reader to check against the paper by eye; none is blocked, fused or
 * reordered for speed.
 *
 * Graph convention: A(u,v) = 1 for an edge u->v. CSR(A) row u lists the
 * out-neighbours of u; CSC(A) column v lists the in-neighbours of v. The BFS
 * frontier recurrence is f' = A^T f .* not(v) (Section 4, Algorithm 1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * Breadth-first search from `source` (Section 2.1): depth[v] is the number of
 * edges on a shortest directed path source->v, -1 when v is unreachable.
 * parent[v] is the vertex from which v was first reached (parent[source] =
 * source, -1 when unreachable). Textbook FIFO-queue BFS over CSR(A).
 * Returns 0, or -1 for a source out of range, -2 if memory runs out.
 */
int oracle_bfs(int32_t V, const int32_t *rowptr, const int32_t *colind, int32_t source,
               int32_t *depth, int32_t *parent) {
  if (source < 0 || source >= V) return -1;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)V);
  if (!queue) return -2;
  for (int32_t i = 0; i < V; ++i) {
    depth[i] = -1;
    if (parent) parent[i] = -1;
  }
  int64_t head = 0, tail = 0;
  depth[source] = 0;
  if (parent) parent[source] = source;
  queue[tail++] = source;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t p = rowptr[u]; p < rowptr[u + 1]; ++p) {
      int32_t v = colind[p];
      if (depth[v] < 0) {
        depth[v] = depth[u] + 1;
        if (parent) parent[v] = u;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return 0;
}

/*
 * Graph500-style validation of a BFS result (depth, parent) from `source`.
 *   1: depth[source] = 0 and parent[source] = source
 *   2: only the source has depth 0; depths are >= -1
 *   3: depth[v] = -1 exactly when parent[v] = -1
 *   4: for every reached v != source, p = parent[v] is a vertex, depth[p] =
 *      depth[v] - 1, and p->v is an edge (p is listed in CSC column v)
 *   5: for every edge u->v with u reached, v is reached and
 *      depth[v] <= depth[u] + 1 (levels are tight; all reachable vertices are
 *      reached)
 * Together 4 and 5 make depth the shortest-path hop count. Returns 0 when
 * valid, otherwise the number of the first failed check, and *bad = the
 * offending vertex.
 */
int oracle_validate(int32_t V, const int32_t *rowptr, const int32_t *colind,
                    const int32_t *colptr, const int32_t *rowind, int32_t source,
                    const int32_t *depth, const int32_t *parent, int64_t *bad) {
  *bad = -1;
  if (source < 0 || source >= V) return 1;
  if (depth[source] != 0 || parent[source] != source) { *bad = source; return 1; }
  for (int32_t v = 0; v < V; ++v) {
    if (depth[v] < -1 || (depth[v] == 0 && v != source)) { *bad = v; return 2; }
    if ((depth[v] == -1) != (parent[v] == -1)) { *bad = v; return 3; }
  }
  for (int32_t v = 0; v < V; ++v) {
    if (v == source || depth[v] < 0) continue;
    int32_t p = parent[v];
    if (p < 0 || p >= V || depth[p] != depth[v] - 1) { *bad = v; return 4; }
    int found = 0;
    for (int64_t q = colptr[v]; q < colptr[v + 1]; ++q)
      if (rowind[q] == p) { found = 1; break; }
    if (!found) { *bad = v; return 4; }
  }
  for (int32_t u = 0; u < V; ++u) {
    if (depth[u] < 0) continue;
    for (int64_t q = rowptr[u]; q < rowptr[u + 1]; ++q) {
      int32_t v = colind[q];
      if (depth[v] < 0 || depth[v] > depth[u] + 1) { *bad = v; return 5; }
    }
  }
  return 0;
}

/*
 * Masked matvec over the Boolean semiring ({0,1}, OR, AND, 0), Equations 4
 * and 5 with the structural complement of Section 3.2:
 *     t(i) = OR over edges j->i of ( x(j) AND 1 )          (t = A^T x)
 *     pass(i) = mask == NULL ? 1 : ((mask(i) != 0) XOR complement)
 *     y(i) = accum ? (y(i) OR (t(i) AND pass(i))) : (t(i) AND pass(i))
 * x, mask and y hold one byte (0 or 1) per vertex. Computed edge by edge
 * over CSR(A).
 */
void oracle_mxv(int32_t V, const int32_t *rowptr, const int32_t *colind, const uint8_t *x,
                const uint8_t *mask, int complement, int accum, uint8_t *y) {
  uint8_t *t = (uint8_t *)calloc((size_t)V + 1, 1);
  for (int32_t j = 0; j < V; ++j) {
    if (!x[j]) continue;
    for (int64_t p = rowptr[j]; p < rowptr[j + 1]; ++p) t[colind[p]] = 1;
  }
  for (int32_t i = 0; i < V; ++i) {
    int pass = mask ? ((mask[i] != 0) ^ (complement != 0)) : 1;
    uint8_t val = (uint8_t)(t[i] && pass);
    y[i] = accum ? (uint8_t)(y[i] || val) : val;
  }
  free(t);
}

/*
 * The parent a pull step that stops at the first hit reports (Section 5.3,
 * Algorithm 2 with early exit): for each reached v != source, the first
 * in-neighbour u of v, in the stored order of CSC column v, with depth[u] =
 * depth[v] - 1. -1 for unreached vertices, source for the source.
 */
void oracle_first_parent(int32_t V, const int32_t *colptr, const int32_t *rowind,
                         const int32_t *depth, int32_t source, int32_t *out) {
  for (int32_t v = 0; v < V; ++v) {
    out[v] = -1;
    if (depth[v] < 0) continue;
    if (v == source) { out[v] = source; continue; }
    for (int64_t q = colptr[v]; q < colptr[v + 1]; ++q)
      if (depth[rowind[q]] == depth[v] - 1) { out[v] = rowind[q]; break; }
  }
}

/*
 * In-neighbour checks a level-L pull with masking and early exit makes when
 * its input is the visited set at the start of the level (Sections 5.2-5.4):
 * for every vertex i unvisited at level start (depth[i] < 0 or depth[i] > L),
 * scan CSC column i in stored order and count entries up to and including the
 * first u with 0 <= depth[u] <= L; all entries when there is none.
 */
int64_t oracle_pull_checks(int32_t V, const int32_t *colptr, const int32_t *rowind,
                           const int32_t *depth, int32_t L) {
  int64_t total = 0;
  for (int32_t i = 0; i < V; ++i) {
    if (depth[i] >= 0 && depth[i] <= L) continue;
    int64_t k = 0;
    for (int64_t q = colptr[i]; q < colptr[i + 1]; ++q) {
      ++k;
      int32_t d = depth[rowind[q]];
      if (d >= 0 && d <= L) break;
    }
    total += k;
  }
  return total;
}
