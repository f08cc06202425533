// Seeded synthetic graph generators (CPU, OpenMP).
//
// This module only makes inputs: it holds none of the BFS / matvec arithmetic
// and is shared by the tests, the benchmark and the oracle-side checks.
//
// Graph shapes follow the workloads the paper measures on (Section 7.1,
// Table 3): scale-free R-MAT graphs and mesh-like graphs, made undirected,
// with self-loops and duplicate edges removed.
//
// Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014) used as a counter-based
// generator: output number n of the stream seeded with s is
// mix64(s + (n + 1) * GAMMA), so any edge can be generated independently of
// the others and the result does not depend on the thread count.
//
// Output format: int32 CSR (rowptr[V+1], colind[nnz]) with every row sorted
// ascending and free of duplicates.

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include <omp.h>

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Output number n of the SplitMix64 stream seeded with `seed`.
inline uint64_t splitmix_at(uint64_t seed, uint64_t n) { return mix64(seed + (n + 1) * GAMMA); }

// Uniform double in [0, 1) with 53 random bits.
inline double u01(uint64_t x) { return double(x >> 11) * (1.0 / 9007199254740992.0); }

// Uniform integer in [0, n) by multiply-shift (bias below 2^-32 for n < 2^32).
inline uint64_t below(uint64_t x, uint64_t n) {
  return uint64_t((unsigned __int128)x * n >> 64);
}

// Independent sub-streams of one user seed.
enum : uint64_t { STREAM_RMAT = 1, STREAM_PERM = 2, STREAM_DELETE = 3, STREAM_SOURCES = 4 };
inline uint64_t stream_seed(uint64_t seed, uint64_t stream) { return mix64(seed ^ mix64(stream * GAMMA)); }

struct Graph {
  int32_t V = 0;
  std::vector<int64_t> rowptr;  // 64-bit while building
  std::vector<int32_t> colind;
};

// One R-MAT edge: at each of `scale` levels pick a quadrant with
// probabilities (a, b, c, d); b sets a bit of the destination, c of the
// source, d of both.
inline void rmat_edge(uint64_t s, int scale, double a, double ab, double abc, uint64_t k,
                      int32_t* src, int32_t* dst) {
  uint32_t u = 0, v = 0;
  for (int l = 0; l < scale; ++l) {
    double r = u01(splitmix_at(s, k * 64 + uint64_t(l)));
    uint32_t bu = 0, bv = 0;
    if (r < a) {
    } else if (r < ab) {
      bv = 1;
    } else if (r < abc) {
      bu = 1;
    } else {
      bu = 1;
      bv = 1;
    }
    u = (u << 1) | bu;
    v = (v << 1) | bv;
  }
  *src = int32_t(u);
  *dst = int32_t(v);
}

// Fisher-Yates permutation of [0, V) drawn from its own stream.
std::vector<int32_t> permutation(int32_t V, uint64_t seed) {
  std::vector<int32_t> p(V);
  std::iota(p.begin(), p.end(), 0);
  uint64_t s = stream_seed(seed, STREAM_PERM);
  for (int64_t i = int64_t(V) - 1; i > 0; --i) {
    uint64_t j = below(splitmix_at(s, uint64_t(i)), uint64_t(i) + 1);
    std::swap(p[i], p[j]);
  }
  return p;
}

// Sort every row, drop duplicates and compact. rowptr/colind are rewritten.
void sort_dedup_rows(Graph& g) {
  const int32_t V = g.V;
  std::vector<int64_t> newdeg(V);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < V; ++i) {
    int32_t* b = g.colind.data() + g.rowptr[i];
    int32_t* e = g.colind.data() + g.rowptr[i + 1];
    std::sort(b, e);
    newdeg[i] = std::unique(b, e) - b;
  }
  std::vector<int64_t> np(V + 1, 0);
  for (int64_t i = 0; i < V; ++i) np[i + 1] = np[i] + newdeg[i];
  std::vector<int32_t> nc(np[V]);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < V; ++i)
    std::memcpy(nc.data() + np[i], g.colind.data() + g.rowptr[i], sizeof(int32_t) * newdeg[i]);
  g.rowptr.swap(np);
  g.colind.swap(nc);
}

// Build an undirected simple graph from an edge generator: each generated
// pair (u, v) with u != v contributes u->v and v->u; duplicates are removed.
template <class EdgeFn>
Graph build_undirected(int32_t V, int64_t m, EdgeFn edge) {
  Graph g;
  g.V = V;
  std::vector<std::atomic<int64_t>> deg(V);
  for (auto& d : deg) d.store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    int32_t u, v;
    edge(k, &u, &v);
    if (u == v) continue;
    deg[u].fetch_add(1, std::memory_order_relaxed);
    deg[v].fetch_add(1, std::memory_order_relaxed);
  }
  g.rowptr.assign(V + 1, 0);
  for (int64_t i = 0; i < V; ++i) g.rowptr[i + 1] = g.rowptr[i] + deg[i].load(std::memory_order_relaxed);
  g.colind.resize(g.rowptr[V]);
  std::vector<std::atomic<int64_t>> cur(V);
  for (int64_t i = 0; i < V; ++i) cur[i].store(g.rowptr[i], std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    int32_t u, v;
    edge(k, &u, &v);  // regenerated: the generator is a pure function of k
    if (u == v) continue;
    g.colind[cur[u].fetch_add(1, std::memory_order_relaxed)] = v;
    g.colind[cur[v].fetch_add(1, std::memory_order_relaxed)] = u;
  }
  sort_dedup_rows(g);
  return g;
}

Graph* finish(Graph&& g) { return new Graph(std::move(g)); }

}  // namespace

extern "C" {

// Raw (directed, unsymmetrized, unpermuted) R-MAT edges number
// [start, start+count) of the stream for `seed`; for testing the generator.
void gen_rmat_edges(int scale, double a, double b, double c, uint64_t seed, int64_t start,
                    int64_t count, int32_t* src, int32_t* dst) {
  const uint64_t s = stream_seed(seed, STREAM_RMAT);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) rmat_edge(s, scale, a, ab, abc, uint64_t(start + i), src + i, dst + i);
}

// R-MAT graph with 2^scale vertices and edgefactor * 2^scale generated edges,
// optionally relabelled by a seeded random permutation, then made undirected
// and simple. Returns an opaque handle (free with gen_graph_free).
void* gen_rmat(int scale, int64_t edgefactor, double a, double b, double c, uint64_t seed,
               int relabel) {
  if (scale < 1 || scale > 30 || edgefactor < 0) return nullptr;
  const int32_t V = int32_t(1) << scale;
  const int64_t m = edgefactor * int64_t(V);
  const uint64_t s = stream_seed(seed, STREAM_RMAT);
  const double ab = a + b, abc = a + b + c;
  std::vector<int32_t> perm;
  if (relabel) perm = permutation(V, seed);
  const int32_t* P = relabel ? perm.data() : nullptr;
  auto edge = [=](int64_t k, int32_t* u, int32_t* v) {
    rmat_edge(s, scale, a, ab, abc, uint64_t(k), u, v);
    if (P) {
      *u = P[*u];
      *v = P[*v];
    }
  };
  return finish(build_undirected(V, m, edge));
}

// n x n x n 7-point lattice (each vertex joined to its axis neighbours),
// vertex id x + n*(y + n*z). Exactly floor(del_frac * M) of the M undirected
// edges, chosen uniformly at random without replacement, are deleted.
void* gen_lattice3d(int32_t n, double del_frac, uint64_t seed) {
  if (n < 1 || int64_t(n) * n * n > INT32_MAX) return nullptr;
  const int64_t n1 = n - 1, nn = int64_t(n) * n;
  const int64_t per_axis = nn * n1;  // edges along one axis
  const int64_t M = 3 * per_axis;
  int64_t D = int64_t(del_frac * double(M));
  if (D < 0) D = 0;
  if (D > M) D = M;
  // Deleted-edge bitmap by a partial Fisher-Yates shuffle of edge ids.
  std::vector<uint8_t> deleted(M, 0);
  if (D > 0) {
    std::vector<int32_t> ids(M);
    std::iota(ids.begin(), ids.end(), 0);
    const uint64_t s = stream_seed(seed, STREAM_DELETE);
    for (int64_t i = 0; i < D; ++i) {
      int64_t j = i + int64_t(below(splitmix_at(s, uint64_t(i)), uint64_t(M - i)));
      std::swap(ids[i], ids[j]);
      deleted[ids[i]] = 1;
    }
  }
  // Edge id of the edge from (x,y,z) to its +1 neighbour along `axis`.
  auto eid = [=](int axis, int64_t x, int64_t y, int64_t z) -> int64_t {
    if (axis == 0) return x + n1 * (y + int64_t(n) * z);
    if (axis == 1) return per_axis + y + n1 * (x + int64_t(n) * z);
    return 2 * per_axis + z + n1 * (x + int64_t(n) * y);
  };
  Graph g;
  g.V = int32_t(nn * n);
  std::vector<int64_t> deg(g.V, 0);
  // Neighbours in ascending id order: -z, -y, -x, +x, +y, +z.
  auto for_nbrs = [&](int64_t x, int64_t y, int64_t z, auto&& f) {
    const int64_t id = x + n * (y + int64_t(n) * z);
    if (z > 0 && !deleted[eid(2, x, y, z - 1)]) f(id - nn);
    if (y > 0 && !deleted[eid(1, x, y - 1, z)]) f(id - n);
    if (x > 0 && !deleted[eid(0, x - 1, y, z)]) f(id - 1);
    if (x < n1 && !deleted[eid(0, x, y, z)]) f(id + 1);
    if (y < n1 && !deleted[eid(1, x, y, z)]) f(id + n);
    if (z < n1 && !deleted[eid(2, x, y, z)]) f(id + nn);
  };
#pragma omp parallel for schedule(static)
  for (int64_t id = 0; id < g.V; ++id) {
    int64_t x = id % n, y = (id / n) % n, z = id / nn, d = 0;
    for_nbrs(x, y, z, [&](int64_t) { ++d; });
    deg[id] = d;
  }
  g.rowptr.assign(g.V + 1, 0);
  for (int64_t i = 0; i < g.V; ++i) g.rowptr[i + 1] = g.rowptr[i] + deg[i];
  g.colind.resize(g.rowptr[g.V]);
#pragma omp parallel for schedule(static)
  for (int64_t id = 0; id < g.V; ++id) {
    int64_t x = id % n, y = (id / n) % n, z = id / nn, p = g.rowptr[id];
    for_nbrs(x, y, z, [&](int64_t w) { g.colind[p++] = int32_t(w); });
  }
  return finish(std::move(g));
}

// nx x ny 4-connected grid, vertex id x + nx*y.
void* gen_grid2d(int32_t nx, int32_t ny) {
  if (nx < 1 || ny < 1 || int64_t(nx) * ny > INT32_MAX) return nullptr;
  Graph g;
  g.V = nx * ny;
  g.rowptr.assign(g.V + 1, 0);
  for (int64_t id = 0; id < g.V; ++id) {
    int64_t x = id % nx, y = id / nx;
    g.rowptr[id + 1] = g.rowptr[id] + (y > 0) + (x > 0) + (x < nx - 1) + (y < ny - 1);
  }
  g.colind.resize(g.rowptr[g.V]);
#pragma omp parallel for schedule(static)
  for (int64_t id = 0; id < g.V; ++id) {
    int64_t x = id % nx, y = id / nx, p = g.rowptr[id];
    if (y > 0) g.colind[p++] = int32_t(id - nx);
    if (x > 0) g.colind[p++] = int32_t(id - 1);
    if (x < nx - 1) g.colind[p++] = int32_t(id + 1);
    if (y < ny - 1) g.colind[p++] = int32_t(id + nx);
  }
  return finish(std::move(g));
}

int32_t gen_graph_nv(void* h) { return static_cast<Graph*>(h)->V; }
int64_t gen_graph_nnz(void* h) { return int64_t(static_cast<Graph*>(h)->colind.size()); }

// Copy the CSR out as int32 arrays (rowptr[V+1], colind[nnz]). Returns -1 if
// nnz does not fit int32 offsets.
int gen_graph_copy(void* h, int32_t* rowptr, int32_t* colind) {
  Graph* g = static_cast<Graph*>(h);
  if (g->rowptr[g->V] > INT32_MAX) return -1;
  for (int64_t i = 0; i <= g->V; ++i) rowptr[i] = int32_t(g->rowptr[i]);
  std::memcpy(colind, g->colind.data(), sizeof(int32_t) * g->colind.size());
  return 0;
}

void gen_graph_free(void* h) { delete static_cast<Graph*>(h); }

// k distinct vertices drawn uniformly without replacement from cand[0..n),
// by a partial Fisher-Yates shuffle on a copy. Returns the number written.
int64_t gen_sample(const int32_t* cand, int64_t n, int64_t k, uint64_t seed, int32_t* out) {
  if (k > n) k = n;
  std::vector<int32_t> c(cand, cand + n);
  const uint64_t s = stream_seed(seed, STREAM_SOURCES);
  for (int64_t i = 0; i < k; ++i) {
    int64_t j = i + int64_t(below(splitmix_at(s, uint64_t(i)), uint64_t(n - i)));
    std::swap(c[i], c[j]);
    out[i] = c[i];
  }
  return k;
}

// Transpose of a CSR (rows sorted in the output): the CSC of the same matrix.
void gen_transpose(int32_t V, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                   int32_t* t_rowptr, int32_t* t_colind) {
  std::vector<int64_t> cnt(V + 1, 0);
  for (int64_t p = 0; p < nnz; ++p) cnt[colind[p] + 1]++;
  for (int64_t i = 0; i < V; ++i) cnt[i + 1] += cnt[i];
  for (int64_t i = 0; i <= V; ++i) t_rowptr[i] = int32_t(cnt[i]);
  // Row order ascending in the source => sorted target rows.
  for (int64_t u = 0; u < V; ++u)
    for (int64_t p = rowptr[u]; p < rowptr[u + 1]; ++p) t_colind[cnt[colind[p]]++] = int32_t(u);
}

int gen_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
