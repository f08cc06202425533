// Host runtime and C ABI of libdobfs (declared in include/dobfs.h).
//
// The BFS level loop of Algorithm 1 is enqueued from the host in batches of
// steps (one kernel launch each, one or two per level); each level's
// direction (the rule of Section 6.3) is decided on the device from the
// previous step's counters, and the host reads the states back once per batch
// from pinned memory. Single-source and multi-source traversals share the
// loop (run_steps) and differ in their kernels.

#include "dobfs.h"
#include "dobfs_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

using namespace dobfs;

struct dobfs_graph_s {
  int device = 0;
  int32_t V = 0;
  int64_t nnz = 0;
  int32_t nwords = 0;
  const int32_t* rowptr = nullptr;  // CSR(A)
  const int32_t* colind = nullptr;
  const int32_t* colptr = nullptr;  // CSC(A)
  const int32_t* rowind = nullptr;
  uint32_t* nz_in = nullptr;        // rows of CSC(A) with at least one entry
  uint32_t* heavy = nullptr;        // rows of CSR(A) with more than kLocalDeg entries
  int4* slab = nullptr;             // first kSlab entries of every CSC(A) column (-1 past its end)
  int32_t* head = nullptr;          // first entry of every CSC(A) column, complemented when more follow
  uint32_t max_outdeg = 0;          // largest CSR(A) row length
  bool symmetric = false;           // given as undirected: the same arrays for CSR(A) and CSC(A)
  std::atomic<int32_t> last_steps{8};   // step count of the previous single-source BFS
  std::atomic<int32_t> last_steps_mb{8};   // the same for multi-source traversals
  void* owned[4] = {nullptr, nullptr, nullptr, nullptr};
  std::mutex mu;                    // guards the internal workspace
  void* ws = nullptr;
  size_t ws_size = 0;
  hipEvent_t ws_event = nullptr;    // recorded on the stream of the last call that used ws
  bool ws_event_recorded = false;
};

namespace {

thread_local std::string t_last_error;

dobfs_status fail(dobfs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_last_error = buf;
  return s;
}

dobfs_status hip_fail(hipError_t e, const char* what, int line) {
  return fail(e == hipErrorOutOfMemory ? DOBFS_ERR_OUT_OF_MEMORY : DOBFS_ERR_DEVICE,
              "%s failed: %s (api.hip:%d)", what, hipGetErrorString(e), line);
}

#define HIPCK(expr)                                               \
  do {                                                            \
    hipError_t e_ = (expr);                                       \
    if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__);  \
  } while (0)

// Makes `device` current for the scope of a call and restores the caller's.
struct DeviceScope {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int device) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    err = hipSetDevice(device);
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace layout of one call (BFS and mxv share it).
struct Layout {
  size_t visA, visB, FA, FB, Q0, Q1, S, R, chunks, flagsA, flagsB, ctrl, total;
  int64_t nflags, nchunks;
};

Layout plan(int32_t V, int64_t nnz) {
  Layout L{};
  const size_t wb = size_t(words_of(V)) * 4, vb = size_t(V) * 4;
  L.nflags = flag_entries(V);
  L.nchunks = max_chunks(nnz);
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    size_t off = cur;
    cur += align_up(bytes);
    return off;
  };
  L.visA = take(wb);
  L.visB = take(wb);
  L.FA = take(wb);
  L.FB = take(wb);
  L.Q0 = take(vb);
  L.Q1 = take(vb);
  L.S = take(vb);
  L.R = take(vb);
  L.chunks = take(size_t(L.nchunks) * 4);
  L.flagsA = take(size_t(L.nflags) * 8);
  L.flagsB = take(size_t(L.nflags) * 8);
  L.ctrl = take(sizeof(Ctrl));
  L.total = cur;
  return L;
}

// Workspace layout of the sort-based push: the common layout, then the
// pair buffers of the sort (nnz keys and values, twice) and its scratch.
struct SortLayout {
  Layout base;
  size_t kA, kB, vA, vB, tmp, tmp_bytes, total;
};

SortLayout plan_sort(int32_t V, int64_t nnz) {
  SortLayout L{};
  L.base = plan(V, nnz);
  size_t cur = L.base.total;
  auto take = [&](size_t bytes) {
    size_t off = cur;
    cur += align_up(bytes);
    return off;
  };
  const size_t nb = size_t(std::max<int64_t>(nnz, 1)) * 4;
  L.kA = take(nb);
  L.kB = take(nb);
  L.vA = take(nb);
  L.vB = take(nb);
  L.tmp_bytes = sort_push_bytes(nnz);
  L.tmp = take(L.tmp_bytes);
  L.total = cur;
  return L;
}

// Workspace layout of a multi-source call with k sources.
struct BatchLayout {
  size_t visA, visB, F, nzF0, nzF1, Q0, Q1, S, R, chunks, flagsA, flagsB, ctrl, lvl, total;
  int64_t nflags, nchunks;
};

BatchLayout plan_batch(int32_t V, int64_t nnz, int32_t k) {
  BatchLayout L{};
  const size_t wb = size_t(words_of(V)) * 4, vb = size_t(V) * 4, qb = size_t(V) * 8;
  L.nflags = flag_entries(V);
  L.nchunks = max_chunks(nnz);
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    size_t off = cur;
    cur += align_up(bytes);
    return off;
  };
  L.visA = take(qb);
  L.visB = take(qb);
  // frontier words: kMbSnap kept levels and two alternating, each buffer 256-byte aligned
  L.F = take(size_t(mb_fstride(V)) * 8 * size_t(kMbSnap + 2));
  L.nzF0 = take(wb);
  L.nzF1 = take(wb);
  L.Q0 = take(vb);
  L.Q1 = take(vb);
  L.S = take(vb);
  L.R = take(vb);
  L.chunks = take(size_t(L.nchunks) * 4);
  L.flagsA = take(size_t(L.nflags) * 8);
  L.flagsB = take(size_t(L.nflags) * 8);
  L.ctrl = take(sizeof(Ctrl));
  L.lvl = take(size_t(V) * size_t(k) * 2);
  L.total = cur;
  return L;
}

// Pinned host copy of the control block, one per thread (never freed: it
// must outlive any call and HIP may already be torn down at thread exit).
Ctrl* host_ctrl() {
  thread_local Ctrl* p = nullptr;
  if (!p) {
    void* q = nullptr;
    if (hipHostMalloc(&q, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess) return nullptr;
    p = static_cast<Ctrl*>(q);
  }
  return p;
}

// Pinned host buffer the level loop's report kernel writes, one per thread.
HostReport* host_report() {
  thread_local HostReport* p = nullptr;
  if (!p) {
    void* q = nullptr;
    if (hipHostMalloc(&q, sizeof(HostReport), hipHostMallocDefault) != hipSuccess) return nullptr;
    p = static_cast<HostReport*>(q);
    p->seq = 0;
  }
  return p;
}

// Sequence numbers of the reports a thread waits for: one counter for every
// loop that shares the thread's pinned buffer, so a stale number never matches.
uint32_t next_report_seq() {
  thread_local uint32_t n = 0;
  return ++n;
}

// Wait until the report with sequence number `seq` has landed: spin on the
// pinned word for a short while (a kernel-to-host write takes ~6 us where a
// stream synchronisation takes ~15 us), then block on the stream, which also
// surfaces any device error.
hipError_t wait_report(const HostReport* r, uint32_t seq, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t it = 1;; ++it) {
    if (__atomic_load_n(&r->seq, __ATOMIC_ACQUIRE) == seq) return hipSuccess;
    if ((it & 255) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000)) break;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  return __atomic_load_n(&r->seq, __ATOMIC_ACQUIRE) == seq ? hipSuccess : hipErrorUnknown;
}

// Where the level loop's report goes: `dev` is what the kernels write, `host`
// what the host reads. The same pinned buffer for both (the host spins on it),
// or a device buffer copied into ordinary host memory after the stream has
// drained (the allocation-free entry point, which may not pin memory).
struct ReportSink {
  HostReport* dev = nullptr;
  HostReport* host = nullptr;
};

hipError_t fetch_report(const ReportSink& r, uint32_t seq, hipStream_t s) {
  if (r.dev == r.host) return wait_report(r.host, seq, s);
  hipError_t e = hipMemcpyAsync(r.host, r.dev, sizeof(HostReport), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  return r.host->seq == seq ? hipSuccess : hipErrorUnknown;
}

// Per-thread, per-device events for the level loop's timers: the start and
// end of every step of a batch (kMaxBatch slots each), of the init kernel,
// and of the whole call.
constexpr int ev_m0(int k) { return k; }
constexpr int ev_m1(int k) { return kMaxBatch + k; }
constexpr int kEvStart = 2 * kMaxBatch, kEvInit0 = kEvStart + 1, kEvInit1 = kEvStart + 2,
              kEvEnd = kEvStart + 3;
constexpr int kEvents = kEvEnd + 1;
hipEvent_t* events_for(int device) {
  thread_local hipEvent_t ev[16][kEvents];
  thread_local bool made[16] = {};
  if (device < 0 || device >= 16) return nullptr;
  if (!made[device]) {
    for (int k = 0; k < kEvents; ++k)
      if (hipEventCreate(&ev[device][k]) != hipSuccess) return nullptr;
    made[device] = true;
  }
  return ev[device];
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

dobfs_options defaults() {
  dobfs_options o;
  std::memset(&o, 0, sizeof o);
  o.mode = DOBFS_MODE_FULL;
  o.heuristic = DOBFS_HEUR_RATIO;
  o.alpha = 0.01f;
  o.beta = 0.01f;
  return o;
}

dobfs_status check_options(const dobfs_options& o) {
  if (o.mode < DOBFS_MODE_FULL || o.mode > DOBFS_MODE_PUSH_SORT_KEYS)
    return fail(DOBFS_ERR_INVALID_ARG, "unknown mode %d", o.mode);
  if (o.heuristic != DOBFS_HEUR_RATIO && o.heuristic != DOBFS_HEUR_EDGES)
    return fail(DOBFS_ERR_INVALID_ARG, "unknown heuristic %d", o.heuristic);
  if (!std::isfinite(o.alpha) || !std::isfinite(o.beta) || o.alpha < 0.f || o.beta < 0.f)
    return fail(DOBFS_ERR_INVALID_ARG, "alpha and beta must be finite and >= 0");
  if (o.n_forced < 0 || (o.n_forced > 0 && !o.forced_dirs))
    return fail(DOBFS_ERR_INVALID_ARG, "forced_dirs missing for n_forced = %d", o.n_forced);
  for (int32_t k = 0; k < o.n_forced; ++k)
    if (o.forced_dirs[k] != DOBFS_DIR_PUSH && o.forced_dirs[k] != DOBFS_DIR_PULL)
      return fail(DOBFS_ERR_INVALID_ARG, "forced_dirs[%d] = %d is not a direction", k,
                  int(o.forced_dirs[k]));
  if (o.flags & ~uint32_t(DOBFS_OPT_TIME_KERNELS | DOBFS_OPT_PERSISTENT))
    return fail(DOBFS_ERR_INVALID_ARG, "unknown option flags 0x%x", o.flags);
  if (o.pull_mid != 0 && (o.pull_mid < kPullFirst || o.pull_mid > (1 << 20)))
    return fail(DOBFS_ERR_INVALID_ARG, "pull_mid = %d not in [%d, 2^20]", o.pull_mid, kPullFirst);
  if (o.bitmap_rows < 0 || o.bitmap_rows > kPullTileV)
    return fail(DOBFS_ERR_INVALID_ARG, "bitmap_rows = %d not in [0, %d]", o.bitmap_rows, kPullTileV);
  if (o.local_unit < 0 || o.local_unit > kThreads)
    return fail(DOBFS_ERR_INVALID_ARG, "local_unit = %d not in [0, %d]", o.local_unit, kThreads);
  if (o.local_chunks < 0 || o.local_chunks > (1 << 20))
    return fail(DOBFS_ERR_INVALID_ARG, "local_chunks = %d not in [0, 2^20]", o.local_chunks);
  return DOBFS_OK;
}

dobfs_status check_offsets_host(int32_t V, int64_t nnz, const int32_t* ptr, const char* name) {
  if (ptr[0] != 0) return fail(DOBFS_ERR_INVALID_ARG, "%s[0] = %d, expected 0", name, ptr[0]);
  for (int32_t i = 0; i < V; ++i)
    if (ptr[i + 1] < ptr[i])
      return fail(DOBFS_ERR_INVALID_ARG, "%s decreases at %d (%d -> %d)", name, i, ptr[i],
                  ptr[i + 1]);
  if (int64_t(ptr[V]) != nnz)
    return fail(DOBFS_ERR_INVALID_ARG, "%s[V] = %d, expected nnz = %lld", name, ptr[V],
                (long long)nnz);
  return DOBFS_OK;
}

dobfs_status check_args(int32_t V, int64_t nnz, const void* a, const void* b, const void* c,
                        const void* d, int32_t device, dobfs_graph* out) {
  if (!out) return fail(DOBFS_ERR_INVALID_ARG, "out is NULL");
  if (V < 1 || V > INT32_MAX - 64) return fail(DOBFS_ERR_INVALID_ARG, "V = %d out of range", V);
  if (nnz < 0 || nnz > INT32_MAX)
    return fail(DOBFS_ERR_INVALID_ARG, "nnz = %lld out of range [0, 2^31-1]", (long long)nnz);
  if (!a || !c) return fail(DOBFS_ERR_INVALID_ARG, "row/column offset array is NULL");
  if (nnz > 0 && (!b || !d)) return fail(DOBFS_ERR_INVALID_ARG, "index array is NULL");
  if (device < 0) return fail(DOBFS_ERR_INVALID_ARG, "device %d", device);
  return DOBFS_OK;
}

dobfs_status check_device(int32_t device) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) return fail(DOBFS_ERR_DEVICE, "no HIP device available");
  if (device < 0 || device >= n)
    return fail(DOBFS_ERR_INVALID_ARG, "device %d not in [0, %d)", device, n);
  return DOBFS_OK;
}

dobfs_status finish_graph(dobfs_graph g, hipStream_t s, uint32_t flags) {
  void* p = nullptr;
  HIPCK(hipMalloc(&p, size_t(std::max(g->nwords, 1)) * 4));
  g->nz_in = static_cast<uint32_t*>(p);
  HIPCK(launch_nz_bits(s, g->colptr, g->V, g->nz_in));
  HIPCK(hipMalloc(&p, size_t(std::max(g->nwords, 1)) * 4));
  g->heavy = static_cast<uint32_t*>(p);
  HIPCK(launch_nz_bits(s, g->rowptr, g->V, g->heavy, kLocalDeg));
  uint32_t* dmax = nullptr;
  HIPCK(hipMalloc(&p, sizeof(uint32_t)));
  dmax = static_cast<uint32_t*>(p);
  hipError_t e = hipMemsetAsync(dmax, 0, sizeof(uint32_t), s);
  if (e == hipSuccess) e = launch_max_degree(s, g->rowptr, g->V, dmax);
  if (e == hipSuccess) e = hipMemcpyAsync(&g->max_outdeg, dmax, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dmax);
  if (e != hipSuccess) return hip_fail(e, "max degree", __LINE__);
  if ((flags & DOBFS_UPLOAD_HUBS_FIRST) && g->nnz > 0) {
    // a reordered copy of CSC(A)'s indices, owned by the graph (the CSR side keeps its order)
    HIPCK(hipMalloc(&p, size_t(g->nnz) * 4));
    e = hubs_first(s, g->rowptr, g->colptr, g->rowind, static_cast<int32_t*>(p), g->V, g->nnz, g->max_outdeg);
    if (e != hipSuccess) {
      (void)hipFree(p);
      return hip_fail(e, "in-neighbour reorder", __LINE__);
    }
    const bool own = g->owned[3] != nullptr && g->owned[3] == static_cast<const void*>(g->rowind);
    if (own) (void)hipFree(g->owned[3]);
    g->owned[3] = p;
    g->rowind = static_cast<const int32_t*>(p);
  }
  HIPCK(hipMalloc(&p, size_t(std::max(g->V, 1)) * sizeof(int4)));
  g->slab = static_cast<int4*>(p);
  HIPCK(hipMalloc(&p, size_t(std::max(g->V, 1)) * sizeof(int32_t)));
  g->head = static_cast<int32_t*>(p);
  HIPCK(launch_slab(s, g->colptr, g->rowind, g->V, g->slab, g->head));
  HIPCK(hipStreamSynchronize(s));
  return DOBFS_OK;
}

void free_graph(dobfs_graph g) {
  if (!g) return;
  for (void* p : g->owned)
    if (p) (void)hipFree(p);
  if (g->nz_in) (void)hipFree(g->nz_in);
  if (g->heavy) (void)hipFree(g->heavy);
  if (g->slab) (void)hipFree(g->slab);
  if (g->head) (void)hipFree(g->head);
  if (g->ws) (void)hipFree(g->ws);
  if (g->ws_event) (void)hipEventDestroy(g->ws_event);
  delete g;
}

// The graph's own workspace, held by one call: its lock, and on release an
// event on the call's stream. When a call returns, blocks of its last kernel
// may still be reading the control block (a step past the end has nothing
// to write, so the report does not wait for it); the next call that takes
// the workspace on another stream waits for that event before its first
// kernel, so nothing it writes can reach those blocks.
struct WsLease {
  std::unique_lock<std::mutex> lock;
  dobfs_graph g = nullptr;
  hipStream_t s = nullptr;
  WsLease() = default;
  WsLease(const WsLease&) = delete;
  WsLease& operator=(const WsLease&) = delete;
  ~WsLease() {
    if (g) (void)hipEventRecord(g->ws_event, s);
  }
};

// Workspace for a call: the caller's, or the graph's own (grown on demand;
// the lease holds its lock for the duration of the call and orders it after
// the previous call on the graph's workspace).
dobfs_status get_workspace(dobfs_graph g, void* workspace, size_t ws_bytes, size_t need, hipStream_t s,
                           WsLease& lease, uint8_t** base) {
  if (workspace) {
    if (ws_bytes < need)
      return fail(DOBFS_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes,
                  need);
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(DOBFS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    *base = static_cast<uint8_t*>(workspace);
    return DOBFS_OK;
  }
  lease.lock = std::unique_lock<std::mutex>(g->mu);
  if (!g->ws_event) HIPCK(hipEventCreateWithFlags(&g->ws_event, hipEventDisableTiming));
  if (g->ws_event_recorded) HIPCK(hipStreamWaitEvent(s, g->ws_event, 0));
  g->ws_event_recorded = true;
  lease.g = g;
  lease.s = s;
  if (g->ws_size < need) {
    if (g->ws) {
      HIPCK(hipDeviceSynchronize());
      HIPCK(hipFree(g->ws));
      g->ws = nullptr;
      g->ws_size = 0;
    }
    HIPCK(hipMalloc(&g->ws, need));
    g->ws_size = need;
  }
  *base = static_cast<uint8_t*>(g->ws);
  return DOBFS_OK;
}


// The argument block of a single-source traversal over workspace `ws`.
BfsArgs bfs_args(dobfs_graph g, uint8_t* ws, const Layout& L, const dobfs_options& opt, int32_t* depth,
                 int32_t* parent) {
  BfsArgs a{};
  a.V = g->V;
  a.nwords = g->nwords;
  a.nnz = g->nnz;
  a.rowptr = g->rowptr;
  a.colind = g->colind;
  a.colptr = g->colptr;
  a.rowind = g->rowind;
  a.slab = g->slab;
  a.head = g->head;
  a.nz_in = g->nz_in;
  a.heavy = g->heavy;
  a.depth = depth;
  a.parent = parent;
  a.vis[0] = reinterpret_cast<uint32_t*>(ws + L.visA);
  a.vis[1] = reinterpret_cast<uint32_t*>(ws + L.visB);
  a.F[0] = reinterpret_cast<uint32_t*>(ws + L.FA);
  a.F[1] = reinterpret_cast<uint32_t*>(ws + L.FB);
  a.Q[0] = reinterpret_cast<int32_t*>(ws + L.Q0);
  a.Q[1] = reinterpret_cast<int32_t*>(ws + L.Q1);
  a.S = reinterpret_cast<int32_t*>(ws + L.S);
  a.R = reinterpret_cast<int32_t*>(ws + L.R);
  a.chunk_first = reinterpret_cast<int32_t*>(ws + L.chunks);
  a.flagsA = reinterpret_cast<uint64_t*>(ws + L.flagsA);
  a.flagsB = reinterpret_cast<uint64_t*>(ws + L.flagsB);
  a.ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  a.mode = opt.mode;
  a.heuristic = opt.heuristic;
  a.alpha = double(opt.alpha);
  a.beta = double(opt.beta);
  a.reuse = (opt.mode == DOBFS_MODE_FULL || opt.mode == DOBFS_MODE_PULL_ONLY ||
             opt.mode == DOBFS_MODE_PUSH_ONLY) ? 1 : 0;
  a.early_exit = (opt.mode != DOBFS_MODE_PULL_MASKED && opt.mode != DOBFS_MODE_PULL_UNMASKED) ? 1 : 0;
  a.mask_after = opt.mode == DOBFS_MODE_PULL_UNMASKED ? 1 : 0;
  a.need_F = a.reuse ? 0 : 1;
  a.edge_rule = opt.heuristic == DOBFS_HEUR_EDGES ? 1 : 0;
  a.local_push = a.need_F ? 0 : 1;  // (the frontier bitmap a push writes is cleared by its scan step)
  a.low_degree = g->max_outdeg <= uint32_t(kLocalDeg) ? 1 : 0;
  a.sched = default_sched();
  if (opt.pull_mid) a.sched.pull_mid = opt.pull_mid;
  if (opt.bitmap_rows) a.sched.bitmap_rows = opt.bitmap_rows;
  if (opt.local_unit) a.sched.local_unit = opt.local_unit;
  if (opt.local_chunks) a.sched.local_chunks = opt.local_chunks;
  return a;
}

// Result of a level loop.
struct LoopResult {
  int64_t levels = 0;   // levels run (the last discovered nothing)
  int64_t sum_new = 0;  // vertices discovered over all levels
  int64_t sum_aux = 0;  // multi-source: (vertex, source) pairs discovered
  LevelState end{};     // state after the last level
  int32_t n_main = 0, n_aux = 0;            // every launch of the step kernel (n_aux: 0)
  float ms_main_all = 0.f, ms_aux_all = 0.f;  // their execution times (when timing; ms_aux_all: 0)
};

// The persistent step loop on one device: how many of its blocks fit at once
// (its grid), the wall-clock rate, and a lock held from one of its launches
// until that launch's report is in. A launch waits at its barriers only
// until its report is written, so with the lock no two launches of the loop
// ever wait on each other for room on the device.
struct PersistentDevice {
  std::mutex mu;
  std::once_flag once;
  int32_t capacity = 0;       // blocks of k_steps that fit at once; 0: the loop is not available
  int32_t capacity_mb = 0;    // the same for k_mb_steps
  double ticks_per_ms = 0.0;  // device wall clock
};
PersistentDevice g_persistent[64];

PersistentDevice* persistent_device(int device) {
  if (device < 0 || device >= 64) return nullptr;
  PersistentDevice* d = &g_persistent[device];
  std::call_once(d->once, [d, device]() {
    int32_t cap = 0, cap_mb = 0;
    int khz = 0;
    if (persistent_capacity(&cap) == hipSuccess && persistent_capacity_mb(&cap_mb) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0 &&
        cap_mb > 0) {
      d->capacity = cap;
      d->capacity_mb = cap_mb;
      d->ticks_per_ms = double(khz);
    }
  });
  return d->capacity > 0 ? d : nullptr;
}

uint32_t env_u32(const char* name, uint32_t dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  const unsigned long long x = std::strtoull(v, nullptr, 10);
  return x > 0xffffffffull ? 0xffffffffu : uint32_t(x);
}

// How run_steps launches the steps of one traversal kind. step(): step k on `blocks` blocks (0:
// the kind's full grid; rp: this step also writes the batch's report, only where self_report);
// before_report(): what must run after a batch's last step (k_last) and before its report;
// persistent(): the persistent form of a batch (rp as for step()); grid(): the full grid of a
// step launch; next_grid(): the blocks for the next batch's launches from the report of the
// batch before (0: the full grid); capacity(): blocks of the persistent kernel that fit at once.
struct SingleSteps {
  const BfsArgs& a;
  static constexpr bool self_report = true;
  int64_t grid() const { return main_blocks(a.nwords); }
  int64_t next_grid(const HostReport&, int32_t) const { return 0; }
  static int32_t capacity(const PersistentDevice& d) { return d.capacity; }
  hipError_t step(hipStream_t s, int32_t k, int64_t, hipEvent_t t0, hipEvent_t t1, const StepReportArgs* rp) const {
    return launch_step(s, a, k, t0, t1, rp);
  }
  hipError_t before_report(hipStream_t, int32_t) const { return hipSuccess; }
  hipError_t persistent(hipStream_t s, int32_t s_first, int32_t n, int32_t blocks, uint32_t spin_limit,
                        bool timing, const StepReportArgs& rp, hipEvent_t t0, hipEvent_t t1) const {
    return launch_steps(s, a, s_first, n, blocks, spin_limit, timing, rp, t0, t1);
  }
};
struct BatchSteps {
  const BatchArgs& a;
  const DepthRows& rows;
  static constexpr bool self_report = false;
  int64_t grid() const {
    return std::max<int64_t>(kExpandBlocks, std::min<int64_t>((int64_t(a.nwords) + kMbTileWords - 1) / kMbTileWords, 8192));
  }
  // Every block of a step decides the level before its work, so a long run of push levels (a
  // high-diameter graph) need not pay for a pull's grid: after a batch without a pull, the next
  // batch's launches get four times the blocks its largest push needed (scan tiles of the
  // frontiers, edge chunks), at least 256. Every body strides over whatever grid it gets, so a
  // pull that comes anyway is only slower.
  int64_t next_grid(const HostReport& r, int32_t batch) const {
    int64_t need = 0;
    for (int32_t k = 0; k < batch; ++k) {
      const LevelState& st = r.steps[k];
      if (st.done) break;
      if (st.dir != DOBFS_DIR_PUSH) return 0;
      need = std::max<int64_t>(need, (int64_t(st.nf) + kScanTile - 1) / kScanTile);
    }
    for (int32_t k = 0; k < r.nrec; ++k) {
      const LevelRecord& x = r.rec[k];
      if (x.dir != DOBFS_DIR_PUSH) return 0;
      need = std::max<int64_t>(need, (x.m_f + kExpandChunk - 1) / kExpandChunk);
      need = std::max<int64_t>(need, (int64_t(x.n_new) + kScanTile - 1) / kScanTile);
    }
    const int64_t g = std::max<int64_t>(256, 4 * need);
    return g < grid() ? g : 0;
  }
  static int32_t capacity(const PersistentDevice& d) { return d.capacity_mb; }
  hipError_t step(hipStream_t s, int32_t k, int64_t blocks, hipEvent_t t0, hipEvent_t t1,
                  const StepReportArgs*) const {
    return launch_mb_step(s, a, k, blocks, t0, t1);
  }
  // the depth rows: a transpose that exits at once unless the state the batch's last step
  // published says the traversal is over, so the last report already finds the rows final
  hipError_t before_report(hipStream_t s, int32_t k_last) const { return launch_mb_depth(s, a, k_last, rows); }
  hipError_t persistent(hipStream_t s, int32_t s_first, int32_t n, int32_t blocks, uint32_t spin_limit,
                        bool timing, const StepReportArgs&, hipEvent_t t0, hipEvent_t t1) const {
    return launch_mb_steps(s, a, s_first, n, blocks, spin_limit, timing, t0, t1);
  }
};

// The level loop of both traversal kinds: the host enqueues steps (one launch
// each) in batches and reads back, once per batch, the state every step
// published and the records of the levels that are complete; steps enqueued
// past the end exit at once. The first batch is one step longer than the
// previous traversal of the same kind on the graph needed; later batches start
// at 4 and double. When timing, step k of a batch has events ev_m0(k) /
// ev_m1(k); a level's scan step counts as its ms_aux, its other step as its
// ms_main. With `pd` (persistent loop on that device) a batch is one launch of
// the persistent kernel running the batch's steps, with the same report;
// per-step times then come from the device clock at each step's start (and the
// launch's end).
// max_levels: a traversal that reaches that many levels fails with too_deep.
template <class Steps>
dobfs_status run_steps(std::atomic<int32_t>& last_steps, hipStream_t s, bool timing, hipEvent_t* ev,
                       const Steps& S, const Ctrl* ctrl, int64_t max_steps, int64_t max_levels,
                       dobfs_status too_deep, const ReportSink& sink, PersistentDevice* pd,
                       dobfs_stats* stats, LoopResult* res) {
  HostReport* rep = sink.host;
  int64_t s0 = 0;
  int32_t rec_first = 0;
  int32_t batch = std::min(std::max(last_steps.load(std::memory_order_relaxed) + 1, 2), kMaxBatch);
  int32_t next_batch = 4;
  auto E = [&](int i) -> hipEvent_t { return timing ? ev[i] : nullptr; };
  const int32_t cap = pd ? Steps::capacity(*pd) : 0;
  const int32_t blocks =
      pd ? int32_t(std::min<int64_t>(S.grid(), int64_t(env_u32("DOBFS_PERSIST_BLOCKS", uint32_t(cap))))) : 0;
  const uint32_t spin_limit = env_u32("DOBFS_SPIN_LIMIT", 1u << 22);
  if (pd && (blocks < 1 || blocks > cap))
    return fail(DOBFS_ERR_INVALID_ARG, "persistent grid of %d blocks (1 .. %d fit)", blocks, cap);
  if (pd) batch = next_batch = kMaxBatch;  // a launch ends with the traversal: no steps past the end
  int64_t grid = 0;  // blocks of the step launches (0: the full grid)
  while (true) {
    if (s0 + batch > max_steps) batch = int32_t(max_steps - s0);
    const uint32_t seq = next_report_seq();
    // untimed, the batch's last step writes the report; timed, a report kernel follows the
    // steps so that every step's end event has completed when the host reads it
    const StepReportArgs rp{sink.dev, seq, int32_t(s0), rec_first};
    const bool self = Steps::self_report && !timing;
    if (pd) {
      std::lock_guard<std::mutex> lk(pd->mu);
      HIPCK(S.persistent(s, int32_t(s0), batch, blocks, spin_limit, timing,
                         self ? rp : StepReportArgs{nullptr, 0u, 0, 0}, E(ev_m0(0)), E(ev_m1(0))));
      HIPCK(S.before_report(s, int32_t(s0 + batch - 1)));
      if (!self) HIPCK(launch_step_report(s, ctrl, int32_t(s0), batch, rec_first, sink.dev, seq));
      HIPCK(fetch_report(sink, seq, s));
    } else {
      for (int32_t k = 0; k < batch; ++k)
        HIPCK(S.step(s, int32_t(s0 + k), grid, E(ev_m0(k)), E(ev_m1(k)), (self && k == batch - 1) ? &rp : nullptr));
      HIPCK(S.before_report(s, int32_t(s0 + batch - 1)));
      if (!self) HIPCK(launch_step_report(s, ctrl, int32_t(s0), batch, rec_first, sink.dev, seq));
      HIPCK(fetch_report(sink, seq, s));
    }
    if (rep->error) {
      (void)hipStreamSynchronize(s);
      return fail(DOBFS_ERR_INTERNAL, "a grid barrier wait of the persistent level loop gave up "
                                      "(spin limit %u polls)", spin_limit);
    }
    res->n_main += pd ? 1 : batch;
    if (pd && timing) res->ms_main_all += elapsed(ev[ev_m0(0)], ev[ev_m1(0)]);
    for (int32_t k = 0; k < batch; ++k) {  // step times, by level
      float t = 0.f;
      if (timing && !pd) {
        t = elapsed(ev[ev_m0(k)], ev[ev_m1(k)]);
        res->ms_main_all += t;
      } else if (timing && !rep->steps[k].done) {  // to the next step's start, or the launch's end
        const unsigned long long t1 =
            (k + 1 < batch && !rep->steps[k + 1].done) ? rep->steps[k + 1].t0 : rep->t_end;
        t = float(double(t1 - rep->steps[k].t0) / pd->ticks_per_ms);
      }
      const LevelState& st = rep->steps[k];
      if (st.done || !stats || st.level >= stats->cap) continue;
      dobfs_level_stats& ls = stats->level[st.level];
      if (st.phase != kPhaseExpand) ls.ms_aux = ls.ms_main = 0.f;  // the level's first step
      if (st.phase == kPhaseScan) ls.ms_aux = t; else ls.ms_main += t;
    }
    for (int32_t k = 0; k < rep->nrec; ++k) {  // records of the levels now complete
      const LevelRecord& r = rep->rec[k];
      const int32_t l = rec_first + k;
      res->sum_new += r.n_new;
      res->sum_aux += int64_t(r.aux);
      if (stats && l < stats->cap) {
        dobfs_level_stats& ls = stats->level[l];
        ls.dir = r.dir;
        ls.nf = r.nf;
        ls.n_new = r.n_new;
        ls.variant = r.variant;
        ls.edges = r.edges;
        ls.m_f = r.m_f;
      }
    }
    rec_first += rep->nrec;
    grid = S.next_grid(*rep, batch);
    const LevelState& end = rep->end;
    if (end.done) {
      res->levels = end.levels;
      res->end = end;
      break;
    }
    if (int64_t(end.level) + 1 >= max_levels) {
      (void)hipStreamSynchronize(s);
      return fail(too_deep, "traversal needs more than %lld levels", (long long)max_levels);
    }
    if (s0 + batch >= max_steps) {
      (void)hipStreamSynchronize(s);
      return fail(DOBFS_ERR_INTERNAL, "traversal needs more than %lld steps", (long long)max_steps);
    }
    s0 += batch;
    batch = next_batch;
    next_batch = std::min(2 * next_batch, kMaxBatch);
  }
  // steps the traversal used, up to the one that found the end (the batch before ended short of it)
  int32_t k_end = 0;
  while (k_end + 1 < batch && !rep->steps[k_end].done) ++k_end;
  last_steps.store(int32_t(s0) + k_end + 1, std::memory_order_relaxed);
  return DOBFS_OK;
}

// stats->edges_g500 after a single-source traversal into depth: the out-degree sum of the
// reached vertices, counted on the device, halved for a graph given as undirected.
// `tail` receives the device's counters (host memory, pinned or not).
dobfs_status reached_edges(dobfs_graph g, hipStream_t s, Ctrl* ctrl, const int32_t* depth,
                           dobfs_stats* stats, LevelSlot* tail) {
  HIPCK(launch_reached_degree(s, g->rowptr, depth, g->V, &ctrl->tail));
  HIPCK(hipMemcpyAsync(tail, &ctrl->tail, sizeof(LevelSlot), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  const int64_t sum = int64_t(sum_slot(*tail).edges);
  stats->edges_g500 = g->symmetric ? sum / 2 : sum;
  return DOBFS_OK;
}

// The sort-based push of Table 2's first row: push at every level with the
// pairs gathered, radix-sorted by key and reduced to their first element
// per key (Algorithm 3 as printed). The first kernel of each level (state +
// frontier scan) is shared with the atomic push; the host reads the level's
// state and edge count back before sizing the sort, as the paper's loop does.
dobfs_status bfs_sort_push(dobfs_graph g, int32_t source, const dobfs_options& opt_in, int32_t* depth,
                           int32_t* parent, void* workspace, size_t ws_bytes, void* stream,
                           dobfs_stats* stats) {
  const SortLayout SL = plan_sort(g->V, g->nnz);
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsLease lease;
  uint8_t* ws = nullptr;
  dobfs_status st = get_workspace(g, workspace, ws_bytes, SL.total, s, lease, &ws);
  if (st != DOBFS_OK) return st;
  hipEvent_t* ev = events_for(g->device);
  if (!ev) return fail(DOBFS_ERR_DEVICE, "event creation failed");
  const bool keys_only = opt_in.mode == DOBFS_MODE_PUSH_SORT_KEYS;
  dobfs_options opt = opt_in;
  opt.mode = DOBFS_MODE_PUSH_ONLY;  // the level state machine: push at every level
  BfsArgs a = bfs_args(g, ws, SL.base, opt, depth, parent);
  a.local_push = 0;  // the gather reads the frontier scan's chunk table
  a.edge_rule = 0;
  uint32_t* kA = reinterpret_cast<uint32_t*>(ws + SL.kA);
  uint32_t* kB = reinterpret_cast<uint32_t*>(ws + SL.kB);
  int32_t* vA = reinterpret_cast<int32_t*>(ws + SL.vA);
  int32_t* vB = reinterpret_cast<int32_t*>(ws + SL.vB);
  void* tmp = ws + SL.tmp;
  int bits = 1;
  while (bits < 32 && (int64_t(1) << bits) < int64_t(g->V)) ++bits;
  Ctrl* c = a.ctrl;
  Ctrl* hc = host_ctrl();
  if (!hc) return fail(DOBFS_ERR_OUT_OF_MEMORY, "pinned host buffer");

  HIPCK(hipEventRecord(ev[kEvStart], s));
  HIPCK(launch_bfs_init(s, a, source, DOBFS_DIR_PUSH));
  int64_t levels = 0, reached = 1;
  for (int32_t L = 0;; ++L) {
    if (int64_t(L) > int64_t(g->V) + 1) return fail(DOBFS_ERR_INTERNAL, "level loop did not terminate");
    HIPCK(launch_level_prep(s, a, L, -1));
    HIPCK(hipMemcpyAsync(&hc->ring[0], &c->ring[L % kRing], sizeof(LevelState), hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(&hc->mf[0], &c->mf[L % kSlots], sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    if (L >= 1)
      HIPCK(hipMemcpyAsync(&hc->rec[0], &c->rec[(L - 1) % kRing], sizeof(LevelRecord), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    const LevelState stL = hc->ring[0];
    if (L >= 1) {
      const LevelRecord& r = hc->rec[0];
      reached += r.n_new;
      if (stats && L - 1 < stats->cap) {
        dobfs_level_stats& ls = stats->level[L - 1];
        ls.dir = r.dir;
        ls.nf = r.nf;
        ls.n_new = r.n_new;
        ls.variant = 0;
        ls.edges = r.edges;
        ls.m_f = r.m_f;
        ls.ms_main = 0.f;
        ls.ms_aux = 0.f;
      }
    }
    if (stL.done) {
      levels = stL.levels;
      break;
    }
    const uint32_t m = hc->mf[0];
    if (m == 0) continue;  // nothing to gather: the next level's state sees no discovery
    ExpandArgs e{};
    e.Q = a.Q[L % 2];
    e.nf = stL.nf;
    e.S = a.S;
    e.R = a.R;
    e.chunk_first = a.chunk_first;
    e.colind = a.colind;
    e.m = m;
    if (keys_only) {  // structure only: the neighbours alone, no frontier vertex alongside
      HIPCK(launch_sort_gather(s, e, kA, nullptr));
      HIPCK(sort_keys(s, tmp, SL.tmp_bytes, kA, kB, m, bits));
      HIPCK(launch_sort_filter(s, kB, nullptr, m, a.vis[stL.vis_idx], depth, nullptr, L, a.Q[(L + 1) % 2],
                               &c->qcount[L % kSlots], &c->slot[L % kSlots]));
    } else {
      HIPCK(launch_sort_gather(s, e, kA, vA));
      HIPCK(sort_pairs(s, tmp, SL.tmp_bytes, kA, kB, vA, vB, m, bits));
      HIPCK(launch_sort_filter(s, kB, vB, m, a.vis[stL.vis_idx], depth, parent, L, a.Q[(L + 1) % 2],
                               &c->qcount[L % kSlots], &c->slot[L % kSlots]));
    }
  }
  HIPCK(hipEventRecord(ev[kEvEnd], s));
  HIPCK(hipEventSynchronize(ev[kEvEnd]));
  if (stats) {
    stats->levels = int32_t(levels);
    stats->ms_total = elapsed(ev[kEvStart], ev[kEvEnd]);
    stats->ms_init = 0.f;
    stats->reached = reached;
    stats->launches_main = stats->launches_aux = 0;
    stats->ms_main_all = stats->ms_aux_all = 0.f;
    return reached_edges(g, s, c, depth, stats, &hc->tail);
  }
  return DOBFS_OK;
}

// Checks shared by the single-source entry points; *opt receives the options in force.
dobfs_status check_bfs_call(dobfs_graph g, int32_t source, const dobfs_options* opt_in, const int32_t* depth,
                            const dobfs_stats* stats, dobfs_options* opt) {
  if (!g) return fail(DOBFS_ERR_INVALID_ARG, "graph is NULL");
  if (!depth) return fail(DOBFS_ERR_INVALID_ARG, "depth is NULL");
  if (source < 0 || source >= g->V)
    return fail(DOBFS_ERR_INVALID_ARG, "source %d not in [0, %d)", source, g->V);
  *opt = opt_in ? *opt_in : defaults();
  dobfs_status st = check_options(*opt);
  if (st != DOBFS_OK) return st;
  if (stats && stats->cap > 0 && !stats->level)
    return fail(DOBFS_ERR_INVALID_ARG, "stats->level is NULL with cap = %d", stats->cap);
  return DOBFS_OK;
}

// One single-source traversal (Algorithm 1) over workspace `ws` laid out as L, on stream s:
// the init kernel, then the step loop. ev: the thread's events (nullptr: no events, so no
// times in the stats); tail: host memory for the reached-edge count.
dobfs_status bfs_steps(dobfs_graph g, int32_t source, const dobfs_options& opt, int32_t* depth,
                       int32_t* parent, uint8_t* ws, const Layout& L, hipStream_t s, const ReportSink& sink,
                       hipEvent_t* ev, LevelSlot* tail, dobfs_stats* stats) {
  const bool timing = ev && (opt.flags & DOBFS_OPT_TIME_KERNELS) != 0;
  BfsArgs a = bfs_args(g, ws, L, opt, depth, parent);
  const int32_t dir0 = opt.n_forced > 0 ? int32_t(opt.forced_dirs[0])
                                        : (opt.mode == DOBFS_MODE_PULL_ONLY ? DOBFS_DIR_PULL : DOBFS_DIR_PUSH);
  a.n_forced = std::min<int32_t>(opt.n_forced, kRing);  // later levels follow the rule
  if (a.n_forced > 0)
    HIPCK(hipMemcpyAsync(a.ctrl->forced, opt.forced_dirs, size_t(a.n_forced), hipMemcpyHostToDevice, s));

  // the whole-call interval only when asked for: the last batch's report already tells the
  // host that every kernel of the traversal has finished, so no further wait is needed
  if (stats && ev) HIPCK(hipEventRecord(ev[kEvStart], s));
  HIPCK(launch_bfs_init(s, a, source, dir0, timing ? ev[kEvInit0] : nullptr,
                        timing ? ev[kEvInit1] : nullptr));
  LoopResult res;
  // a level takes at most two steps; scan tile flags carry 2 * step + 2 in 30 bits
  const int64_t max_steps = std::min<int64_t>(2 * (int64_t(g->V) + 2), (int64_t(1) << 29) - 2);
  PersistentDevice* pd = nullptr;
  if (opt.flags & DOBFS_OPT_PERSISTENT) {
    pd = persistent_device(g->device);
    if (!pd) return fail(DOBFS_ERR_UNSUPPORTED, "the persistent level loop is not available on device %d", g->device);
  }
  dobfs_status st = run_steps(g->last_steps, s, timing, ev, SingleSteps{a}, a.ctrl, max_steps,
                              INT64_MAX, DOBFS_ERR_INTERNAL, sink, pd, stats, &res);
  if (st != DOBFS_OK) return st;
  if (stats) {
    if (ev) {
      HIPCK(hipEventRecord(ev[kEvEnd], s));
      HIPCK(hipEventSynchronize(ev[kEvEnd]));
    }
    stats->levels = int32_t(res.levels);
    stats->ms_total = ev ? elapsed(ev[kEvStart], ev[kEvEnd]) : 0.f;
    stats->ms_init = timing ? elapsed(ev[kEvInit0], ev[kEvInit1]) : 0.f;
    stats->reached = 1 + res.sum_new;
    stats->launches_main = res.n_main;
    stats->launches_aux = res.n_aux;
    stats->ms_main_all = res.ms_main_all;
    stats->ms_aux_all = res.ms_aux_all;
    return reached_edges(g, s, a.ctrl, depth, stats, tail);
  }
  return DOBFS_OK;
}

// ---- the allocation-free single-source call ----
// Its workspace and level report live in `scratch`, one copy per device that
// loads the library, held until the process ends. Host code never passes the
// symbol itself to a kernel: its device address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticScratchBytes = DOBFS_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[64] = {};

// Device address of `scratch` on `device` (current when called).
dobfs_status static_scratch(int device, uint8_t** out) {
  if (device < 0 || device >= 64) return fail(DOBFS_ERR_INVALID_ARG, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __LINE__);
    if (!p) return fail(DOBFS_ERR_DEVICE, "static scratch has no address on device %d", device);
    g_scratch_ptr[device] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch_ptr[device];
  return DOBFS_OK;
}

}  // namespace

extern "C" {

const char* dobfs_status_string(dobfs_status s) {
  switch (s) {
    case DOBFS_OK: return "DOBFS_OK";
    case DOBFS_ERR_INVALID_ARG: return "DOBFS_ERR_INVALID_ARG";
    case DOBFS_ERR_OUT_OF_MEMORY: return "DOBFS_ERR_OUT_OF_MEMORY";
    case DOBFS_ERR_DEVICE: return "DOBFS_ERR_DEVICE";
    case DOBFS_ERR_WORKSPACE_TOO_SMALL: return "DOBFS_ERR_WORKSPACE_TOO_SMALL";
    case DOBFS_ERR_UNSUPPORTED: return "DOBFS_ERR_UNSUPPORTED";
    case DOBFS_ERR_INTERNAL: return "DOBFS_ERR_INTERNAL";
    case DOBFS_ERR_TIMEOUT: return "DOBFS_ERR_TIMEOUT";
  }
  return "DOBFS_ERR_UNKNOWN";
}

const char* dobfs_last_error(void) { return t_last_error.c_str(); }

int32_t dobfs_version(void) { return 100; }

dobfs_status dobfs_options_default(dobfs_options* opt) {
  if (!opt) return fail(DOBFS_ERR_INVALID_ARG, "opt is NULL");
  *opt = defaults();
  return DOBFS_OK;
}

int32_t dobfs_next_direction(const dobfs_options* opt, int32_t dir, int64_t V, int64_t nf,
                             int64_t n_new, int64_t m_f, int64_t m_u) {
  const dobfs_options o = opt ? *opt : defaults();
  return next_direction_rule(o.heuristic, double(o.alpha), double(o.beta), dir, V, nf, n_new, m_f,
                             m_u);
}

dobfs_status dobfs_graph_upload(int32_t V, int64_t nnz, const int32_t* csr_rowptr,
                                const int32_t* csr_colind, const int32_t* csc_colptr,
                                const int32_t* csc_rowind, int32_t device, uint32_t flags,
                                dobfs_graph* out) {
  t_last_error.clear();
  dobfs_status st = check_args(V, nnz, csr_rowptr, csr_colind, csc_colptr, csc_rowind, device, out);
  if (st != DOBFS_OK) return st;
  if (flags & ~uint32_t(DOBFS_UPLOAD_VALIDATE | DOBFS_UPLOAD_HUBS_FIRST))
    return fail(DOBFS_ERR_INVALID_ARG, "unknown upload flags 0x%x", flags);
  if ((st = check_offsets_host(V, nnz, csr_rowptr, "csr_rowptr")) != DOBFS_OK) return st;
  if ((st = check_offsets_host(V, nnz, csc_colptr, "csc_colptr")) != DOBFS_OK) return st;
  {  // indices are always checked: an out-of-range entry would send kernels out of bounds
    for (int64_t p = 0; p < nnz; ++p) {
      if (csr_colind[p] < 0 || csr_colind[p] >= V)
        return fail(DOBFS_ERR_INVALID_ARG, "csr_colind[%lld] = %d out of range", (long long)p,
                    csr_colind[p]);
      if (csc_rowind[p] < 0 || csc_rowind[p] >= V)
        return fail(DOBFS_ERR_INVALID_ARG, "csc_rowind[%lld] = %d out of range", (long long)p,
                    csc_rowind[p]);
    }
  }
  if ((st = check_device(device)) != DOBFS_OK) return st;
  DeviceScope ds(device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice", __LINE__);
  dobfs_graph g = new dobfs_graph_s;
  g->device = device;
  g->V = V;
  g->nnz = nnz;
  g->nwords = words_of(V);
  const bool shared = (csr_rowptr == csc_colptr) && (csr_colind == csc_rowind);
  g->symmetric = shared;
  auto upload = [&](const int32_t* src, size_t n, int slot) -> const int32_t* {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * 4) != hipSuccess) return nullptr;
    g->owned[slot] = p;
    if (n && hipMemcpy(p, src, n * 4, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return static_cast<const int32_t*>(p);
  };
  g->rowptr = upload(csr_rowptr, size_t(V) + 1, 0);
  g->colind = g->rowptr ? upload(csr_colind, size_t(nnz), 1) : nullptr;
  if (shared) {
    g->colptr = g->rowptr;
    g->rowind = g->colind;
  } else if (g->colind) {
    g->colptr = upload(csc_colptr, size_t(V) + 1, 2);
    g->rowind = g->colptr ? upload(csc_rowind, size_t(nnz), 3) : nullptr;
  }
  if (!g->rowptr || !g->colind || !g->colptr || !g->rowind) {
    hipError_t e = hipGetLastError();
    free_graph(g);
    return hip_fail(e == hipSuccess ? hipErrorOutOfMemory : e, "graph upload", __LINE__);
  }
  if ((st = finish_graph(g, nullptr, flags)) != DOBFS_OK) {
    free_graph(g);
    return st;
  }
  *out = g;
  return DOBFS_OK;
}

dobfs_status dobfs_graph_wrap_device(int32_t V, int64_t nnz, const int32_t* csr_rowptr,
                                     const int32_t* csr_colind, const int32_t* csc_colptr,
                                     const int32_t* csc_rowind, int32_t device, uint32_t flags,
                                     void* stream, dobfs_graph* out) {
  t_last_error.clear();
  dobfs_status st = check_args(V, nnz, csr_rowptr, csr_colind, csc_colptr, csc_rowind, device, out);
  if (st != DOBFS_OK) return st;
  if (flags & ~uint32_t(DOBFS_UPLOAD_VALIDATE | DOBFS_UPLOAD_HUBS_FIRST))
    return fail(DOBFS_ERR_INVALID_ARG, "unknown upload flags 0x%x", flags);
  if ((st = check_device(device)) != DOBFS_OK) return st;
  DeviceScope ds(device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice", __LINE__);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t* err = nullptr;
  HIPCK(hipMalloc(&err, 4));
  int32_t herr = 0;
  hipError_t e = hipMemsetAsync(err, 0, 4, s);
  if (e == hipSuccess) e = launch_check_offsets(s, csr_rowptr, V, nnz, err);
  if (e == hipSuccess) e = launch_check_offsets(s, csc_colptr, V, nnz, err);
  if (e == hipSuccess && nnz > 0) {  // indices always checked (see dobfs_graph_upload)
    e = launch_check_indices(s, csr_colind, nnz, V, err);
    if (e == hipSuccess) e = launch_check_indices(s, csc_rowind, nnz, V, err);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(err);
  if (e != hipSuccess) return hip_fail(e, "device offset check", __LINE__);
  if (herr) return fail(DOBFS_ERR_INVALID_ARG, "device graph arrays failed checks (code %d)", herr);
  dobfs_graph g = new dobfs_graph_s;
  g->device = device;
  g->V = V;
  g->nnz = nnz;
  g->nwords = words_of(V);
  g->rowptr = csr_rowptr;
  g->colind = csr_colind;
  g->colptr = csc_colptr;
  g->rowind = csc_rowind;
  g->symmetric = (csr_rowptr == csc_colptr) && (csr_colind == csc_rowind);
  if ((st = finish_graph(g, s, flags)) != DOBFS_OK) {
    free_graph(g);
    return st;
  }
  *out = g;
  return DOBFS_OK;
}

dobfs_status dobfs_graph_destroy(dobfs_graph g) {
  t_last_error.clear();
  if (!g) return DOBFS_OK;
  DeviceScope ds(g->device);
  free_graph(g);
  return DOBFS_OK;
}

dobfs_status dobfs_graph_info(dobfs_graph g, int32_t* V, int64_t* nnz, int32_t* device) {
  if (!g) return fail(DOBFS_ERR_INVALID_ARG, "graph is NULL");
  if (V) *V = g->V;
  if (nnz) *nnz = g->nnz;
  if (device) *device = g->device;
  return DOBFS_OK;
}

dobfs_status dobfs_bfs_workspace_bytes(dobfs_graph g, const dobfs_options* opt, size_t* bytes) {
  if (!g || !bytes) return fail(DOBFS_ERR_INVALID_ARG, "graph or bytes is NULL");
  *bytes = (opt && (opt->mode == DOBFS_MODE_PUSH_SORT || opt->mode == DOBFS_MODE_PUSH_SORT_KEYS))
               ? plan_sort(g->V, g->nnz).total
                                                       : plan(g->V, g->nnz).total;
  return DOBFS_OK;
}

dobfs_status dobfs_mxv_workspace_bytes(dobfs_graph g, size_t* bytes) {
  if (!g || !bytes) return fail(DOBFS_ERR_INVALID_ARG, "graph or bytes is NULL");
  *bytes = plan(g->V, g->nnz).total;
  return DOBFS_OK;
}
dobfs_status dobfs_bfs(dobfs_graph g, int32_t source, const dobfs_options* opt_in, int32_t* depth,
                       int32_t* parent, void* workspace, size_t ws_bytes, void* stream,
                       dobfs_stats* stats) {
  t_last_error.clear();
  dobfs_options opt;
  dobfs_status st = check_bfs_call(g, source, opt_in, depth, stats, &opt);
  if (st != DOBFS_OK) return st;
  DeviceScope ds(g->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice", __LINE__);
  if (opt.mode == DOBFS_MODE_PUSH_SORT_KEYS && parent)
    return fail(DOBFS_ERR_INVALID_ARG, "the key-only sort push computes no parents: parent must be NULL");
  if (opt.mode == DOBFS_MODE_PUSH_SORT || opt.mode == DOBFS_MODE_PUSH_SORT_KEYS)
    return bfs_sort_push(g, source, opt, depth, parent, workspace, ws_bytes, stream, stats);
  const Layout L = plan(g->V, g->nnz);
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsLease lease;
  uint8_t* ws = nullptr;
  if ((st = get_workspace(g, workspace, ws_bytes, L.total, s, lease, &ws)) != DOBFS_OK) return st;
  HostReport* rep = host_report();
  Ctrl* hc = host_ctrl();
  if (!rep || !hc) return fail(DOBFS_ERR_OUT_OF_MEMORY, "pinned host buffer");
  hipEvent_t* ev = events_for(g->device);
  if (!ev) return fail(DOBFS_ERR_DEVICE, "event creation failed");
  return bfs_steps(g, source, opt, depth, parent, ws, L, s, ReportSink{rep, rep}, ev, &hc->tail, stats);
}

dobfs_status dobfs_bfs_static(dobfs_graph g, int32_t source, const dobfs_options* opt_in, int32_t* depth,
                              int32_t* parent, void* stream, dobfs_stats* stats) {
  t_last_error.clear();
  dobfs_options opt;
  dobfs_status st = check_bfs_call(g, source, opt_in, depth, stats, &opt);
  if (st != DOBFS_OK) return st;
  if (opt.mode == DOBFS_MODE_PUSH_SORT || opt.mode == DOBFS_MODE_PUSH_SORT_KEYS)
    return fail(DOBFS_ERR_UNSUPPORTED, "the sort-based push needs a workspace beyond the static scratch");
  if (opt.flags & DOBFS_OPT_TIME_KERNELS)
    return fail(DOBFS_ERR_UNSUPPORTED, "kernel timing needs events, which this call does not create");
  const Layout L = plan(g->V, g->nnz);
  const size_t rep_off = align_up(L.total);
  if (rep_off + sizeof(HostReport) > kStaticScratchBytes)
    return fail(DOBFS_ERR_INVALID_ARG,
                "graph needs %zu bytes of scratch (V = %d, nnz = %lld); the static scratch holds %zu",
                rep_off + sizeof(HostReport), g->V, (long long)g->nnz, kStaticScratchBytes);
  DeviceScope ds(g->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice", __LINE__);
  uint8_t* base = nullptr;
  if ((st = static_scratch(g->device, &base)) != DOBFS_OK) return st;
  thread_local HostReport host_rep;  // ordinary host memory: the report is copied in after the stream drains
  thread_local LevelSlot host_tail;
  const ReportSink sink{reinterpret_cast<HostReport*>(base + rep_off), &host_rep};
  return bfs_steps(g, source, opt, depth, parent, base, L, static_cast<hipStream_t>(stream), sink,
                   nullptr, &host_tail, stats);
}

dobfs_status dobfs_bfs_batch_workspace_bytes(dobfs_graph g, int32_t k, size_t* bytes) {
  if (!g || !bytes) return fail(DOBFS_ERR_INVALID_ARG, "graph or bytes is NULL");
  if (k < 1 || k > kMaxSources) return fail(DOBFS_ERR_INVALID_ARG, "k = %d not in [1, 64]", k);
  *bytes = plan_batch(g->V, g->nnz, k).total;
  return DOBFS_OK;
}

dobfs_status dobfs_bfs_batch(dobfs_graph g, const int32_t* sources, int32_t k,
                             const dobfs_options* opt_in, int32_t* depth, void* workspace,
                             size_t ws_bytes, void* stream, dobfs_stats* stats) {
  t_last_error.clear();
  if (!g) return fail(DOBFS_ERR_INVALID_ARG, "graph is NULL");
  if (!depth) return fail(DOBFS_ERR_INVALID_ARG, "depth is NULL");
  if (k < 1 || k > kMaxSources) return fail(DOBFS_ERR_INVALID_ARG, "k = %d not in [1, 64]", k);
  DepthRows rows{};
  for (int32_t b = 0; b < k; ++b) rows.row[b] = depth + int64_t(b) * g->V;
  return bfs_batch_rows(g, sources, k, opt_in, rows, workspace, ws_bytes, stream, stats);
}

}  // extern "C"

// The multi-source traversal with each source's depth row at its own
// address (dobfs_bfs_batch lays them out contiguously; the server writes
// them straight into the callers' buffers).
dobfs_status dobfs::bfs_batch_rows(dobfs_graph g, const int32_t* sources, int32_t k, const dobfs_options* opt_in,
                            const DepthRows& rows, void* workspace, size_t ws_bytes, void* stream,
                            dobfs_stats* stats) {
  if (!sources) return fail(DOBFS_ERR_INVALID_ARG, "sources is NULL");
  if (k < 1 || k > kMaxSources) return fail(DOBFS_ERR_INVALID_ARG, "k = %d not in [1, 64]", k);
  for (int32_t b = 0; b < k; ++b)
    if (sources[b] < 0 || sources[b] >= g->V)
      return fail(DOBFS_ERR_INVALID_ARG, "sources[%d] = %d not in [0, %d)", b, sources[b], g->V);
  const dobfs_options opt = opt_in ? *opt_in : defaults();
  dobfs_status st = check_options(opt);
  if (st != DOBFS_OK) return st;
  if (opt.mode != DOBFS_MODE_FULL && opt.mode != DOBFS_MODE_PUSH_ONLY && opt.mode != DOBFS_MODE_PULL_ONLY)
    return fail(DOBFS_ERR_UNSUPPORTED, "multi-source BFS runs modes FULL, PUSH_ONLY and PULL_ONLY");
  if (stats && stats->cap > 0 && !stats->level)
    return fail(DOBFS_ERR_INVALID_ARG, "stats->level is NULL with cap = %d", stats->cap);

  DeviceScope ds(g->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice", __LINE__);
  const BatchLayout L = plan_batch(g->V, g->nnz, k);
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsLease lease;
  uint8_t* ws = nullptr;
  if ((st = get_workspace(g, workspace, ws_bytes, L.total, s, lease, &ws)) != DOBFS_OK) return st;
  const bool timing = (opt.flags & DOBFS_OPT_TIME_KERNELS) != 0;
  hipEvent_t* ev = events_for(g->device);
  if (!ev) return fail(DOBFS_ERR_DEVICE, "event creation failed");

  BatchArgs a{};
  a.V = g->V;
  a.nwords = g->nwords;
  a.nnz = g->nnz;
  a.rowptr = g->rowptr;
  a.colind = g->colind;
  a.colptr = g->colptr;
  a.rowind = g->rowind;
  a.nz_in = g->nz_in;
  a.slab = g->slab;
  a.lvl = reinterpret_cast<uint16_t*>(ws + L.lvl);
  a.k = k;
  a.active = k == 64 ? ~0ull : ((1ull << k) - 1ull);
  a.vis[0] = reinterpret_cast<uint64_t*>(ws + L.visA);
  a.vis[1] = reinterpret_cast<uint64_t*>(ws + L.visB);
  a.Fs = reinterpret_cast<uint64_t*>(ws + L.F);
  a.fstride = mb_fstride(g->V);
  a.nzF[0] = reinterpret_cast<uint32_t*>(ws + L.nzF0);
  a.nzF[1] = reinterpret_cast<uint32_t*>(ws + L.nzF1);
  a.Q[0] = reinterpret_cast<int32_t*>(ws + L.Q0);
  a.Q[1] = reinterpret_cast<int32_t*>(ws + L.Q1);
  a.S = reinterpret_cast<int32_t*>(ws + L.S);
  a.R = reinterpret_cast<int32_t*>(ws + L.R);
  a.chunk_first = reinterpret_cast<int32_t*>(ws + L.chunks);
  a.flagsA = reinterpret_cast<uint64_t*>(ws + L.flagsA);
  a.flagsB = reinterpret_cast<uint64_t*>(ws + L.flagsB);
  a.ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  a.mode = opt.mode;
  a.heuristic = opt.heuristic;
  a.alpha = double(opt.alpha);
  a.beta = double(opt.beta);
  a.edge_rule = opt.heuristic == DOBFS_HEUR_EDGES ? 1 : 0;
  a.nuniq = 0;
  for (int32_t b = 0; b < k; ++b) {
    a.src[b] = sources[b];
    bool seen = false;
    for (int32_t c = 0; c < a.nuniq; ++c) seen = seen || a.uniq[c] == sources[b];
    if (!seen) a.uniq[a.nuniq++] = sources[b];
  }
  const int32_t dir0 = opt.n_forced > 0 ? int32_t(opt.forced_dirs[0])
                                        : (opt.mode == DOBFS_MODE_PULL_ONLY ? DOBFS_DIR_PULL : DOBFS_DIR_PUSH);
  a.n_forced = std::min<int32_t>(opt.n_forced, kRing);  // later levels follow the rule
  if (a.n_forced > 0)
    HIPCK(hipMemcpyAsync(a.ctrl->forced, opt.forced_dirs, size_t(a.n_forced), hipMemcpyHostToDevice, s));
  // levels are kept as uint16 (level L stamps L + 1)
  const int64_t cap = std::min<int64_t>(int64_t(g->V) + 2, 0xfffe);
  // a level takes at most two steps; scan tile flags carry 2 * step + 2 in 30 bits
  const int64_t max_steps = std::min<int64_t>(2 * cap + 2, (int64_t(1) << 29) - 2);
  HostReport* rep = host_report();  // pinned: the device writes the reports into it
  if (!rep) return fail(DOBFS_ERR_OUT_OF_MEMORY, "pinned host buffer");
  const ReportSink sink{rep, rep};

  if (stats) HIPCK(hipEventRecord(ev[kEvStart], s));
  HIPCK(launch_mb_init(s, a, dir0, L.nflags, timing ? ev[kEvInit0] : nullptr,
                       timing ? ev[kEvInit1] : nullptr));
  LoopResult res;
  PersistentDevice* pd = nullptr;
  if (opt.flags & DOBFS_OPT_PERSISTENT) {
    pd = persistent_device(g->device);
    if (!pd) return fail(DOBFS_ERR_UNSUPPORTED, "the persistent level loop is not available on device %d", g->device);
  }
  st = run_steps(g->last_steps_mb, s, timing, ev, BatchSteps{a, rows}, a.ctrl, max_steps, cap,
                 cap < int64_t(g->V) + 2 ? DOBFS_ERR_UNSUPPORTED : DOBFS_ERR_INTERNAL, sink, pd, stats, &res);
  if (st != DOBFS_OK) return st;
  if (!stats) return DOBFS_OK;
  HIPCK(hipEventRecord(ev[kEvEnd], s));
  HIPCK(hipEventSynchronize(ev[kEvEnd]));
  {
    stats->levels = int32_t(res.levels);
    stats->ms_total = elapsed(ev[kEvStart], ev[kEvEnd]);
    stats->ms_init = timing ? elapsed(ev[kEvInit0], ev[kEvInit1]) : 0.f;
    stats->reached = k + res.sum_aux;  // (vertex, source) pairs, the sources included
    stats->launches_main = res.n_main;
    stats->launches_aux = res.n_aux;
    stats->ms_main_all = res.ms_main_all;
    stats->ms_aux_all = res.ms_aux_all;
    stats->edges_g500 = 0;
  }
  return DOBFS_OK;
}

dobfs_status dobfs::set_error(dobfs_status s, const char* what) { return fail(s, "%s", what); }

dobfs_status dobfs::check_batch_options(const dobfs_options& opt) {
  dobfs_status st = check_options(opt);
  if (st != DOBFS_OK) return st;
  if (opt.mode != DOBFS_MODE_FULL && opt.mode != DOBFS_MODE_PUSH_ONLY && opt.mode != DOBFS_MODE_PULL_ONLY)
    return fail(DOBFS_ERR_UNSUPPORTED, "multi-source BFS runs modes FULL, PUSH_ONLY and PULL_ONLY");
  return DOBFS_OK;
}

extern "C" {

dobfs_status dobfs_mxv(dobfs_graph g, const uint32_t* x_bits, const int32_t* x_idx,
                       int32_t x_nnz, const uint32_t* mask_bits, int32_t complement,
                       int32_t direction, uint32_t flags_in, uint32_t* y_bits, int32_t* y_idx,
                       int32_t* y_witness, int32_t* y_nnz, void* workspace, size_t ws_bytes,
                       void* stream) {
  t_last_error.clear();
  if (!g) return fail(DOBFS_ERR_INVALID_ARG, "graph is NULL");
  if (!y_bits) return fail(DOBFS_ERR_INVALID_ARG, "y_bits is NULL");
  if (direction != DOBFS_DIR_PUSH && direction != DOBFS_DIR_PULL)
    return fail(DOBFS_ERR_INVALID_ARG, "direction %d", direction);
  if (flags_in & ~uint32_t(DOBFS_MXV_EARLY_EXIT | DOBFS_MXV_ACCUM_OR))
    return fail(DOBFS_ERR_INVALID_ARG, "unknown mxv flags 0x%x", flags_in);
  if (!x_bits && (x_nnz < 0 || x_nnz > g->V || (x_nnz > 0 && !x_idx)))
    return fail(DOBFS_ERR_INVALID_ARG, "x: need x_bits, or x_idx with 0 <= x_nnz <= V");
  DeviceScope ds(g->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice", __LINE__);
  const Layout L = plan(g->V, g->nnz);
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsLease lease;
  uint8_t* ws = nullptr;
  dobfs_status st = get_workspace(g, workspace, ws_bytes, L.total, s, lease, &ws);
  if (st != DOBFS_OK) return st;
  const int32_t V = g->V, nwords = g->nwords;
  uint32_t* rbits = reinterpret_cast<uint32_t*>(ws + L.visA);
  uint32_t* xbits = reinterpret_cast<uint32_t*>(ws + L.FA);
  int32_t* list = reinterpret_cast<int32_t*>(ws + L.Q0);
  int32_t* S = reinterpret_cast<int32_t*>(ws + L.S);
  int32_t* R = reinterpret_cast<int32_t*>(ws + L.R);
  int32_t* chunks = reinterpret_cast<int32_t*>(ws + L.chunks);
  uint64_t* flagsA = reinterpret_cast<uint64_t*>(ws + L.flagsA);
  uint64_t* flagsB = reinterpret_cast<uint64_t*>(ws + L.flagsB);
  Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  const bool accum = (flags_in & DOBFS_MXV_ACCUM_OR) != 0;

  HIPCK(launch_ctrl_init(s, ctrl, flagsA, L.nflags));
  HIPCK(launch_fill(s, reinterpret_cast<uint32_t*>(flagsB), L.nflags * 2, 0u));
  LevelSlot* out_slot;
  if (direction == DOBFS_DIR_PULL) {
    const uint32_t* x = x_bits;
    if (!x) {
      HIPCK(launch_fill(s, xbits, nwords, 0u));
      if (x_nnz > 0) HIPCK(launch_s2d(s, x_idx, x_nnz, V, xbits));
      x = xbits;
    } else if (x_bits < y_bits + nwords && y_bits < x_bits + nwords) {
      // x overlaps y (the in-place form y = y OR A^T y .* not y): every tile writes its own
      // words of y whole while other tiles still read x at in-neighbour positions, so the
      // pull reads a copy of x made before it starts
      HIPCK(hipMemcpyAsync(xbits, x_bits, size_t(nwords) * 4, hipMemcpyDeviceToDevice, s));
      x = xbits;
    }
    PullArgs pa{};
    pa.V = V;
    pa.nwords = nwords;
    pa.colptr = g->colptr;
    pa.rowind = g->rowind;
    pa.slab = g->slab;
    pa.head = g->head;
    pa.x = x;
    pa.mask = mask_bits;
    pa.complement = complement ? 1 : 0;
    pa.mask_after = 0;
    pa.nz = g->nz_in;
    pa.out_base = accum ? y_bits : nullptr;
    pa.out = y_bits;
    pa.parent = y_witness;
    pa.early_exit = (flags_in & DOBFS_MXV_EARLY_EXIT) ? 1 : 0;
    pa.mid = kPullMid;
    pa.count_out = 1;
    pa.slot = &ctrl->slot[0];
    HIPCK(launch_pull(s, pa));
    out_slot = &ctrl->slot[0];
  } else {
    // The column-based matvec reads x as a sorted list of distinct indices
    // with its degree prefix: a dense x goes through DENSE2SPARSE fused with
    // the degree scan; a given list is made canonical the same way (scatter,
    // then compact), so repeated indices cannot inflate the expansion. The
    // list length and edge total stay on the device.
    const uint32_t* xd = x_bits;
    if (!xd) {
      HIPCK(launch_fill(s, xbits, nwords, 0u));
      if (x_nnz > 0) HIPCK(launch_s2d(s, x_idx, x_nnz, V, xbits));
      xd = xbits;
    }
    ScanBitsArgs sb{};
    sb.a = xd;
    sb.nwords = nwords;
    sb.V = V;
    sb.rowptr = g->rowptr;
    sb.Qout = list;
    sb.S = S;
    sb.R = R;
    sb.chunk_first = chunks;
    sb.flagsA = flagsA;
    sb.flagsB = flagsB;
    sb.epochA = 1;
    sb.epochB = 2;
    sb.ticket = &ctrl->ticket[0];
    sb.nf_out = &ctrl->nf32;
    sb.mf_out = &ctrl->mf32;
    HIPCK(launch_scan_bits(s, sb));
    HIPCK(launch_fill(s, rbits, nwords, 0u));
    ExpandArgs ea{};
    ea.Q = list;
    ea.S = S;
    ea.R = R;
    ea.chunk_first = chunks;
    ea.colind = g->colind;
    ea.claim = rbits;
    ea.mask = mask_bits;
    ea.complement = complement ? 1 : 0;
    ea.parent = y_witness;
    ea.slot = &ctrl->slot[0];
    HIPCK(launch_expand(s, ea, &ctrl->mf32, &ctrl->nf32));
    HIPCK(launch_mxv_finalize(s, y_bits, rbits, nwords, V, accum ? 1 : 0, &ctrl->slot[1]));
    out_slot = &ctrl->slot[1];
  }
  if (y_idx) {
    ScanBitsArgs sb{};
    sb.a = y_bits;
    sb.nwords = nwords;
    sb.V = V;
    sb.Qout = y_idx;
    sb.flagsA = flagsA;
    sb.flagsB = flagsB;
    sb.epochA = 3;
    sb.epochB = 4;
    sb.ticket = &ctrl->ticket[1];
    sb.nf_out = &ctrl->nf32;
    HIPCK(launch_scan_bits(s, sb));
  }
  if (y_nnz || y_idx) {
    Ctrl* host = host_ctrl();
    if (!host) return fail(DOBFS_ERR_OUT_OF_MEMORY, "pinned host buffer");
    HIPCK(hipMemcpyAsync(host, ctrl, offsetof(Ctrl, ring), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    if (y_nnz) *y_nnz = int32_t(sum_slot(host->slot[out_slot - ctrl->slot]).aux);
  } else {
    HIPCK(hipGetLastError());
  }
  return DOBFS_OK;
}

}  // extern "C"
