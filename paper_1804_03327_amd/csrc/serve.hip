// Query server of libdobfs (declared in include/dobfs.h): single-source BFS
// queries are answered by multi-source traversals that run several at a time.
//
// Each slot is a host thread with its own HIP stream. A free slot takes the
// graph whose oldest queued query has waited longest, takes up to max_batch
// queued queries of that graph in arrival order, waits until the batch's
// workspace can be carved out of the server's memory pool (one device
// allocation of mem_budget bytes: admission by memory), and runs them as one
// multi-source traversal whose depth rows are written straight into the
// callers' buffers. A batch of one runs the single-source traversal instead
// (depths only): a smaller workspace, and on deep graphs fewer launches.
// Queries that arrive while a batch is on the GPU go to the next free slot,
// so their traversal overlaps the running one on the device. Graphs whose
// batches have been taking long (a running mean of their service times above
// kLongMs) may hold at most slots - 1 slots at once, so one slot stays free for
// the others' queries instead of queueing them behind deep traversals; and
// their queries are batched only once kLongBatchMin of them are queued, fewer
// going one per slot: on a deep graph a multi-source traversal of a few
// sources takes longer than the same single-source traversals side by side.

#include "dobfs.h"
#include "dobfs_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace dobfs;

namespace {

constexpr int kMaxSlots = 16;
constexpr double kLongMs = 2.0;  // a graph whose batches take longer than this on average is "long"
// Fewest queued queries of a long graph that one multi-source traversal takes (2048x2048 grid:
// 2 / 4 / 8 sources take 84 / 100 / 99 ms together, two single-source traversals on two
// streams 41 ms, one alone 32 ms).
constexpr int32_t kLongBatchMin = 8;

// First-fit allocator over one device allocation, in 256-byte units.
struct Pool {
  uint8_t* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_at;  // offset -> length of every free range, coalesced

  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
  void reset(uint8_t* p, size_t n) {
    base = p;
    size = n;
    free_at.clear();
    if (n) free_at[0] = n;
  }
  bool can_take(size_t need) const {
    need = round(need);
    for (const auto& f : free_at)
      if (f.second >= need) return true;
    return false;
  }
  size_t take(size_t need) {  // SIZE_MAX when no free range is large enough
    need = round(need);
    for (auto it = free_at.begin(); it != free_at.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, len = it->second;
      free_at.erase(it);
      if (len > need) free_at[off + need] = len - need;
      return off;
    }
    return SIZE_MAX;
  }
  void give(size_t off, size_t need) {
    need = round(need);
    auto next = free_at.lower_bound(off);
    if (next != free_at.end() && off + need == next->first) {  // merge with the range after
      need += next->second;
      next = free_at.erase(next);
    }
    if (next != free_at.begin()) {  // merge with the range before
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += need;
        return;
      }
    }
    free_at[off] = need;
  }
};

struct Query {
  int32_t graph = 0, source = 0;
  int32_t* depth = nullptr;
  int32_t batch_size = 0;
  int32_t status = DOBFS_OK;
  bool done = false;
  double t_submit = 0, t_start = 0, t_done = 0;
};

struct GraphInfo {
  int32_t V = 0;
  int64_t nnz = 0;
  double mean_ms = 0.0;  // running mean of this graph's batch service times (0: none yet)
  int32_t running = 0;   // slots running a batch of this graph
};

}  // namespace

struct dobfs_server_s {
  dobfs_server_options opt{};
  std::vector<dobfs_graph> graphs;
  std::vector<GraphInfo> info;
  int device = 0;
  size_t budget = 0;
  Pool pool;                       // batches' workspaces are carved out of one allocation
  int32_t long_running = 0;        // slots running a batch of a long graph
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_mem, cv_done;
  std::deque<Query> queries;       // every query, indexed by id
  std::deque<uint64_t> pending;    // ids not yet taken, in arrival order
  bool stop = false;

  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  void* pool_mem = nullptr;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

size_t batch_bytes(dobfs_graph g, int32_t k) {
  size_t b = 0;
  if (dobfs_bfs_batch_workspace_bytes(g, k, &b) != DOBFS_OK) return SIZE_MAX;
  return b;
}

// Workspace of a batch of k queries: the single-source call's for k = 1.
size_t run_bytes(dobfs_graph g, const dobfs_options& opt, int32_t k) {
  size_t b = 0;
  if (k == 1) return dobfs_bfs_workspace_bytes(g, &opt, &b) == DOBFS_OK ? b : SIZE_MAX;
  return batch_bytes(g, k);
}

bool is_long(const GraphInfo& g) { return g.mean_ms > kLongMs; }

// The graph a free slot serves next: that of the oldest queued query, skipping
// long graphs while slots - 1 slots already run long batches; -1 if none may go.
int32_t pick_graph(dobfs_server s) {
  const bool long_full = s->opt.slots > 1 && s->long_running >= s->opt.slots - 1;
  for (uint64_t id : s->pending) {
    const int32_t gi = s->queries[id].graph;
    if (!long_full || !is_long(s->info[size_t(gi)])) return gi;
  }
  return -1;
}

void worker(dobfs_server s, int slot) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    int32_t gi = -1;
    s->cv_work.wait(lk, [&] {
      if (s->stop && s->pending.empty()) return true;
      gi = pick_graph(s);
      return gi >= 0;
    });
    if (gi < 0) break;  // stopping and nothing left
    // up to max_batch of the graph's queries, in arrival order
    std::vector<uint64_t> take;
    for (auto it = s->pending.begin(); it != s->pending.end() && int32_t(take.size()) < s->opt.max_batch;) {
      if (s->queries[*it].graph == gi) {
        take.push_back(*it);
        it = s->pending.erase(it);
      } else {
        ++it;
      }
    }
    int32_t k = int32_t(take.size());
    if (k < kLongBatchMin && is_long(s->info[size_t(gi)])) k = 1;  // the rest go to other slots
    // admission by memory: the batch's workspace must fit in the pool
    while (k > 1 && run_bytes(s->graphs[gi], s->opt.opt, k) > s->budget) --k;
    if (take.size() > size_t(k)) {  // the rest back to the head, in order, for the other slots
      for (size_t q = take.size(); q > size_t(k); --q) s->pending.push_front(take[q - 1]);
      s->cv_work.notify_all();
    }
    take.resize(size_t(k));
    const size_t need = run_bytes(s->graphs[gi], s->opt.opt, k);
    if (need > s->budget) {  // not even one source fits
      const double t = s->now_ms();
      for (uint64_t id : take) {
        Query& q = s->queries[id];
        q.status = DOBFS_ERR_OUT_OF_MEMORY;
        q.batch_size = k;
        q.t_start = q.t_done = t;
        q.done = true;
      }
      s->cv_done.notify_all();
      continue;
    }
    GraphInfo& info = s->info[size_t(gi)];
    const bool lng = is_long(info);
    ++info.running;
    if (lng) ++s->long_running;
    s->cv_mem.wait(lk, [&] { return s->pool.can_take(need); });
    const size_t off = s->pool.take(need);
    std::vector<int32_t> src(static_cast<size_t>(k));
    DepthRows rows{};
    const double t_start = s->now_ms();
    for (int32_t b = 0; b < k; ++b) {
      Query& q = s->queries[take[size_t(b)]];
      src[size_t(b)] = q.source;
      rows.row[b] = q.depth;
      q.t_start = t_start;
    }
    lk.unlock();
    void* ws = s->pool.base + off;
    // both calls return once the depth rows are final
    const dobfs_status st =
        k == 1 ? dobfs_bfs(s->graphs[gi], src[0], &s->opt.opt, rows.row[0], nullptr, ws, need,
                           s->streams[size_t(slot)], nullptr)
               : bfs_batch_rows(s->graphs[gi], src.data(), k, &s->opt.opt, rows, ws, need,
                                s->streams[size_t(slot)], nullptr);
    // a later batch may reuse this memory from another stream: the traversal's last kernels
    // may still read their control block after the results are final
    (void)hipStreamSynchronize(s->streams[size_t(slot)]);
    lk.lock();
    s->pool.give(off, need);
    const double t_done = s->now_ms();
    info.mean_ms = info.mean_ms == 0.0 ? (t_done - t_start) : 0.75 * info.mean_ms + 0.25 * (t_done - t_start);
    --info.running;
    if (lng) --s->long_running;
    for (uint64_t id : take) {
      Query& q = s->queries[id];
      q.status = st;
      q.batch_size = k;
      q.t_done = t_done;
      q.done = true;
    }
    s->cv_mem.notify_all();
    s->cv_done.notify_all();
    s->cv_work.notify_all();  // a long slot freed, or queries left
  }
}

void release(dobfs_server s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  (void)hipSetDevice(s->device);
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->pool_mem) (void)hipFree(s->pool_mem);
  delete s;
}

}  // namespace

extern "C" {

dobfs_status dobfs_server_options_default(dobfs_server_options* o) {
  if (!o) return set_error(DOBFS_ERR_INVALID_ARG, "options pointer is NULL");
  *o = dobfs_server_options{};
  o->slots = 4;
  o->max_batch = 64;
  o->mem_budget = 0;
  return dobfs_options_default(&o->opt);
}

dobfs_status dobfs_server_create(const dobfs_graph* graphs, int32_t n_graphs, const dobfs_server_options* opt,
                                 dobfs_server* out) {
  if (!out) return set_error(DOBFS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!graphs || n_graphs < 1) return set_error(DOBFS_ERR_INVALID_ARG, "need at least one graph");
  dobfs_server_options o;
  if (opt) {
    o = *opt;
  } else {
    dobfs_server_options_default(&o);
  }
  if (o.slots < 1 || o.slots > kMaxSlots) return set_error(DOBFS_ERR_INVALID_ARG, "slots must be in [1, 16]");
  if (o.max_batch < 1 || o.max_batch > kMaxSources)
    return set_error(DOBFS_ERR_INVALID_ARG, "max_batch must be in [1, 64]");
  dobfs_status st = check_batch_options(o.opt);
  if (st != DOBFS_OK) return st;
  if (o.opt.n_forced > 0) return set_error(DOBFS_ERR_UNSUPPORTED, "forced directions are per traversal, not per server");

  auto s = new dobfs_server_s();
  s->opt = o;
  s->t0 = std::chrono::steady_clock::now();
  size_t largest = 0;
  for (int32_t i = 0; i < n_graphs; ++i) {
    GraphInfo gi;
    int32_t dev = -1;
    if (!graphs[i] || dobfs_graph_info(graphs[i], &gi.V, &gi.nnz, &dev) != DOBFS_OK) {
      delete s;
      return set_error(DOBFS_ERR_INVALID_ARG, "a graph handle is NULL or invalid");
    }
    if (i == 0) s->device = dev;
    if (dev != s->device) {
      delete s;
      return set_error(DOBFS_ERR_INVALID_ARG, "all graphs of a server must be on one device");
    }
    s->graphs.push_back(graphs[i]);
    s->info.push_back(gi);
    largest = std::max(largest, std::max(run_bytes(graphs[i], o.opt, 1), run_bytes(graphs[i], o.opt, o.max_batch)));
  }
  s->budget = o.mem_budget ? o.mem_budget : Pool::round(largest) * size_t(o.slots);
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(s->device) != hipSuccess) {
    delete s;
    return set_error(DOBFS_ERR_DEVICE, "hipSetDevice failed");
  }
  for (int k = 0; k < o.slots; ++k) {
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
      release(s);
      if (prev >= 0) (void)hipSetDevice(prev);
      return set_error(DOBFS_ERR_DEVICE, "hipStreamCreateWithFlags failed");
    }
    s->streams.push_back(stream);
  }
  if (hipMalloc(&s->pool_mem, s->budget) != hipSuccess) {
    s->pool_mem = nullptr;
    release(s);
    if (prev >= 0) (void)hipSetDevice(prev);
    return set_error(DOBFS_ERR_OUT_OF_MEMORY, "server memory pool allocation failed");
  }
  s->pool.reset(static_cast<uint8_t*>(s->pool_mem), s->budget);
  if (prev >= 0) (void)hipSetDevice(prev);
  for (int k = 0; k < o.slots; ++k) s->workers.emplace_back(worker, s, k);
  *out = s;
  return DOBFS_OK;
}

dobfs_status dobfs_server_submit(dobfs_server s, int32_t graph, int32_t source, int32_t* depth, uint64_t* id) {
  if (!s || !id || !depth) return set_error(DOBFS_ERR_INVALID_ARG, "server, depth or id is NULL");
  if (graph < 0 || graph >= int32_t(s->graphs.size()))
    return set_error(DOBFS_ERR_INVALID_ARG, "graph index out of range");
  if (source < 0 || source >= s->info[size_t(graph)].V)
    return set_error(DOBFS_ERR_INVALID_ARG, "source out of range");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return set_error(DOBFS_ERR_INVALID_ARG, "server is shutting down");
    Query q;
    q.graph = graph;
    q.source = source;
    q.depth = depth;
    q.t_submit = s->now_ms();
    *id = uint64_t(s->queries.size());
    s->queries.push_back(q);
    s->pending.push_back(*id);
  }
  s->cv_work.notify_one();
  return DOBFS_OK;
}

dobfs_status dobfs_server_wait(dobfs_server s, uint64_t id, int32_t timeout_ms, dobfs_query_info* info) {
  if (!s) return set_error(DOBFS_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  if (id >= s->queries.size()) return set_error(DOBFS_ERR_INVALID_ARG, "unknown query id");
  auto ready = [&] { return s->queries[id].done; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return set_error(DOBFS_ERR_TIMEOUT, "query not done yet");
  }
  const Query& q = s->queries[id];
  if (info) {
    info->graph = q.graph;
    info->source = q.source;
    info->batch_size = q.batch_size;
    info->status = q.status;
    info->t_submit_ms = q.t_submit;
    info->t_start_ms = q.t_start;
    info->t_done_ms = q.t_done;
  }
  if (q.status != DOBFS_OK) return set_error(dobfs_status(q.status), "the query's traversal failed");
  return DOBFS_OK;
}

dobfs_status dobfs_server_destroy(dobfs_server s) {
  if (!s) return set_error(DOBFS_ERR_INVALID_ARG, "server is NULL");
  release(s);
  return DOBFS_OK;
}

}  // extern "C"
