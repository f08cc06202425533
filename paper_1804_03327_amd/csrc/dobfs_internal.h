// Internal declarations shared by the HIP kernels and the host runtime of
// libdobfs. Not part of the public ABI (see include/dobfs.h).
#pragma once

#include <hip/hip_runtime.h>

#include "dobfs.h"

#include <cstddef>
#include <cstdint>

namespace dobfs {

// ---- per-level counters ----
// Same-address device atomics serialize (about 11 ns each on MI355X), so
// every block adds its partial sums into one of kStripes counters, each on
// its own 128-byte line; readers add the stripes up.
constexpr int kStripes = 32;
struct alignas(128) Stripe {
  uint32_t count;  // vertices discovered (BFS) / result bits (mxv)
  uint32_t aux;    // mxv: popcount of the whole output vector; multi-source: (vertex, source) pairs
  uint64_t edges;  // adjacency entries read (push) or in-neighbours checked (pull)
  uint64_t mnew;   // out-edges of the vertices discovered (edge-count rule only)
  uint64_t insub;  // in-edges of the vertices discovered (edge-count rule only; multi-source:
                   // of the vertices every source has now reached)
  uint64_t fbits;  // multi-source: OR of the source bits discovered
  uint64_t mu;     // edge-count rule, single source: in-edges of the vertices still unvisited
                   // entering a push that follows a pull, recounted by that level's scan
  uint32_t maxdeg; // largest out-degree of the vertices a push level discovered
  uint32_t tilemax; // pull levels: most rows found in one tile, or UINT32_MAX when a found row
                    // has an out-degree above kLocalDeg
};
struct LevelSlot {
  Stripe s[kStripes];
};
constexpr int kSlots = 4;  // level L accumulates into slot L % kSlots

// Traversal state entering a level, written by that level's first kernel.
struct alignas(64) LevelState {
  int32_t dir;         // DOBFS_DIR_* of this level
  int32_t done;        // 1: a previous level discovered nothing; nothing left to do
  int32_t list_valid;  // 1: the frontier is already a list (the previous level pushed)
  int32_t vis_idx;     // which of the two visited bitmaps is current
  int32_t nf;          // frontier size entering the level
  int32_t levels;      // when done: number of levels run
  int32_t level;       // index of this level
  int32_t local;       // push level expanded with block-local load balancing, no global scan:
                       // 1 over the frontier list, 2 over the bits the previous pull found;
                       // multi-source pull: 1 when it merges the winners of the push before
  int32_t share;       // local 1: blocks that share one unit's edge chunks (local_share)
  int32_t phase;       // step loops: kPhaseWhole, kPhaseScan or kPhaseExpand
  int64_t m_u;         // edge-count rule: in-edges of still-unvisited vertices
  uint64_t active;     // multi-source: sources whose frontier entering the level is non-empty
  uint64_t t0;         // single source, persistent loop: device clock when the step started
};
static_assert(sizeof(LevelState) == 64, "one state per 64-byte line");
// What one step of a step loop does for its level: all of it
// (a pull, or a push that shares out its own work), or one of the two steps of
// a push that needs the global degree scan.
constexpr int32_t kPhaseWhole = 0, kPhaseScan = 1, kPhaseExpand = 2;
// Per-level statistics for the host, written by the next level's first kernel.
struct LevelRecord {
  int32_t dir, nf, n_new, variant;  // variant: dobfs_level_stats.variant
  int64_t edges, m_f;
  uint64_t mnew, insub;
  uint64_t aux;        // multi-source: (vertex, source) pairs discovered
};
constexpr int kRing = 1024;  // levels of state / records kept on the device

// Grid barrier of the persistent step loop. Blocks arrive on one of
// kBarGroups counters (each on its own line, so arrivals on different
// counters do not serialise), the last arrival of a group on `top`, and the
// last group's arrival publishes the next generation, which every block
// waits for. Counters only grow during a traversal (the init kernel zeroes
// them): a group's last arrival is the one that makes its count a multiple
// of the group's size. `abort` is raised by a block whose wait exceeded the
// spin limit; every waiting block then leaves.
constexpr int kBarGroups = 16;
struct alignas(128) BarCounter {
  unsigned long long n;
};
struct GridBar {
  BarCounter group[kBarGroups];
  BarCounter top;
  alignas(128) uint32_t gen;
  alignas(128) uint32_t abort;
  alignas(128) unsigned long long t_end;  // timing: latest block end of the last launch (device clock)
};

struct Ctrl {
  unsigned long long ticket[2];  // scan tile tickets, one counter per level (or step) parity
  uint32_t mf32;                 // m_f of the latest frontier scan (expand reads it)
  uint32_t nf32;                 // frontier length of the latest bitmap scan
  int64_t src_outdeg;            // out-degree of the BFS source
  int64_t src_indeg;             // in-degree of the BFS source
  uint32_t qcount[kSlots];       // frontier-list append counter of each level
  uint32_t mf[kSlots];           // push: out-edges of the level's input frontier
  uint8_t pad[128 - 56 - 4 * kSlots];
  LevelSlot slot[kSlots];
  LevelState ring[kRing];
  LevelRecord rec[kRing];
  int8_t forced[kRing];          // step loops: forced direction of levels 0 .. n_forced-1
  LevelSlot tail;                // after a traversal: out-degree sum of the reached vertices (edges)
  GridBar bar;                   // the persistent loops' grid barrier
};
static_assert(sizeof(Stripe) == 128, "stripe layout");
static_assert(offsetof(Ctrl, slot) % 128 == 0, "slots start on a line");

// Host-side totals of one level.
struct LevelTotals {
  uint64_t count, aux, edges, mnew, insub, mu;
};
inline LevelTotals sum_slot(const LevelSlot& s) {
  LevelTotals t{0, 0, 0, 0, 0, 0};
  for (int k = 0; k < kStripes; ++k) {
    t.count += s.s[k].count;
    t.aux += s.s[k].aux;
    t.edges += s.s[k].edges;
    t.mnew += s.s[k].mnew;
    t.insub += s.s[k].insub;
    t.mu += s.s[k].mu;
  }
  return t;
}

// ---- launch geometry (all kernels use 256-thread blocks = 4 wave64) ----
constexpr int kThreads = 256;
constexpr int kScanIPT = 8;                          // list scan: frontier entries per thread
constexpr int kScanTile = kThreads * kScanIPT;      // 2048 entries per tile
constexpr int kBitsWPT = 4;                          // bitmap scan: words per thread
constexpr int kBitsTile = kThreads * kBitsWPT;      // 1024 words (32768 vertices) per tile
constexpr int kScanBlocksMax = 256;                  // scan grids stride over tiles by ticket
constexpr int kExpandEPT = 4;                        // expand: edges per thread per chunk
constexpr int kExpandChunk = kThreads * kExpandEPT; // 1024 edges per chunk
constexpr int kExpandWin = kExpandChunk + 1;         // frontier entries cached in LDS per chunk
constexpr int kExpandBuf = 2048;                     // winners buffered in LDS before a list flush
constexpr int kExpandBlocks = 1024;                  // expand grid (strides over chunks)
constexpr int kPullTileWords = 128;                  // pull: bitmap words owned by a block (measured
                                                     // best of 8..256 on RMAT-22: fewer, fuller blocks)
constexpr int kPullTileV = kPullTileWords * 32;      // 4096 rows per block
constexpr int kSlab = 4;                             // in-neighbours per row kept in the dense slab
constexpr int kPullFirst = kSlab;                    // pull phase 1 checks a row's slab entries
constexpr int kPullMid = 32;                         // rows still open continue thread-per-row up to here
constexpr int kPullStep = 4;                         // in-neighbours a thread loads at once past kPullFirst
constexpr int kPullBatch = 4;                        // open rows a thread works on at once (slab)
constexpr int kPullHeadBatch = 8;                    // candidate rows a thread works on at once (head)
constexpr int kLocalDeg = 32;                        // graphs with no out-degree above this always push locally
constexpr int kLocalUnit = 128;                      // local push: frontier vertices a block takes at once
constexpr int kLocalChunks = 4;                      // local push: most edge chunks one block may get
constexpr int kBitmapLocalRows = 512;                // bitmap push: most frontier rows in one pull tile

inline int32_t words_of(int64_t V) { return int32_t((V + 31) / 32); }
inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }
inline int64_t bits_tiles(int64_t nwords) { return (nwords + kBitsTile - 1) / kBitsTile; }
__host__ __device__ inline int64_t pull_tiles(int64_t nwords) {
  return (nwords + kPullTileWords - 1) / kPullTileWords;
}
// Blocks of a level's second kernel: the pull's tiles, at least the push's expand grid.
__host__ __device__ inline int64_t main_blocks(int64_t nwords) {
  const int64_t t = pull_tiles(nwords);
  return t > kExpandBlocks ? t : kExpandBlocks;
}
// Schedule settings of the single-source kernels a caller may tune (the tuning fields of
// dobfs_options; 0 there selects the defaults above).
struct Sched {
  int32_t pull_mid;      // pull: in-neighbours a thread scans before a wave takes the row (kPullMid)
  int32_t bitmap_rows;   // bitmap push: most rows one pull tile may have found (kBitmapLocalRows)
  int32_t local_unit;    // local push: frontier vertices a block takes at once, 1..kThreads (kLocalUnit)
  int32_t local_chunks;  // local push: most edge chunks of a unit one block may get (kLocalChunks)
};
inline Sched default_sched() { return Sched{kPullMid, kBitmapLocalRows, kLocalUnit, kLocalChunks}; }

// Whether a push over a frontier list of nf vertices with m_f out-edges in all, none above
// maxdeg, can balance its load inside blocks (no global degree scan): the list is cut into
// units of `unit` vertices, a unit holds at most min(m_f, unit * maxdeg) edges, and
// when there are fewer units than blocks each unit's edge chunks are shared by
// blocks / units blocks. Local when no block gets more than `chunks` chunks of a unit.
// (Every thread of a level's first kernel evaluates this: 32-bit arithmetic, two divisions.)
__host__ __device__ inline uint32_t local_unit_chunks_bound(int64_t m_f, int64_t maxdeg, int32_t unit) {
  const int64_t cap = int64_t(unit) * maxdeg;
  const int64_t edges = m_f < cap ? m_f : cap;
  const int64_t chunks = (edges + kExpandChunk - 1) >> 10;  // kExpandChunk = 1024
  return chunks > 0xffffffffll ? 0xffffffffu : uint32_t(chunks);
}
__host__ __device__ inline uint32_t local_units(int64_t nf, int32_t unit) {
  return uint32_t((uint64_t(nf) + uint32_t(unit) - 1) / uint32_t(unit));
}
__host__ __device__ inline bool local_fits(int64_t nf, int64_t m_f, int64_t maxdeg, int64_t blocks, int32_t unit,
                                           int32_t max_chunks) {
  static_assert(kExpandChunk == 1024, "shift below");
  const uint32_t units = local_units(nf, unit);
  if (units == 0) return true;
  const uint32_t per_unit = units < uint32_t(blocks) ? uint32_t(blocks) / units : 1u;
  return uint64_t(local_unit_chunks_bound(m_f, maxdeg, unit)) <= uint64_t(max_chunks) * per_unit;
}
// Blocks that share each unit's chunks in a local push: as many as the unit's
// chunks could need, at most blocks / units (so idle blocks exit at once).
__host__ __device__ inline int32_t local_share(int64_t nf, int64_t m_f, int64_t maxdeg, int64_t blocks, int32_t unit) {
  const uint32_t units = local_units(nf, unit);
  if (units == 0 || units >= uint32_t(blocks)) return 1;
  const uint32_t chunks = local_unit_chunks_bound(m_f, maxdeg, unit);
  const uint32_t most = uint32_t(blocks) / units;
  return int32_t(chunks < 1u ? 1u : (chunks < most ? chunks : most));
}
inline int64_t max_chunks(int64_t nnz) { return nnz / kExpandChunk + 2; }
inline int64_t flag_entries(int64_t V) {
  const int64_t a = scan_tiles(V), b = bits_tiles(words_of(V));
  return (a > b ? a : b) + 1;
}
inline int32_t scan_grid(int64_t V) {
  const int64_t t = flag_entries(V);
  return int32_t(t < kScanBlocksMax ? t : kScanBlocksMax);
}

// ---- argument blocks ----
struct PullArgs {
  int32_t V, nwords;
  const int32_t* colptr;
  const int32_t* rowind;
  const int4* slab;          // first kSlab entries of every CSC column (-1 past its end)
  const int32_t* head;       // first entry of every CSC column: j, or ~j when more follow
  const uint32_t* x;         // input vector bits
  const uint32_t* mask;      // nullable: rows that pass = mask XOR complement
  int32_t complement;
  int32_t mask_after;        // 1: compute every row, apply the mask to the result
  const uint32_t* nz;        // rows with in-degree > 0
  const uint32_t* out_base;  // nullable: OR-ed into out (visited snapshot / old y)
  uint32_t* out;             // every word of the block's tile is written
  uint32_t* found_out;       // nullable: result bits alone
  int32_t* depth;            // nullable
  int32_t* parent;           // nullable: parent (BFS) or witness (mxv)
  int32_t level;
  int32_t early_exit;
  int32_t mid;               // in-neighbours a thread scans before a wave takes the row
  int32_t count_out;         // 1: add popcount(out) to the stripes' aux (mxv)
  const uint32_t* heavy;     // nullable: rows of out-degree above kLocalDeg (tilemax bookkeeping)
  LevelSlot* slot;
};

struct ExpandArgs {
  const int32_t* Q;          // frontier list
  int32_t nf;
  const int32_t* S;          // exclusive scan of out-degrees
  const int32_t* R;          // row start of each frontier vertex
  const int32_t* chunk_first;  // first frontier entry of every edge chunk
  const int32_t* colind;
  uint32_t m;                // total edges of the expansion
  uint32_t* claim;           // bitmap claimed with atomicOr (visited / result)
  const uint32_t* mask;      // nullable: filter before the claim
  int32_t complement;
  int32_t* depth;            // nullable
  int32_t* parent;           // nullable: parent / witness
  int32_t level;
  int32_t* Qout;             // nullable: winners appended here
  uint32_t* qcount;          // append counter for Qout
  uint32_t* found_out;       // nullable: winners' bits also set here
  const int32_t* rowptr;     // CSR(A) offsets (local push: degrees of the frontier)
  const int32_t* out_rowptr; // nullable: out-degrees of winners -> mnew
  const int32_t* in_colptr;  // nullable: in-degrees of winners -> insub
  // bitmap push (a frontier the previous pull left as bits): the frontier bits, the visited
  // set before that pull, rows with in-edges, and where the recount of m_u goes (nullable)
  int32_t share;             // local list push: blocks per unit (LevelState::share)
  int32_t unit;              // local push: frontier vertices a block takes at once
  const uint32_t* front;
  const uint32_t* vis_before;
  const uint32_t* nz;
  LevelSlot* mu_slot;
  LevelSlot* slot;
};

// Everything a BFS level kernel needs; the per-level choices come from the
// LevelState the level's first kernel writes.
struct BfsArgs {
  int32_t V, nwords;
  int64_t nnz;
  const int32_t* rowptr;
  const int32_t* colind;
  const int32_t* colptr;
  const int32_t* rowind;
  const int4* slab;          // first kSlab entries of every CSC column (-1 past its end)
  const int32_t* head;       // first entry of every CSC column: j, or ~j when more follow
  const uint32_t* nz_in;
  const uint32_t* heavy;     // vertices of out-degree above kLocalDeg
  int32_t* depth;
  int32_t* parent;
  uint32_t* vis[2];
  uint32_t* F[2];            // frontier bitmaps (modes without operand reuse)
  int32_t* Q[2];             // frontier lists, level L reads Q[L % 2]
  int32_t* S;
  int32_t* R;
  int32_t* chunk_first;
  uint64_t* flagsA;
  uint64_t* flagsB;
  Ctrl* ctrl;
  int32_t mode;
  int32_t heuristic;
  double alpha, beta;
  int32_t reuse;             // pull reads the visited set (operand reuse)
  int32_t early_exit;
  int32_t mask_after;        // unmasked pull
  int32_t need_F;            // frontier bitmaps maintained
  int32_t edge_rule;
  int32_t local_push;        // push levels of small out-degree may skip the global scan
  int32_t low_degree;        // every out-degree of the graph is <= kLocalDeg
  int32_t n_forced;          // levels whose direction Ctrl::forced fixes
  Sched sched;
};

// ---- multi-source BFS: up to 64 sources, one bit of a uint64 per source ----
constexpr int kMaxSources = 64;
struct BatchArgs {
  int32_t V, nwords;
  int64_t nnz;
  const int32_t* rowptr;
  const int32_t* colind;
  const int32_t* colptr;
  const int32_t* rowind;
  const uint32_t* nz_in;
  const int4* slab;          // first kSlab entries of every CSC column (-1 past its end)
  uint16_t* lvl;             // [V][k]: level at which source b reached v, for levels >= kMbSnap only
  int32_t k;                 // sources
  int32_t nuniq;             // distinct sources
  uint64_t active;           // the k source bits
  uint64_t* vis[2];          // per vertex: sources that reached it
  uint64_t* Fs;              // kMbSnap + 2 buffers of fstride words; level L's frontier in mb_frontier(a, L)
  int64_t fstride;           // V rounded up to a multiple of 32 (every buffer 256-byte aligned)
  uint32_t* nzF[2];          // one bit per vertex: its frontier word is nonzero; level L reads nzF[L % 2]
                             // (written by a pull, or by a push that marks instead of listing)
  int32_t* Q[2];
  int32_t* S;
  int32_t* R;
  int32_t* chunk_first;
  uint64_t* flagsA;
  uint64_t* flagsB;
  Ctrl* ctrl;
  int32_t mode;
  int32_t heuristic;
  double alpha, beta;
  int32_t edge_rule;
  int32_t local_push;        // always 0: the multi-source push always scans
  int32_t n_forced;          // levels whose direction Ctrl::forced fixes
  int32_t low_degree;        // unused here
  Sched sched;               // unused here (no local push)
  int32_t src[kMaxSources];  // source of bit b
  int32_t uniq[kMaxSources]; // the distinct sources: the first frontier list
};
// Multi-source frontier words: per vertex, the sources whose frontier holds it.
// The frontier of level L is exactly the set of (vertex, source) pairs first
// reached at level L, so the frontiers of levels below kMbSnap are kept, one
// buffer each, and stand in for those levels' depths; later levels alternate
// between two more buffers and record their depths in the level table.
constexpr int kMbSnap = 16;
__host__ __device__ inline int32_t mb_frontier_slot(int32_t L) { return L < kMbSnap ? L : kMbSnap + (L & 1); }
__host__ __device__ inline int64_t mb_fstride(int64_t V) { return (V + 31) / 32 * 32; }
// whether level L's frontier buffer held the frontier of level L - 2 in this traversal
__host__ __device__ inline bool mb_frontier_recycled(int32_t L) { return L >= kMbSnap + 2; }
// A multi-source push over more edges than this marks its winners in the
// next frontier's non-zero bitmap (non-returning atomics) instead of listing
// them: every block reserving list space with one returning atomic on a single
// counter serialises a wide push. The next level lists the bitmap only if it
// pushes too.
constexpr uint32_t kMbMarkEdges = 64u * kExpandChunk;
__host__ __device__ inline bool mb_push_marks(uint32_t m) { return m > kMbMarkEdges; }
constexpr int kMbDenseMerge = 16;  // a push's winners merge into Vis densely once they are V/16 or more
constexpr int kMbTileWords = 8;                 // multi-source pull: bitmap words of rows per block
constexpr int kMbTileV = kMbTileWords * 32;     // 256 rows, one per thread: a tile's rows all run at once
constexpr int kMbMid = 32;                      // multi-source pull: in-neighbours a thread scans before a wave takes over
constexpr int kMbLong = kMbTileV;               // multi-source pull: rows a tile can hand to its waves

struct ScanBitsArgs {
  const uint32_t* a;         // bits = a AND NOT b_not
  const uint32_t* b_not;     // nullable
  int32_t nwords, V;
  const int32_t* rowptr;     // nullable: no degrees / S / R / chunk table
  int32_t* Qout;             // the set bits as an ascending list
  int32_t* S;
  int32_t* R;
  int32_t* chunk_first;
  uint64_t* flagsA;
  uint64_t* flagsB;
  uint32_t epochA, epochB;
  unsigned long long* ticket;
  uint32_t* nf_out;          // list length
  uint32_t* mf_out;          // total degree (when rowptr)
  // nullable: also add up the in-degrees of the rows set in unv_nz AND NOT unv_vis (the
  // vertices still unvisited) into mu_slot's stripes
  LevelSlot* mu_slot;
  const uint32_t* unv_nz;
  const uint32_t* unv_vis;
  const int32_t* colptr;
};

// ---- launchers (kernels.hip, batch.hip); each returns hipGetLastError() ----
// Where a launcher takes events t0 / t1 they receive the kernel's own start
// and end times (AMD's extended launch), so an event interval is the
// kernel's execution alone, not the gap before it.
hipError_t launch_bfs_init(hipStream_t s, const BfsArgs& a, int32_t source, int32_t dir0,
                          hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_level_prep(hipStream_t s, const BfsArgs& a, int32_t level, int32_t forced_dir,
                            hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_ctrl_init(hipStream_t s, Ctrl* ctrl, uint64_t* flags, int64_t nflags);
hipError_t launch_scan_bits(hipStream_t s, const ScanBitsArgs& a);
hipError_t launch_expand(hipStream_t s, const ExpandArgs& a, const uint32_t* m_dev,
                         const uint32_t* nf_dev);
hipError_t launch_pull(hipStream_t s, const PullArgs& a);
hipError_t launch_fill(hipStream_t s, uint32_t* p, int64_t n, uint32_t v);
hipError_t launch_s2d(hipStream_t s, const int32_t* idx, int32_t n, int32_t V, uint32_t* bits);
hipError_t launch_mxv_finalize(hipStream_t s, uint32_t* y, const uint32_t* r, int32_t nwords,
                               int32_t V, int accum, LevelSlot* slot);
// bit v set when row v of the offsets has more than min_len entries
hipError_t launch_nz_bits(hipStream_t s, const int32_t* ptr, int32_t V, uint32_t* bits, int32_t min_len = 0);
hipError_t launch_slab(hipStream_t s, const int32_t* ptr, const int32_t* ind, int32_t V, int4* slab,
                       int32_t* head);
hipError_t launch_max_degree(hipStream_t s, const int32_t* ptr, int32_t V, uint32_t* out);
// slot->s[*].edges += out-degrees (CSR offsets ptr) of the vertices with depth >= 0; slot zeroed first
hipError_t launch_reached_degree(hipStream_t s, const int32_t* ptr, const int32_t* depth, int32_t V,
                                 LevelSlot* slot);
// What the host needs after a batch of levels: the state after the batch and
// the records of its levels. Written into pinned host memory by one block,
// `seq` last (system-scope release), so the host can spin on it.
constexpr int kMaxBatch = 64;
struct HostReport {
  LevelState end;
  LevelRecord rec[kMaxBatch];
  LevelState steps[kMaxBatch];  // the state each step of the batch published
  int32_t nrec;                 // records in rec (levels rec_first ..)
  int32_t error;                // persistent loop: 1 when a grid barrier wait gave up
  unsigned long long t_end;     // persistent loop, timed: device clock when its last block ended
  uint32_t seq;
};
// single-source step loop (kernels.hip); a step given report arguments also
// writes the report of the batch it ends (block 0, after publishing its state)
struct StepReportArgs {
  HostReport* host;  // nullptr: no report
  uint32_t seq;
  int32_t s_first, rec_first;
};
hipError_t launch_step(hipStream_t s, const BfsArgs& a, int32_t step, hipEvent_t t0 = nullptr,
                       hipEvent_t t1 = nullptr, const StepReportArgs* rp = nullptr);
hipError_t launch_step_report(hipStream_t s, const Ctrl* ctrl, int32_t s_first, int32_t n, int32_t rec_first,
                              HostReport* host, uint32_t seq);
// The persistent form of the step loop: one launch runs steps s_first .. s_first + n - 1 with a
// grid barrier between steps (over `blocks` co-resident blocks, each looping over the virtual
// blocks of one step launch), the report written as the step loop's last step writes it.
// spin_limit bounds every barrier wait (polls); timing: per-step start times in the published
// states and the launch's end in ctrl->bar.t_end.
hipError_t launch_steps(hipStream_t s, const BfsArgs& a, int32_t s_first, int32_t n, int32_t blocks,
                        uint32_t spin_limit, bool timing, const StepReportArgs& rp, hipEvent_t t0 = nullptr,
                        hipEvent_t t1 = nullptr);
// Blocks of the persistent step loop that fit on the current device at once.
hipError_t persistent_capacity(int32_t* blocks);
hipError_t launch_mb_init(hipStream_t s, const BatchArgs& a, int32_t dir0, int64_t nflags,
                         hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// Step `step` of the multi-source step loop (k_mb_step) on `blocks` blocks (0 or more than
// the full grid: the full grid).
hipError_t launch_mb_step(hipStream_t s, const BatchArgs& a, int32_t step, int64_t blocks = 0,
                          hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// The persistent form of the multi-source step loop (k_mb_steps): steps s_first .. s_first +
// n - 1 in one launch of `blocks` co-resident blocks, a grid barrier between steps; the report
// is written afterwards by launch_step_report.
hipError_t launch_mb_steps(hipStream_t s, const BatchArgs& a, int32_t s_first, int32_t n, int32_t blocks,
                           uint32_t spin_limit, bool timing, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// Blocks of k_mb_steps that fit on the current device at once.
hipError_t persistent_capacity_mb(int32_t* blocks);
// Destination of each source's depth row (int32[V], device).
struct DepthRows {
  int32_t* row[kMaxSources];
};
// depth rows from the level table, when the state step `step` published says the traversal
// is over (its vis_idx names the final visited words); otherwise nothing
hipError_t launch_mb_depth(hipStream_t s, const BatchArgs& a, int32_t step, const DepthRows& rows);
hipError_t launch_check_offsets(hipStream_t s, const int32_t* ptr, int32_t V, int64_t nnz,
                                int32_t* err);
hipError_t launch_check_indices(hipStream_t s, const int32_t* idx, int64_t nnz, int32_t V,
                                int32_t* err);

// ---- sort-based push (sortpush.hip) ----
size_t sort_push_bytes(int64_t nnz);  // radix-sort scratch for nnz pairs (enough for nnz keys alone)
// rowind_out = every CSC column of rowind_in reordered by decreasing out-degree of its rows
// (stable: equal degrees keep their order); allocates and frees its own scratch.
hipError_t hubs_first(hipStream_t s, const int32_t* rowptr, const int32_t* colptr, const int32_t* rowind_in,
                      int32_t* rowind_out, int32_t V, int64_t nnz, uint32_t maxdeg);
hipError_t launch_sort_gather(hipStream_t s, const ExpandArgs& a, uint32_t* keys, int32_t* vals);
hipError_t sort_pairs(hipStream_t s, void* tmp, size_t tmp_bytes, const uint32_t* kin, uint32_t* kout,
                      const int32_t* vin, int32_t* vout, uint32_t m, int bits);
hipError_t sort_keys(hipStream_t s, void* tmp, size_t tmp_bytes, const uint32_t* kin, uint32_t* kout, uint32_t m,
                     int bits);
hipError_t launch_sort_filter(hipStream_t s, const uint32_t* keys, const int32_t* vals, uint32_t m, uint32_t* vis,
                              int32_t* depth, int32_t* parent, int32_t level, int32_t* Qout, uint32_t* qcount,
                              LevelSlot* slot);

// ---- host runtime entry points shared between api.hip and serve.hip ----
// Multi-source traversal writing source b's depths to rows.row[b].
dobfs_status bfs_batch_rows(dobfs_graph g, const int32_t* sources, int32_t k, const dobfs_options* opt,
                            const DepthRows& rows, void* workspace, size_t ws_bytes, void* stream,
                            dobfs_stats* stats);
// Options a multi-source traversal accepts (sets the thread's last error otherwise).
dobfs_status check_batch_options(const dobfs_options& opt);
// Records `what` as the calling thread's last error and returns s.
dobfs_status set_error(dobfs_status s, const char* what);

// Direction rule of Section 6.3 (and Beamer's edge form); identical on host and device.
__host__ __device__ inline int32_t next_direction_rule(int32_t heuristic, double alpha, double beta,
                                                       int32_t dir, int64_t V, int64_t nf,
                                                       int64_t n_new, int64_t m_f, int64_t m_u) {
  if (heuristic == 1) {  // edge counts
    if (dir == 0) return double(m_f) > alpha * double(m_u) ? 1 : 0;
    return double(n_new) < beta * double(V) ? 0 : 1;
  }
  if (dir == 0) return (n_new > nf && double(n_new) > alpha * double(V)) ? 1 : 0;
  return (n_new < nf && double(n_new) < beta * double(V)) ? 0 : 1;
}

}  // namespace dobfs
