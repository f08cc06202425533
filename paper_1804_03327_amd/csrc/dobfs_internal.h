// Internal declarations shared by the HIP kernels and the host runtime of
// libdobfs. Not part of the public ABI (see include/dobfs.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace dobfs {

// ---- per-level counters ----
// Same-address device atomics serialize (about 11 ns each on MI355X), so
// every block adds its partial sums into one of kStripes counters, each on
// its own 128-byte line; the host adds the stripes up after the level.
constexpr int kStripes = 32;
struct alignas(128) Stripe {
  uint32_t count;  // vertices discovered (BFS) / result bits (mxv)
  uint32_t aux;    // mxv: popcount of the whole output vector
  uint64_t edges;  // adjacency entries read (push) or in-neighbours checked (pull)
  uint64_t mnew;   // out-edges of the vertices discovered (edge-count rule only)
  uint64_t insub;  // in-edges of the vertices discovered (edge-count rule only)
};
struct LevelSlot {
  Stripe s[kStripes];
};
constexpr int kSlots = 4;  // level L accumulates into slot L % kSlots

struct Ctrl {
  unsigned long long ticket;  // tile tickets of the single-pass scans (monotone within a call)
  uint32_t mf32;              // m_f of the latest push scan, read by the expand kernel
  uint32_t d2s_count;         // output length of the latest dense-to-sparse conversion
  int64_t src_outdeg;         // out-degree of the BFS source
  int64_t src_indeg;          // in-degree of the BFS source
  uint32_t qcount[kSlots];    // frontier-list append counter of each level
  uint64_t mf[kSlots];        // push: out-edges of the input frontier
  uint8_t pad[128 - 48 - 8 * kSlots];
  LevelSlot slot[kSlots];
};
static_assert(sizeof(Stripe) == 128, "stripe layout");
static_assert(offsetof(Ctrl, slot) % 128 == 0, "slots start on a line");

// Host-side totals of one level.
struct LevelTotals {
  uint64_t count, aux, edges, mnew, insub;
};
inline LevelTotals sum_slot(const LevelSlot& s) {
  LevelTotals t{0, 0, 0, 0, 0};
  for (int k = 0; k < kStripes; ++k) {
    t.count += s.s[k].count;
    t.aux += s.s[k].aux;
    t.edges += s.s[k].edges;
    t.mnew += s.s[k].mnew;
    t.insub += s.s[k].insub;
  }
  return t;
}

// ---- launch geometry (all kernels use 256-thread blocks = 4 wave64) ----
constexpr int kThreads = 256;
constexpr int kScanIPT = 8;                       // push scan: frontier entries per thread
constexpr int kScanTile = kThreads * kScanIPT;   // 2048 entries per tile
constexpr int kExpandEPT = 4;                     // push expand: edges per thread per chunk
constexpr int kExpandChunk = kThreads * kExpandEPT;  // 1024 edges per chunk
constexpr int kExpandWin = kExpandChunk + 1;      // frontier entries cached in LDS per chunk
constexpr int kExpandBuf = 4096;                  // winners buffered in LDS before a queue flush
constexpr int kExpandBlocks = 1024;               // expand grid (strides over chunks)
constexpr int kPullTileWords = 64;                // pull: bitmap words owned by a block
constexpr int kPullTileV = kPullTileWords * 32;   // 2048 rows per block
constexpr int kPullFirst = 4;                     // in-neighbours one thread checks before handing a row to its wave
constexpr int kPullBatch = 4;                     // candidate rows a thread works on at once
constexpr int kD2SWPT = 4;                        // D2S: words per thread
constexpr int kD2STile = kThreads * kD2SWPT;      // 1024 words per tile

inline int32_t words_of(int64_t V) { return int32_t((V + 31) / 32); }
inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }
inline int64_t d2s_tiles(int64_t nwords) { return (nwords + kD2STile - 1) / kD2STile; }
inline int64_t max_chunks(int64_t nnz) { return nnz / kExpandChunk + 2; }

// ---- kernel argument blocks ----
struct PullArgs {
  int32_t V, nwords;
  const int32_t* colptr;
  const int32_t* rowind;
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
  int32_t count_out;         // 1: add popcount(out) to the stripes' aux (mxv)
  int32_t edge_rule;         // 1: add in-degrees of the results to the stripes' insub
  LevelSlot* slot;
  LevelSlot* reset;          // nullable: zeroed by block 0 before use by the next level
  int32_t reset_level;       // slot index of `reset` (its queue counter is zeroed too)
  Ctrl* ctrl;
};

struct ExpandArgs {
  const int32_t* Q;          // frontier list
  int32_t nf;                // frontier length (used when nf_dev is null)
  const uint32_t* nf_dev;    // nullable: frontier length on the device
  const int32_t* S;          // exclusive scan of out-degrees
  const int32_t* R;          // row start of each frontier vertex
  const int32_t* chunk_first;  // first frontier entry of every edge chunk
  const int32_t* colind;
  Ctrl* ctrl;                // mf32 = total edges; qcount = append counter
  uint32_t* claim;           // bitmap claimed with atomicOr (visited / result)
  const uint32_t* mask;      // nullable: filter before the claim
  int32_t complement;
  int32_t* depth;            // nullable
  int32_t* parent;           // nullable: parent / witness
  int32_t level;
  int32_t* Qout;             // nullable: winners appended here
  int32_t qslot;             // which ctrl->qcount counts the appends
  const int32_t* out_rowptr; // nullable: CSR(A) offsets; out-degrees of winners -> mnew
  const int32_t* in_colptr;  // nullable: CSC(A) offsets; in-degrees of winners -> insub
  LevelSlot* slot;
  LevelSlot* reset;
  int32_t reset_level;
};

// ---- launchers (kernels.hip); each returns hipGetLastError() ----
hipError_t launch_bfs_init(hipStream_t s, int32_t V, int32_t nwords, int32_t source,
                           const int32_t* rowptr, const int32_t* colptr, int32_t* depth,
                           int32_t* parent, uint32_t* vis, int32_t* Q, Ctrl* ctrl, uint64_t* flags,
                           int64_t nflags);
hipError_t launch_ctrl_init(hipStream_t s, Ctrl* ctrl, uint64_t* flags, int64_t nflags);
hipError_t launch_push_scan(hipStream_t s, int64_t tiles, const int32_t* Q, int32_t nf,
                            const uint32_t* nf_dev, const int32_t* rowptr, int32_t* S, int32_t* R,
                            int32_t* chunk_first, Ctrl* ctrl, unsigned long long ticket_base,
                            uint32_t epoch, uint64_t* flags, int32_t level_slot, LevelSlot* reset,
                            int32_t reset_level);
hipError_t launch_push_expand(hipStream_t s, int32_t blocks, const ExpandArgs& a);
hipError_t launch_pull(hipStream_t s, bool early_exit, const PullArgs& a);
hipError_t launch_d2s(hipStream_t s, const uint32_t* a, const uint32_t* b_not, int32_t nwords,
                      int32_t V, int32_t* out, Ctrl* ctrl, unsigned long long ticket_base,
                      uint32_t epoch, uint64_t* flags, uint32_t* count_out);
hipError_t launch_fill(hipStream_t s, uint32_t* p, int64_t n, uint32_t v);
hipError_t launch_s2d(hipStream_t s, const int32_t* idx, int32_t n, const uint32_t* n_dev,
                      int32_t V, uint32_t* bits);
hipError_t launch_mxv_finalize(hipStream_t s, uint32_t* y, const uint32_t* r, int32_t nwords,
                               int32_t V, int accum, LevelSlot* slot);
hipError_t launch_nz_bits(hipStream_t s, const int32_t* ptr, int32_t V, uint32_t* bits);
hipError_t launch_check_offsets(hipStream_t s, const int32_t* ptr, int32_t V, int64_t nnz,
                                int32_t* err);
hipError_t launch_check_indices(hipStream_t s, const int32_t* idx, int64_t nnz, int32_t V,
                                int32_t* err);

}  // namespace dobfs
