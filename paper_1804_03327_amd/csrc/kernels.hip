// HIP kernels of libdobfs for gfx950 (CDNA4, wave64).
//
// One BFS level is the Boolean masked matvec f' = A^T f .* not(v)
// (Algorithm 1). Push computes it column by column from the frontier list
// (Equation 5, Section 6.2); pull computes it row by row over the rows the
// mask lets through, stopping at the first hit (Equation 4, Algorithm 2,
// Sections 5.2-5.4). Everything is integer / bitwise: no MFMA.
//
// The level loop is a loop of steps, one launch of k_step each: a level is
// one step (a pull, or a push that shares out its own work inside blocks), or
// two when its push needs the global degree scan (scan step, expansion step).
// Every block of a step decides the level itself on the device (the rule of
// Section 6.3, from the counters the previous step left). The host enqueues
// many steps ahead and reads the states back once per batch. k_steps runs the
// same steps in one persistent launch; k_level_prep serves the sort-based
// push of Table 2's first rows, whose host loop sizes the sort per level.
//
// Memory layout (HBM): CSR(A) and CSC(A) int32 arrays; bit vectors as uint32
// words (bit i = word i>>5, bit i&31); frontier lists as int32.
//
// Rates that shaped these kernels (measured on MI355X): random 4-byte loads
// from a 512 KiB L2-resident bitmap ~270 G/s; atomics on distinct words
// ~27 G/s; atomics on one address ~0.09 G/s (serialized); streaming reads
// ~6.4 TB/s; a kernel boundary ~3 us; a host round trip ~15 us. So the
// bitmaps are read with plain loads first, per-level counters are striped
// over kStripes lines, list appends are batched per block in LDS, and levels
// are decided on the device.

#include "device_common.h"

#include <algorithm>

namespace dobfs {
namespace {

// ----------------------------------------------------------------- push
struct ExpandShared {
  int32_t sS[kExpandWin], sR[kExpandWin], sQ[kExpandWin];
  int32_t buf[kExpandBuf];
  uint32_t nbuf, base;
};

// Load-balanced gather over the concatenated adjacency of the frontier: a
// block takes chunks of kExpandChunk consecutive edges; each edge finds its
// frontier vertex by a search over the chunk's window of the scan (the
// interval-gather step of Section 6.2), so supervertices spread over many
// blocks and adjacent lanes read adjacent column indices. Each thread carries
// kExpandEPT edges at once so their loads overlap. The merge + mask filter of
// the paper's sort-based version is one atomicOr per edge whose target still
// looks unvisited: the first setter of a bit owns the vertex (Boolean OR
// makes any winner exact), which both deduplicates and applies the mask
// not(v). Winners are buffered in LDS and appended to the next frontier list
// with one atomic per flush.
__device__ __forceinline__ void expand_body(const ExpandArgs& a, ExpandShared& sh, uint32_t bid, uint32_t nblk) {
  const int32_t nf = a.nf;
  const uint32_t m = a.m;
  if (nf <= 0 || m == 0) return;
  const uint32_t nchunks = (m + kExpandChunk - 1) / kExpandChunk;
  if (bid >= nchunks) return;
  if (threadIdx.x == 0) sh.nbuf = 0;
  unsigned long long won_total = 0, mnew = 0, insub = 0;
  uint32_t maxdeg = 0;
  const uint32_t cflip = a.complement ? 1u : 0u;

  auto flush = [&]() {  // all threads; callers are past a barrier
    const uint32_t nb = sh.nbuf;
    if (nb == 0) return;
    if (threadIdx.x == 0) sh.base = atomicAdd(a.qcount, nb);
    __syncthreads();
    const uint32_t b = sh.base;
    for (uint32_t k = threadIdx.x; k < nb; k += kThreads) a.Qout[b + k] = sh.buf[k];
    __syncthreads();
    if (threadIdx.x == 0) sh.nbuf = 0;
    __syncthreads();
  };

  for (uint32_t c = bid; c < nchunks; c += nblk) {
    const uint32_t e0 = c * kExpandChunk;
    const uint32_t e1 = min(e0 + uint32_t(kExpandChunk), m);
    const int32_t k0 = a.chunk_first[c];
    const int32_t k1 = (c + 1 < nchunks) ? a.chunk_first[c + 1] : nf - 1;
    const int32_t n = k1 - k0 + 1;
    const bool in_lds = n <= kExpandWin;
    __syncthreads();  // previous chunk's LDS readers are done, nbuf is settled
    if (a.Qout && sh.nbuf + kExpandChunk > kExpandBuf) flush();
    if (in_lds) {
      for (int32_t i = threadIdx.x; i < n; i += kThreads) {
        sh.sS[i] = a.S[k0 + i];
        sh.sR[i] = a.R[k0 + i];
        sh.sQ[i] = a.Q[k0 + i];
      }
    }
    __syncthreads();
    int32_t w[kExpandEPT], u[kExpandEPT], pos[kExpandEPT];
    bool valid[kExpandEPT], won[kExpandEPT];
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      const uint32_t e = e0 + uint32_t(t * kThreads) + threadIdx.x;
      valid[t] = e < e1;
      pos[t] = 0;
      u[t] = 0;
      if (valid[t]) {
        int32_t s, rs;
        if (in_lds) {
          const int32_t kk = thread_search(sh.sS, 0, n, e);
          s = sh.sS[kk]; rs = sh.sR[kk]; u[t] = sh.sQ[kk];
        } else {
          const int32_t kk = thread_search(a.S, k0, k1 + 1, e);
          s = a.S[kk]; rs = a.R[kk]; u[t] = a.Q[kk];
        }
        pos[t] = rs + int32_t(e - uint32_t(s));
      }
    }
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) w[t] = valid[t] ? a.colind[pos[t]] : 0;
    uint32_t seen[kExpandEPT];
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      bool pass = valid[t];
      if (pass && a.mask) pass = (get_bit(a.mask, w[t]) ^ cflip) != 0;
      valid[t] = pass;
      seen[t] = pass ? a.claim[w[t] >> 5] : 0xffffffffu;
    }
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      const uint32_t bit = 1u << (w[t] & 31);
      won[t] = false;
      if (valid[t] && !(seen[t] & bit)) won[t] = !(atomicOr(a.claim + (w[t] >> 5), bit) & bit);
    }
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      if (won[t]) {
        ++won_total;
        if (a.depth) a.depth[w[t]] = a.level + 1;
        if (a.parent) a.parent[w[t]] = u[t];
        if (a.found_out) atomicOr(a.found_out + (w[t] >> 5), 1u << (w[t] & 31));
        uint32_t dw = 0;
        if (a.out_rowptr) {
          dw = uint32_t(a.out_rowptr[w[t] + 1] - a.out_rowptr[w[t]]);
          mnew += dw;
          maxdeg = max(maxdeg, dw);
        }
        if (a.in_colptr)  // an undirected graph keeps one offset array for both directions
          insub += a.in_colptr == a.out_rowptr ? uint64_t(dw) : uint64_t(a.in_colptr[w[t] + 1] - a.in_colptr[w[t]]);
      }
      if (a.Qout) {
        const uint64_t bal = __ballot(won[t]);
        if (bal) {
          const int cnt = __popcll(bal);
          const int leader = __ffsll((unsigned long long)bal) - 1;
          uint32_t p = 0;
          if (lane() == leader) p = atomicAdd(&sh.nbuf, uint32_t(cnt));
          p = __shfl(p, leader, 64);
          if (won[t]) sh.buf[p + __popcll(bal & lanemask_lt())] = w[t];
        }
      }
    }
  }
  __syncthreads();
  if (a.Qout) flush();
  unsigned long long v[4] = {won_total, mnew, insub, 0};
  block_sum4(v);
  maxdeg = block_max32(maxdeg);
  if (threadIdx.x == 0) {
    // every edge of a chunk is read exactly once; the block's chunks sum to its edges
    unsigned long long edges = 0;
    for (uint32_t c = bid; c < nchunks; c += nblk)
      edges += min(uint32_t(kExpandChunk), m - c * kExpandChunk);
    stripe_add(a.slot, v[0], 0, edges, v[1], v[2]);
    stripe_max(a.slot, maxdeg);
  }
}

// Pushes that need no global degree scan: the load balancing of the
// column-based matvec is done inside each block. A block takes a.unit
// frontier vertices at a time (a unit), scans their degrees in LDS and walks
// the unit's edges kExpandChunk at a time, each edge finding its vertex by a
// search over the unit's prefix; the claim and the winners' bookkeeping are
// those of expand_body.
// Local culling (the block-level dedupe Section 7.3 credits Gunrock with): a
// direct-mapped table in LDS of the targets this block has already sent on to
// the claim in this step. An edge whose target is found there is dropped
// before its visited-word load and claim: the edge that entered the target
// goes on to claim it (or finds it claimed), so the target is still reached
// at this level, from a frontier vertex, and the depths and the validity of
// the parents do not change. A collision only overwrites an entry, which
// costs a redundant claim, never a lost one. Only levels with a frontier of
// kCullMinFrontier vertices or more cull: smaller ones are bound by their
// chain of dependent loads, which the table's atomics would only lengthen.
constexpr int kCullBits = 10;
constexpr int32_t kCullMinFrontier = 8192;
constexpr uint32_t kCullNone = 0xffffffffu;  // no vertex id (ids are below 2^31)

struct LocalShared {
  int32_t off[kThreads + 1], beg[kThreads], src[kThreads];
  int32_t buf[kExpandBuf];
  uint16_t list[kPullTileV];  // bitmap push: the block's frontier rows (offsets in its slice)
  uint32_t cull[1 << kCullBits];
  uint32_t nbuf, base;
};

// Empties the culling table (all threads; a barrier follows before its first use).
__device__ __forceinline__ void cull_reset(LocalShared& sh) {
  for (int i = threadIdx.x; i < (1 << kCullBits); i += kThreads) sh.cull[i] = kCullNone;
}

// True when target w is new to this block's table (and enters it).
__device__ __forceinline__ bool cull_enter(LocalShared& sh, int32_t w) {
  const uint32_t h = (uint32_t(w) * 2654435761u) >> (32 - kCullBits);
  return atomicExch(&sh.cull[h], uint32_t(w)) != uint32_t(w);
}

struct LocalAcc {
  unsigned long long won = 0, mnew = 0, insub = 0, edges = 0;
  uint32_t maxdeg = 0;
};

// Appends the buffered winners to the next frontier list (all threads; the
// callers are past a barrier).
__device__ __forceinline__ void local_flush(const ExpandArgs& a, LocalShared& sh) {
  const uint32_t nb = sh.nbuf;
  if (nb == 0) return;
  if (threadIdx.x == 0) sh.base = atomicAdd(a.qcount, nb);
  __syncthreads();
  const uint32_t b = sh.base;
  for (uint32_t k = threadIdx.x; k < nb; k += kThreads) a.Qout[b + k] = sh.buf[k];
  __syncthreads();
  if (threadIdx.x == 0) sh.nbuf = 0;
  __syncthreads();
}

// Loads unit vertex v (-1: none) of this thread, scans the unit's degrees
// into sh.off / beg / src and returns the unit's edge count. The scan's
// first barrier also orders the previous unit's LDS reads before the writes.
__device__ __forceinline__ uint32_t local_unit_prefix(const ExpandArgs& a, LocalShared& sh, int32_t v) {
  int32_t b = 0, d = 0;
  if (v >= 0) {
    b = a.rowptr[v];
    d = a.rowptr[v + 1] - b;
  }
  uint32_t total;
  const uint32_t ex = block_excl_scan(uint32_t(d), &total);
  sh.off[threadIdx.x] = int32_t(ex);
  sh.beg[threadIdx.x] = b;
  sh.src[threadIdx.x] = v;
  if (threadIdx.x == 0) sh.off[kThreads] = int32_t(total);
  return total;
}

// The chunks first, first + step, ... of a unit of n vertices whose prefix
// local_unit_prefix() wrote.
__device__ __forceinline__ void local_unit_chunks(const ExpandArgs& a, LocalShared& sh, int32_t n, uint32_t total, uint32_t first,
                                  uint32_t step, bool cull, LocalAcc& acc) {
  const int tid = threadIdx.x;
  for (uint32_t e0 = first; e0 < total; e0 += step) {
    __syncthreads();  // the unit's prefix is written, nbuf is settled
    if (sh.nbuf + kExpandChunk > uint32_t(kExpandBuf)) local_flush(a, sh);
    int32_t w[kExpandEPT], uu[kExpandEPT];
    bool valid[kExpandEPT], won[kExpandEPT];
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      const uint32_t e = e0 + uint32_t(t * kThreads + tid);
      valid[t] = e < total;
      w[t] = 0;
      uu[t] = 0;
      if (valid[t]) {
        const int32_t k = thread_search(sh.off, 0, n, e);
        uu[t] = sh.src[k];
        w[t] = a.colind[sh.beg[k] + int32_t(e - uint32_t(sh.off[k]))];
      }
    }
    if (cull) {
#pragma unroll
      for (int t = 0; t < kExpandEPT; ++t)
        if (valid[t]) valid[t] = cull_enter(sh, w[t]);
    }
    uint32_t seen[kExpandEPT];
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) seen[t] = valid[t] ? a.claim[w[t] >> 5] : 0xffffffffu;
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      const uint32_t bit = 1u << (w[t] & 31);
      won[t] = false;
      if (valid[t] && !(seen[t] & bit)) won[t] = !(atomicOr(a.claim + (w[t] >> 5), bit) & bit);
    }
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      if (won[t]) {
        ++acc.won;
        a.depth[w[t]] = a.level + 1;
        if (a.parent) a.parent[w[t]] = uu[t];
        if (a.found_out) atomicOr(a.found_out + (w[t] >> 5), 1u << (w[t] & 31));
        uint32_t dw = 0;
        if (a.out_rowptr) {
          dw = uint32_t(a.out_rowptr[w[t] + 1] - a.out_rowptr[w[t]]);
          acc.mnew += dw;
          acc.maxdeg = max(acc.maxdeg, dw);
        }
        if (a.in_colptr)
          acc.insub += a.in_colptr == a.out_rowptr ? uint64_t(dw) : uint64_t(a.in_colptr[w[t] + 1] - a.in_colptr[w[t]]);
      }
      const uint64_t bal = __ballot(won[t]);
      if (bal) {
        const int cnt = __popcll(bal);
        const int leader = __ffsll((unsigned long long)bal) - 1;
        uint32_t p = 0;
        if (lane() == leader) p = atomicAdd(&sh.nbuf, uint32_t(cnt));
        p = __shfl(p, leader, 64);
        if (won[t]) sh.buf[p + __popcll(bal & lanemask_lt())] = w[t];
      }
    }
  }
}

// A block's counters into the level's stripes (all threads).
__device__ __forceinline__ void local_finish(const ExpandArgs& a, LocalShared& sh, LocalAcc& acc, unsigned long long mu) {
  __syncthreads();
  local_flush(a, sh);
  unsigned long long vv[4] = {acc.won, acc.mnew, acc.insub, acc.edges};
  block_sum4(vv);
  unsigned long long vm[4] = {mu, 0, 0, 0};
  if (a.mu_slot) block_sum4(vm);
  const uint32_t maxdeg = block_max32(acc.maxdeg);
  if (threadIdx.x == 0) {
    stripe_add(a.slot, vv[0], 0, vv[3], vv[1], vv[2]);
    stripe_max(a.slot, maxdeg);
    if (vm[0]) atomicAdd(&a.mu_slot->s[blockIdx.x % kStripes].mu, vm[0]);
  }
}

// Push over a frontier list whose sizes local_fits() accepts: with fewer
// units than blocks, each unit gets a.share blocks (local_share: what its
// chunks could need, at most gridDim / units), which all scan the unit's
// degrees and take its chunks in turn; otherwise a block takes whole units.
__device__ __forceinline__ void local_expand_body(const ExpandArgs& a, LocalShared& sh, int32_t bid, int32_t nblk) {
  const int32_t nf = a.nf;
  const int32_t unit = a.unit;
  const int32_t nunits = (nf + unit - 1) / unit;
  const int32_t G = nblk;
  const int32_t per_unit = max(1, a.share);  // blocks sharing one unit's chunks (at most G / nunits)
  const int32_t nwork = nunits * per_unit;     // (unit, share) pairs
  if (bid >= nwork) return;                // no work: no counters to add
  const int tid = threadIdx.x;
  if (tid == 0) sh.nbuf = 0;
  const bool cull = nf >= kCullMinFrontier;
  if (cull) cull_reset(sh);
  LocalAcc acc;
  for (int32_t wi = bid; wi < nwork; wi += G) {
    const int32_t u = per_unit == 1 ? wi : wi / per_unit, share = per_unit == 1 ? 0 : wi - u * per_unit;
    const int32_t i = u * unit + tid;
    const uint32_t total = local_unit_prefix(a, sh, (tid < unit && i < nf) ? a.Q[i] : -1);
    acc.edges += (tid == 0 && share == 0) ? total : 0;  // each unit's edges counted once
    local_unit_chunks(a, sh, min(unit, nf - u * unit), total, uint32_t(share) * kExpandChunk,
                      uint32_t(per_unit) * kExpandChunk, cull, acc);
  }
  local_finish(a, sh, acc, 0);
}

// Push over the frontier a pull left as bits (a.front), when no pull tile
// found more than sched.bitmap_rows rows and none of high out-degree: block b
// lists the frontier rows of its own slice of the bitmap (at most one pull
// tile) in LDS and expands them unit by unit, so the level needs neither the
// bitmap-to-list conversion nor the degree scan. Under the edge-count rule
// the block also adds up the in-degrees of its slice's rows still unvisited
// when the level started (m_u, which the pulls do not track).
__device__ __forceinline__ void bitmap_expand_body(const ExpandArgs& a, int32_t nwords, int32_t V, LocalShared& sh,
                                                   int32_t bid, int32_t nblk) {
  const int32_t G = nblk;
  const int32_t wpb = (nwords + G - 1) / G;  // words per block; at most kPullTileWords
  const int32_t w0 = bid * wpb;
  if (w0 >= nwords) return;
  const int32_t w1 = min(w0 + wpb, nwords);
  const int tid = threadIdx.x;
  if (tid == 0) sh.nbuf = 0;
  const bool cull = a.nf >= kCullMinFrontier;
  if (cull) cull_reset(sh);
  const int32_t w = w0 + tid;
  const bool mine = tid < wpb && w < w1;
  const uint32_t fb = mine ? a.front[w] & valid_bits(w, V) : 0u;
  unsigned long long mu = 0;
  if (a.mu_slot && mine) {
    uint32_t u = a.nz[w] & ~(a.vis_before[w] | fb) & valid_bits(w, V);
    while (u) {
      const int32_t v = w * 32 + __ffs(u) - 1;
      mu += uint64_t(a.in_colptr[v + 1] - a.in_colptr[v]);
      u &= u - 1;
    }
  }
  uint32_t nfront;
  const uint32_t pos = block_excl_scan(uint32_t(__popc(fb)), &nfront);
  {
    uint32_t b = fb, p = pos;
    while (b) {
      sh.list[p++] = uint16_t(tid * 32 + __ffs(b) - 1);
      b &= b - 1;
    }
  }
  LocalAcc acc;
  const uint32_t unit = uint32_t(a.unit);
  for (uint32_t u0 = 0; u0 < nfront; u0 += unit) {
    __syncthreads();  // the list is written (first unit) / the previous unit's chunks are done
    const uint32_t i = u0 + uint32_t(tid);
    const int32_t v = (uint32_t(tid) < unit && i < nfront) ? w0 * 32 + int32_t(sh.list[i]) : -1;
    const uint32_t total = local_unit_prefix(a, sh, v);
    acc.edges += tid == 0 ? total : 0;
    local_unit_chunks(a, sh, int32_t(min(unit, nfront - u0)), total, 0, kExpandChunk, cull, acc);
  }
  local_finish(a, sh, acc, mu);
}

// ----------------------------------------------------------------- pull
struct PullShared {
  uint16_t cand[kPullTileV];
  uint16_t mid[kPullTileV];
  uint16_t lng[kPullTileV];
  uint32_t found[kPullTileWords];
  int32_t ncand, nopen, nmid, nlong;
};

// Row-based masked matvec (Algorithm 2) over CSC(A) for the rows of one
// tile of kPullTileWords bitmap words: list the rows the mask lets through
// (output sparsity, Section 5.2) and check each row's in-neighbours in stored
// order, stopping at the first hit (early exit, Section 5.3). The phases
// keep many loads in flight: every candidate's first in-neighbour from the
// head array (kPullHeadBatch rows per thread at once); the slab (in-neighbours
// 1..3, one 16-byte read) of the rows still open, kPullBatch per thread; then
// rows still open, one per thread, kPullStep positions per load round, up to
// a.mid; then what is left, one row per wave, 64 in-neighbours per step
// with the lowest hitting lane kept. Every phase scans positions in
// order and keeps the first hit, so the reported parent is always the first
// in stored order. Results gather in LDS and the tile's words of the output
// vector are written whole, so no atomics touch the output bitmap. `x` (the
// input vector) is never written here, which keeps the visited snapshot exact
// when x = visited (operand reuse, Section 5.4).
template <bool EE>
__device__ __forceinline__ void pull_body(const PullArgs& a, int32_t tile, PullShared& sh) {
  const int tid = threadIdx.x;
  const int32_t w0 = tile * kPullTileWords;
  const int32_t v0 = w0 * 32;
  const uint32_t cflip = a.complement ? 0xffffffffu : 0u;

  // the tile's candidate rows (mask passed, in-degree > 0) listed in order:
  // two threads per bitmap word, sixteen bits each, placed by a block scan
  {
    static_assert(kPullTileWords * 2 == kThreads, "two threads per tile word");
    const int lw = tid >> 1, half = tid & 1;
    const int32_t w = w0 + lw;
    if (half == 0) sh.found[lw] = 0;
    uint32_t cw = 0;
    if (w < a.nwords) {
      const uint32_t pass = a.mask ? (a.mask[w] ^ cflip) : 0xffffffffu;
      cw = (a.mask_after ? 0xffffffffu : pass) & a.nz[w] & valid_bits(w, a.V);
      cw = half ? (cw >> 16) : (cw & 0xffffu);
    }
    uint32_t total;
    uint32_t pos = block_excl_scan(uint32_t(__popc(cw)), &total);
    const int base_bit = lw * 32 + half * 16;
    while (cw) {
      sh.cand[pos++] = uint16_t(base_bit + __ffs(cw) - 1);
      cw &= cw - 1;
    }
    if (tid == 0) {
      sh.ncand = int32_t(total);
      sh.nopen = 0;
      sh.nmid = 0;
      sh.nlong = 0;
    }
  }
  __syncthreads();
  const int32_t ncand = sh.ncand;
  unsigned long long checks = 0;

  auto record = [&](int32_t off, int32_t j) {
    const int32_t i = v0 + off;
    if (a.mask_after && a.mask && !(get_bit(a.mask, i) ^ (cflip & 1u))) return;
    atomicOr(&sh.found[off >> 5], 1u << (off & 31));
    if (a.depth) a.depth[i] = a.level + 1;
    if (a.parent) a.parent[i] = j;
  };

  // phase 1a: every candidate's first in-neighbour from the head array (4
  // bytes per row, so a level touching few rows of a line reads little),
  // kPullHeadBatch rows per thread with every load issued before any test.
  // Rows with more in-neighbours that this does not settle are listed in
  // sh.lng (free until phase 2) for the slab pass; the flag bit marks a row
  // already found (no early exit: keep counting, do not record again).
  for (int32_t base = 0; base < ncand; base += kPullHeadBatch * kThreads) {
    int32_t idx[kPullHeadBatch], h[kPullHeadBatch];
    uint32_t wd[kPullHeadBatch];
#pragma unroll
    for (int t = 0; t < kPullHeadBatch; ++t) {
      idx[t] = base + t * kThreads + tid;
      h[t] = idx[t] < ncand ? a.head[v0 + int32_t(sh.cand[idx[t]])] : 0;
    }
#pragma unroll
    for (int t = 0; t < kPullHeadBatch; ++t) {
      const int32_t j = h[t] < 0 ? ~h[t] : h[t];
      wd[t] = idx[t] < ncand ? a.x[j >> 5] : 0u;
    }
#pragma unroll
    for (int t = 0; t < kPullHeadBatch; ++t) {
      if (idx[t] >= ncand) continue;
      const int32_t j = h[t] < 0 ? ~h[t] : h[t];
      const bool hit = ((wd[t] >> (j & 31)) & 1u) != 0;
      ++checks;
      if (hit) record(int32_t(sh.cand[idx[t]]), j);
      if (h[t] < 0 && (!EE || !hit)) sh.lng[atomicAdd(&sh.nopen, 1)] = uint16_t(idx[t] | (hit ? 0x8000 : 0));
    }
  }
  __syncthreads();

  // phase 1b: rows still open read their slab (the first kSlab in-neighbours
  // in one 16-byte load; position 0 was the head) and test positions 1..3 in
  // order; a row with more in-neighbours than the slab holds goes on to phase 2
  const int32_t nopen = sh.nopen;
  for (int32_t base = 0; base < nopen; base += kPullBatch * kThreads) {
    int32_t ent[kPullBatch], off[kPullBatch], hitj[kPullBatch];
    int4 hd[kPullBatch];
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) {
      const int32_t r = base + t * kThreads + tid;
      ent[t] = r < nopen ? int32_t(sh.lng[r]) : -1;
      off[t] = ent[t] >= 0 ? int32_t(sh.cand[ent[t] & 0x7fff]) : -1;
    }
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) hd[t] = off[t] >= 0 ? a.slab[v0 + off[t]] : make_int4(-1, -1, -1, -1);
    uint32_t wd[kPullBatch][kSlab - 1];
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) {
      const int32_t e[kSlab - 1] = {hd[t].y, hd[t].z, hd[t].w};
#pragma unroll
      for (int q = 0; q < kSlab - 1; ++q) wd[t][q] = e[q] >= 0 ? a.x[e[q] >> 5] : 0u;
    }
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) {
      hitj[t] = -1;
      if (off[t] < 0) continue;
      const bool done = (ent[t] & 0x8000) != 0;
      const int32_t e[kSlab - 1] = {hd[t].y, hd[t].z, hd[t].w};
#pragma unroll
      for (int q = 0; q < kSlab - 1; ++q) {
        if (e[q] < 0 || (EE && hitj[t] >= 0)) continue;  // past the row's end / stopped at a hit
        ++checks;
        if (hitj[t] < 0 && !done && ((wd[t][q] >> (e[q] & 31)) & 1u)) hitj[t] = e[q];
      }
      if (hitj[t] >= 0) record(off[t], hitj[t]);
    }
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) {
      // a full slab may hide more in-neighbours: the extent decides
      if (off[t] < 0 || hd[t].w < 0 || (EE && hitj[t] >= 0)) continue;
      const int32_t beg = a.colptr[v0 + off[t]], end = a.colptr[v0 + off[t] + 1];
      if (end > beg + kSlab)
        sh.mid[atomicAdd(&sh.nmid, 1)] = uint16_t((ent[t] & 0x7fff) | (((ent[t] & 0x8000) || hitj[t] >= 0) ? 0x8000 : 0));
    }
  }
  __syncthreads();

  // phase 2: open rows, one per thread, kPullStep positions per load round
  const int32_t nmid = sh.nmid;
  for (int32_t r = tid; r < nmid; r += kThreads) {
    const uint16_t ent = sh.mid[r];
    const bool done = (ent & 0x8000) != 0;  // no early exit: already recorded, keep counting
    const int32_t off = sh.cand[ent & 0x7fff];
    const int32_t i = v0 + off;
    const int32_t beg0 = a.colptr[i], end = a.colptr[i + 1];
    const int32_t lim = end - beg0 > a.mid ? beg0 + a.mid : end;  // (no overflow near 2^31 entries)
    int32_t hit = -1;
    unsigned long long n = 0;
    for (int32_t p = beg0 + kPullFirst; p < lim && (!EE || hit < 0); p += kPullStep) {
      int32_t jj[kPullStep];
#pragma unroll
      for (int u = 0; u < kPullStep; ++u) jj[u] = p + u < lim ? a.rowind[p + u] : -1;
#pragma unroll
      for (int u = 0; u < kPullStep; ++u) {
        if (jj[u] < 0) continue;
        if (EE && hit >= 0) continue;  // stopped at the first hit of this round
        ++n;
        if (hit < 0 && !done && get_bit(a.x, jj[u])) hit = jj[u];
      }
    }
    checks += n;
    if (hit >= 0) record(off, hit);
    if (end > lim && (!EE || hit < 0))
      sh.lng[atomicAdd(&sh.nlong, 1)] = uint16_t((ent & 0x7fff) | ((done || hit >= 0) ? 0x8000 : 0));
  }
  __syncthreads();

  // phase 3: what is left, one row per wave, 64 in-neighbours per step
  const int32_t nlong = sh.nlong;
  const int wv = tid >> 6;
  for (int32_t r = wv; r < nlong; r += kThreads / 64) {
    const uint16_t ent = sh.lng[r];
    const bool done = (ent & 0x8000) != 0;
    const int32_t off = sh.cand[ent & 0x7fff];
    const int32_t i = v0 + off;
    const int32_t beg0 = a.colptr[i], end = a.colptr[i + 1];
    const int32_t beg = beg0 + a.mid;
    int32_t hit = -1;
    unsigned long long n = 0;
    for (int32_t p = beg; p < end; p += 64) {
      const int32_t q = p + lane();
      int32_t jj = 0;
      bool h = false;
      if (q < end) {
        jj = a.rowind[q];
        h = get_bit(a.x, jj) != 0;
      }
      const uint64_t bal = __ballot(h);
      if (EE) {
        if (bal) {
          const int first = __ffsll((unsigned long long)bal) - 1;
          n += uint64_t(first + 1);
          hit = __shfl(jj, first, 64);
          break;
        }
        n += uint64_t(min(64, end - p));
      } else {
        n += uint64_t(min(64, end - p));
        if (bal && hit < 0 && !done) {
          const int first = __ffsll((unsigned long long)bal) - 1;
          hit = __shfl(jj, first, 64);
        }
      }
    }
    if (lane() == 0) {
      checks += n;
      if (hit >= 0) record(off, hit);
    }
  }
  __syncthreads();

  unsigned long long nfound = 0, nout = 0, nheavy = 0;
  for (int lw = tid; lw < kPullTileWords; lw += kThreads) {
    const int32_t w = w0 + lw;
    if (w < a.nwords) {
      const uint32_t f = sh.found[lw];
      const uint32_t o = ((a.out_base ? a.out_base[w] : 0u) | f) & valid_bits(w, a.V);
      a.out[w] = o;
      if (a.found_out) a.found_out[w] = f;
      nfound += __popc(f);
      nout += a.count_out ? __popc(o) : 0;
      if (a.heavy && f) nheavy += __popc(f & a.heavy[w]);
    }
  }
  unsigned long long v[4] = {nfound, nout, checks, nheavy};
  block_sum4(v);
  if (tid == 0) {
    stripe_add(a.slot, v[0], v[1], v[2], 0, 0);
    // how a push over these results could share out its work (see bitmap_expand_body)
    const uint32_t tm = v[3] ? 0xffffffffu : uint32_t(v[0]);
    if (a.heavy && tm) atomicMax(&a.slot->s[blockIdx.x % kStripes].tilemax, tm);
  }
}

// ----------------------------------------------------- BFS level kernels
// Algorithm 1 initialisation: depth/parent unreached except the source,
// visited = {s}, frontier list = [s] (and frontier bitmap = {s} when the
// mode keeps one); clears the counters and scan descriptors and writes the
// state entering level 0.
__global__ __launch_bounds__(kThreads) void k_bfs_init(BfsArgs a, int32_t source, int32_t dir0,
                                                       int64_t nflags) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int32_t V = a.V;
  // 16-byte stores when both outputs allow them
  const bool vec = (reinterpret_cast<uintptr_t>(a.depth) % 16 == 0) &&
                   (!a.parent || reinterpret_cast<uintptr_t>(a.parent) % 16 == 0);
  const int64_t nvec = vec ? V / 4 : 0;
  int4* d4 = reinterpret_cast<int4*>(a.depth);
  int4* p4 = reinterpret_cast<int4*>(a.parent);
  for (int64_t i = t0; i < nvec; i += stride) {
    const int64_t b = i * 4;
    int4 d = make_int4(-1, -1, -1, -1), p = d;
    if (source >= b && source < b + 4) {
      const int k = int(source - b);
      if (k == 0) { d.x = 0; p.x = source; }
      if (k == 1) { d.y = 0; p.y = source; }
      if (k == 2) { d.z = 0; p.z = source; }
      if (k == 3) { d.w = 0; p.w = source; }
    }
    d4[i] = d;
    if (a.parent) p4[i] = p;
  }
  for (int64_t i = nvec * 4 + t0; i < V; i += stride) {
    a.depth[i] = (i == source) ? 0 : -1;
    if (a.parent) a.parent[i] = (i == source) ? source : -1;
  }
  const uint32_t sbit = 1u << (source & 31);
  for (int64_t w = t0; w < a.nwords; w += stride) {
    const uint32_t v = (w == (source >> 5)) ? sbit : 0u;
    a.vis[0][w] = v;
    if (a.need_F) a.F[0][w] = v;
  }
  for (int64_t k = t0; k < nflags; k += stride) {
    a.flagsA[k] = 0;
    a.flagsB[k] = 0;
  }
  if (blockIdx.x == 0) {
    Ctrl* c = a.ctrl;
    for (int k = threadIdx.x; k < kSlots * kStripes; k += blockDim.x)
      zero_stripe(c->slot[k / kStripes].s[k % kStripes]);
    if (threadIdx.x < kBarGroups) c->bar.group[threadIdx.x].n = 0;
    if (threadIdx.x == 0) {
      c->bar.top.n = 0;
      c->bar.gen = 0;
      c->bar.abort = 0;
      c->bar.t_end = 0;
      a.Q[0][0] = source;
      c->ticket[0] = 0;
      c->ticket[1] = 0;
      c->mf32 = 0;
      c->nf32 = 0;
      c->src_outdeg = a.rowptr[source + 1] - a.rowptr[source];
      c->src_indeg = a.colptr[source + 1] - a.colptr[source];
      for (int s = 0; s < kSlots; ++s) {
        c->qcount[s] = 0;
        c->mf[s] = 0;
      }
      LevelState st;
      st.dir = dir0;
      st.done = 0;
      st.list_valid = 1;
      st.vis_idx = 0;
      st.nf = 1;
      st.levels = 0;
      st.level = 0;
      st.m_u = a.nnz - c->src_indeg;
      st.active = 0;
      st.local = (a.local_push && dir0 == 0 &&
                  local_fits(1, c->src_outdeg, c->src_outdeg, main_blocks(a.nwords), a.sched.local_unit,
                             a.sched.local_chunks)) ? 1 : 0;
      st.share = local_share(1, c->src_outdeg, c->src_outdeg, main_blocks(a.nwords), a.sched.local_unit);
      st.phase = (dir0 == 0 && !st.local) ? kPhaseScan : kPhaseWhole;
      c->ring[0] = st;
    }
  }
}

// First kernel of level L: decide the level (device-side), publish state
// and the previous level's record, reset the next level's counters, and for a
// push level build the frontier list with its degree prefix.
__global__ __launch_bounds__(kThreads) void k_level_prep(BfsArgs a, int32_t L, int32_t forced) {
  Ctrl* c = a.ctrl;
  LevelTotals tot;
  LevelState prev;
  const LevelState st = level_state(a, L, forced, &tot, &prev);
  publish_level(c, L, st, prev, tot);
  if (st.done) return;
  if (st.dir != 0) return;
  uint32_t* mf_out = &c->mf[L % kSlots];
  if (a.need_F) {  // winners of this push level will be set in F[(L+1)%2]
    uint32_t* fn = a.F[(L + 1) % 2];
    for (int32_t w = blockIdx.x * kThreads + threadIdx.x; w < a.nwords; w += gridDim.x * kThreads) fn[w] = 0;
  }
  if (st.local) return;  // no scan: the expansion balances its load itself
  if (st.list_valid) {
    scan_list(a.Q[L % 2], st.nf, a.rowptr, a.S, a.R, a.chunk_first, a.flagsA, uint32_t(2 * L + 1),
              &c->ticket[L % 2], mf_out);
  } else {
    ScanBitsArgs sb{};
    if (a.reuse) {  // discovered at the last pull = new visited AND NOT old visited
      sb.a = a.vis[st.vis_idx];
      sb.b_not = a.vis[st.vis_idx ^ 1];
    } else {
      sb.a = a.F[L % 2];
      sb.b_not = nullptr;
    }
    sb.nwords = a.nwords;
    sb.V = a.V;
    sb.rowptr = a.rowptr;
    sb.Qout = a.Q[L % 2];
    sb.S = a.S;
    sb.R = a.R;
    sb.chunk_first = a.chunk_first;
    sb.flagsA = a.flagsA;
    sb.flagsB = a.flagsB;
    sb.epochA = uint32_t(2 * L + 1);
    sb.epochB = uint32_t(2 * L + 2);
    sb.ticket = &c->ticket[L % 2];
    sb.nf_out = &c->nf32;
    sb.mf_out = mf_out;
    // edge-count rule: m_u afresh, since the pulls before did not track it
    sb.mu_slot = a.edge_rule ? &c->slot[L % kSlots] : nullptr;
    sb.unv_nz = a.nz_in;
    sb.unv_vis = a.vis[st.vis_idx];
    sb.colptr = a.colptr;
    scan_bits(sb);
  }
}

union LevelShared {
  ExpandShared e;
  LocalShared l;
  PullShared p;
};

// ------------------------------------------------- single-source step loop
// One launch per step: a level is one step (a pull, or a push that shares
// out its own work), or two when its push needs the global degree scan (the
// scan step, then the expansion step). Every block derives the step's state
// from the state the previous step published and the counters it left (one
// round trip), so no kernel of its own decides the level. The counters of
// step s gather in slot s % kSlots; step s clears slot (s + 2) % kSlots, which
// nothing reads or writes until step s + 2.

__device__ __forceinline__ LevelState step_state(const BfsArgs& a, int32_t s, LevelTotals* tot, LevelState* prev_out,
                                 bool* new_level) {
  const Ctrl* c = a.ctrl;
  *new_level = false;
  *tot = LevelTotals{0, 0, 0, 0, 0, 0};
  if (s == 0) {  // level 0 as the init kernel left it
    const LevelState st = c->ring[0];
    *prev_out = st;
    return st;
  }
  const StripeLanes x = load_stripes(c->slot[(s - 1) % kSlots]);
  const LevelState prev = c->ring[(s - 1) % kRing];
  stripes_needed(x);
  *prev_out = prev;
  if (prev.done) return prev;  // past the end
  if (prev.phase == kPhaseScan) {  // the expansion the scan step prepared
    LevelState st = prev;
    st.phase = kPhaseExpand;
    return st;
  }
  const int32_t L = prev.level + 1;
  const int32_t forced = L < a.n_forced ? int32_t(c->forced[L]) : -1;
  *new_level = true;
  return next_state(a, L, forced, prev, x, (s - 1) % kSlots, tot);
}

// The last step of a batch writes the batch's report itself (block 0, right
// after publishing): the states the batch's steps published (its own from
// registers), the records of the levels complete by now (the one it has just
// written from registers too), then the sequence number with a system-scope
// release. When the traversal is over this step has no work of its own, so
// the report lands after every kernel of the traversal has finished.
// n_steps: steps the report covers (the persistent loop reports the whole launch's range when
// the traversal ends early, the states past the end being copies of the final one).
__device__ __forceinline__ void step_report(const Ctrl* c, const StepReportArgs& rp, int32_t s,
                                            const LevelState& st, const LevelState& prev,
                                            const LevelTotals& tot, bool new_level, int32_t error,
                                            int32_t n_steps = -1) {
  HostReport* host = rp.host;
  const int32_t n = n_steps > 0 ? n_steps : s - rp.s_first + 1;
  for (int k = threadIdx.x; k < n - 1; k += blockDim.x) host->steps[k] = c->ring[(rp.s_first + k) % kRing];
  const int32_t upto = st.done ? st.levels : st.level;  // records exist for levels < upto
  const int32_t nrec = max(0, min(upto - rp.rec_first, kMaxBatch));
  for (int k = threadIdx.x; k < nrec; k += blockDim.x) {
    const int32_t l = rp.rec_first + k;
    host->rec[k] = (new_level && l == st.level - 1) ? step_record(c, s, prev, tot) : c->rec[l % kRing];
  }
  if (threadIdx.x == 0) {
    host->steps[n - 1] = st;
    host->end = st;
    host->nrec = nrec;
    host->error = error;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    __hip_atomic_store(&host->seq, rp.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// The scan step of a push level: its frontier list with the degree prefix
// and chunk table (Section 6.2), from the list the push before left or from
// the bits the pull before found. Its m_f goes where the expansion step reads it.
__device__ __forceinline__ void step_scan(const BfsArgs& a, const LevelState& st, int32_t s) {
  Ctrl* c = a.ctrl;
  const int32_t L = st.level;
  uint32_t* mf_out = &c->mf[(s + 1) % kSlots];
  if (a.need_F) {  // winners of this push level will be set in F[(L+1)%2]
    uint32_t* fn = a.F[(L + 1) % 2];
    for (int32_t w = blockIdx.x * kThreads + threadIdx.x; w < a.nwords; w += gridDim.x * kThreads) fn[w] = 0;
  }
  if (st.list_valid) {
    scan_list(a.Q[L % 2], st.nf, a.rowptr, a.S, a.R, a.chunk_first, a.flagsA, uint32_t(2 * s + 1),
              &c->ticket[s % 2], mf_out);
  } else {
    ScanBitsArgs sb{};
    if (a.reuse) {  // discovered at the last pull = new visited AND NOT old visited
      sb.a = a.vis[st.vis_idx];
      sb.b_not = a.vis[st.vis_idx ^ 1];
    } else {
      sb.a = a.F[L % 2];
      sb.b_not = nullptr;
    }
    sb.nwords = a.nwords;
    sb.V = a.V;
    sb.rowptr = a.rowptr;
    sb.Qout = a.Q[L % 2];
    sb.S = a.S;
    sb.R = a.R;
    sb.chunk_first = a.chunk_first;
    sb.flagsA = a.flagsA;
    sb.flagsB = a.flagsB;
    sb.epochA = uint32_t(2 * s + 1);
    sb.epochB = uint32_t(2 * s + 2);
    sb.ticket = &c->ticket[s % 2];
    sb.nf_out = &c->nf32;
    sb.mf_out = mf_out;
    // edge-count rule: m_u afresh, since the pulls before did not track it; the
    // expansion step's slot, which the next level reads
    sb.mu_slot = a.edge_rule ? &c->slot[(s + 1) % kSlots] : nullptr;
    sb.unv_nz = a.nz_in;
    sb.unv_vis = a.vis[st.vis_idx];
    sb.colptr = a.colptr;
    scan_bits(sb);
  }
}

// The argument block of step s's push (level st.level).
__device__ __forceinline__ ExpandArgs step_expand_args(const BfsArgs& a, const LevelState& st, int32_t s,
                                                       uint32_t m, const uint32_t* front,
                                                       const uint32_t* vis_before, LevelSlot* mu_slot) {
  Ctrl* c = a.ctrl;
  const int32_t L = st.level;
  ExpandArgs e;
  e.Q = a.Q[L % 2];
  e.nf = st.nf;
  e.S = a.S;
  e.R = a.R;
  e.chunk_first = a.chunk_first;
  e.colind = a.colind;
  e.m = m;
  e.claim = a.vis[st.vis_idx];
  e.mask = nullptr;
  e.complement = 0;
  e.depth = a.depth;
  e.parent = a.parent;
  e.level = L;
  e.Qout = a.Q[(L + 1) % 2];
  e.qcount = &c->qcount[s % kSlots];
  e.found_out = a.need_F ? a.F[(L + 1) % 2] : nullptr;
  e.rowptr = a.rowptr;
  // winners' out-degrees: the next level's m_f (edge-count rule) and its largest degree
  // (whether it can skip the scan; known for all levels when the whole graph has low degree)
  e.out_rowptr = (a.edge_rule || !a.low_degree) ? a.rowptr : nullptr;
  e.in_colptr = a.edge_rule ? a.colptr : nullptr;
  e.slot = &c->slot[s % kSlots];
  e.share = st.share;
  e.unit = a.sched.local_unit;
  e.front = front;
  e.vis_before = vis_before;
  e.nz = a.nz_in;
  e.mu_slot = mu_slot;
  return e;
}

// The work of step s (state st) that virtual block bid of nblk does: the step's launch has
// nblk = main_blocks(nwords) blocks; the persistent loop runs several virtual blocks per block.
// The scan step's tiles go by ticket, so there every block calls it once (bid = blockIdx.x).
template <bool EE>
__device__ __forceinline__ void step_body(const BfsArgs& a, const LevelState& st, int32_t s, LevelShared& sh,
                                          int32_t bid, int32_t nblk) {
  Ctrl* c = a.ctrl;
  if (st.phase == kPhaseScan) {
    step_scan(a, st, s);
    return;
  }
  const int32_t L = st.level;
  LevelSlot* slot = &c->slot[s % kSlots];
  if (st.dir == 0) {
    // each push body gets its own argument block, built whole, so the compiler keeps it in
    // registers (one block modified across branches went to scratch memory)
    if (st.phase == kPhaseExpand) {
      const ExpandArgs e = step_expand_args(a, st, s, c->mf[s % kSlots], nullptr, nullptr, nullptr);
      expand_body(e, sh.e, uint32_t(bid), uint32_t(nblk));
    } else if (st.local == 2) {  // frontier = what the pull before found (written whole, untouched here)
      const ExpandArgs e = step_expand_args(a, st, s, 0u, a.F[L % 2], a.vis[st.vis_idx ^ 1],
                                            a.edge_rule ? slot : nullptr);  // m_u afresh: pulls skip it
      bitmap_expand_body(e, a.nwords, a.V, sh.l, bid, nblk);
    } else {
      const ExpandArgs e = step_expand_args(a, st, s, 0u, nullptr, nullptr, nullptr);
      local_expand_body(e, sh.l, bid, nblk);
    }
  } else {
    const int32_t tiles = (a.nwords + kPullTileWords - 1) / kPullTileWords;
    if (bid >= tiles) return;
    PullArgs p;
    p.V = a.V;
    p.nwords = a.nwords;
    p.colptr = a.colptr;
    p.rowind = a.rowind;
    p.slab = a.slab;
    p.head = a.head;
    p.x = a.reuse ? a.vis[st.vis_idx] : a.F[L % 2];  // operand reuse: A^T v .* not(v) (Section 5.4)
    p.mask = a.vis[st.vis_idx];
    p.complement = 1;
    p.mask_after = a.mask_after;
    p.nz = a.nz_in;
    p.out_base = a.vis[st.vis_idx];
    p.out = a.vis[st.vis_idx ^ 1];
    p.found_out = (a.need_F || a.local_push) ? a.F[(L + 1) % 2] : nullptr;  // a bitmap push may read it
    p.heavy = a.heavy;
    p.depth = a.depth;
    p.parent = a.parent;
    p.level = L;
    p.early_exit = EE;
    p.mid = a.sched.pull_mid;
    p.count_out = 0;
    p.slot = slot;
    pull_body<EE>(p, bid, sh.p);
  }
}

template <bool EE>
__global__ __launch_bounds__(kThreads) void k_step(BfsArgs a, int32_t s, StepReportArgs rp) {
  __shared__ LevelShared sh;
  LevelTotals tot;
  LevelState prev;
  bool new_level;
  const LevelState st = step_state(a, s, &tot, &prev, &new_level);
  if (blockIdx.x == 0) {
    publish_step(a.ctrl, s, st, prev, tot, new_level);
    if (rp.host) step_report(a.ctrl, rp, s, st, prev, tot, new_level, 0);
  }
  if (st.done) return;
  step_body<EE>(a, st, s, sh, int32_t(blockIdx.x), int32_t(gridDim.x));
}


// The persistent step loop: steps s_first .. s_first + n - 1 in one launch of
// co-resident blocks, a grid barrier between consecutive steps in place of a
// kernel boundary. Every block derives each step's state as k_step does;
// block 0 publishes it (with its start time when timing) and, at the launch's
// last step or when the traversal is over, writes the batch's report. The
// report says whether a barrier wait gave up; then every block leaves.
template <bool EE>
__global__ __launch_bounds__(kThreads) void k_steps(BfsArgs a, int32_t s_first, int32_t n, uint32_t spin_limit,
                                                    int32_t timing, StepReportArgs rp) {
  __shared__ LevelShared sh;
  __shared__ uint32_t s_gen;
  GridBar* bar = &a.ctrl->bar;
  if (threadIdx.x == 0)  // no barrier of this traversal is in progress between launches
    s_gen = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const uint32_t gen0 = s_gen;
  const int32_t nvb = int32_t(main_blocks(a.nwords));
  for (int32_t k = 0; k < n; ++k) {
    const int32_t s = s_first + k;
    LevelTotals tot;
    LevelState prev;
    bool new_level;
    LevelState st = step_state(a, s, &tot, &prev, &new_level);
    if (blockIdx.x == 0) {
      if (timing) st.t0 = wall_clock64();
      publish_step(a.ctrl, s, st, prev, tot, new_level);
      // over early: the launch's remaining steps read as the final state, as steps enqueued
      // past the end publish it in the one-launch-per-step loop
      if (st.done)
        for (int32_t j = 1 + int32_t(threadIdx.x); j < n - k; j += kThreads) a.ctrl->ring[(s + j) % kRing] = st;
      if (rp.host && (k == n - 1 || st.done)) {
        __syncthreads();
        step_report(a.ctrl, rp, s, st, prev, tot, new_level, 0, n);
      }
    }
    if (st.done) break;
    for (int32_t vb = int32_t(blockIdx.x); vb < nvb; vb += int32_t(gridDim.x)) {
      __syncthreads();  // the previous virtual block's LDS readers are done
      step_body<EE>(a, st, s, sh, st.phase == kPhaseScan ? int32_t(blockIdx.x) : vb, nvb);
      if (st.phase == kPhaseScan) break;  // tiles by ticket: one call per block
    }
    if (k == n - 1) break;  // the kernel boundary ends the last step
    if (!grid_barrier(bar, gen0 + uint32_t(k) + 1u, spin_limit)) {
      if (blockIdx.x == 0 && rp.host) step_report(a.ctrl, rp, s, st, prev, tot, new_level, 1);
      break;
    }
  }
  if (timing) {
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_max(&bar->t_end, (unsigned long long)wall_clock64(), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Copies the states the steps s_first .. s_first + n - 1 published, and the
// records of the levels that are complete after them from rec_first on, into
// pinned host memory; then publishes `seq` with a system-scope release.
__global__ void k_step_report(const Ctrl* c, int32_t s_first, int32_t n, int32_t rec_first, HostReport* host,
                              uint32_t seq) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) host->steps[k] = c->ring[(s_first + k) % kRing];
  const LevelState end = c->ring[(s_first + n - 1) % kRing];
  const int32_t upto = end.done ? end.levels : end.level;  // records exist for levels < upto
  const int32_t nrec = max(0, min(upto - rec_first, kMaxBatch));
  for (int k = threadIdx.x; k < nrec; k += blockDim.x) host->rec[k] = c->rec[(rec_first + k) % kRing];
  if (threadIdx.x == 0) {
    host->end = end;
    host->nrec = nrec;
    host->error = int32_t(c->bar.abort != 0);
    host->t_end = c->bar.t_end;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    __hip_atomic_store(&host->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// ------------------------------------------------------- mxv kernels
__global__ __launch_bounds__(kThreads) void k_scan_bits(ScanBitsArgs a) { scan_bits(a); }

__global__ __launch_bounds__(kThreads) void k_expand(ExpandArgs a, const uint32_t* m_dev,
                                                     const uint32_t* nf_dev) {
  __shared__ ExpandShared sh;
  if (m_dev) a.m = *m_dev;
  if (nf_dev) a.nf = int32_t(*nf_dev);
  expand_body(a, sh, blockIdx.x, gridDim.x);
}

template <bool EE>
__global__ __launch_bounds__(kThreads) void k_pull(PullArgs a) {
  __shared__ PullShared sh;
  pull_body<EE>(a, int32_t(blockIdx.x), sh);
}

__global__ __launch_bounds__(kThreads) void k_ctrl_init(Ctrl* ctrl, uint64_t* flags,
                                                        int64_t nflags) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t k = t0; k < nflags; k += stride) flags[k] = 0;
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < kSlots * kStripes; k += blockDim.x)
      zero_stripe(ctrl->slot[k / kStripes].s[k % kStripes]);
    if (threadIdx.x == 0) {
      ctrl->ticket[0] = 0;
      ctrl->ticket[1] = 0;
      ctrl->mf32 = 0;
      ctrl->nf32 = 0;
      ctrl->src_outdeg = 0;
      ctrl->src_indeg = 0;
      for (int s = 0; s < kSlots; ++s) {
        ctrl->qcount[s] = 0;
        ctrl->mf[s] = 0;
      }
    }
  }
}

// --------------------------------------------------------------- helpers
__global__ __launch_bounds__(kThreads) void k_fill(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// SPARSE2DENSE: scatter an index list into a (zeroed) bit vector.
__global__ __launch_bounds__(kThreads) void k_s2d(const int32_t* idx, int32_t n, int32_t V,
                                                  uint32_t* bits) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += stride) {
    const int32_t v = idx[k];
    if (v >= 0 && v < V) atomicOr(&bits[v >> 5], 1u << (v & 31));
  }
}

// y = (accum ? y : 0) | r, and the popcount of the result.
__global__ __launch_bounds__(kThreads) void k_mxv_finalize(uint32_t* y, const uint32_t* r,
                                                           int32_t nwords, int32_t V, int accum,
                                                           LevelSlot* slot) {
  const int32_t w = blockIdx.x * kThreads + threadIdx.x;
  unsigned long long nres = 0, nout = 0;
  if (w < nwords) {
    const uint32_t vb = valid_bits(w, V);
    const uint32_t rr = r[w] & vb;
    const uint32_t o = ((accum ? y[w] : 0u) | rr) & vb;
    y[w] = o;
    nres = __popc(rr);
    nout = __popc(o);
  }
  unsigned long long v[4] = {nres, nout, 0, 0};
  block_sum4(v);
  if (threadIdx.x == 0) stripe_add(slot, v[0], v[1], 0, 0, 0);
}

// Rows with a non-empty adjacency list, as a bit vector.
__global__ __launch_bounds__(kThreads) void k_nz_bits(const int32_t* ptr, int32_t V, uint32_t* bits,
                                                      int32_t min_len) {
  const int32_t w = blockIdx.x * kThreads + threadIdx.x;
  const int32_t nwords = (V + 31) / 32;
  if (w >= nwords) return;
  uint32_t b = 0;
  for (int k = 0; k < 32; ++k) {
    const int32_t i = w * 32 + k;
    if (i < V && ptr[i + 1] - ptr[i] > min_len) b |= 1u << k;
  }
  bits[w] = b;
}

// First entry of every CSC column (-1 for an empty column): the pull's
// first check reads it densely.
__global__ __launch_bounds__(kThreads) void k_slab(const int32_t* ptr, const int32_t* ind, int32_t V,
                                                   int4* slab, int32_t* head) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < V; i += stride) {
    const int32_t b = ptr[i], d = ptr[i + 1] - b;
    slab[i] = make_int4(d > 0 ? ind[b] : -1, d > 1 ? ind[b + 1] : -1, d > 2 ? ind[b + 2] : -1,
                        d > 3 ? ind[b + 3] : -1);
    // the head: the first entry, complemented when more follow (0 for an empty
    // column, which the pull never lists)
    head[i] = d == 0 ? 0 : (d == 1 ? ind[b] : ~ind[b]);
  }
}

// Largest row length of a CSR offset array (one atomic per block).
__global__ __launch_bounds__(kThreads) void k_max_degree(const int32_t* ptr, int32_t V, uint32_t* out) {
  uint32_t m = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < V; i += stride)
    m = max(m, uint32_t(ptr[i + 1] - ptr[i]));
  m = block_max32(m);
  if (threadIdx.x == 0 && m) atomicMax(out, m);
}

// Out-degree sum over the reached vertices (the Graph500 edge count before
// halving): a grid stride over depth, one stripe atomic per block.
__global__ __launch_bounds__(kThreads) void k_reached_degree(const int32_t* ptr, const int32_t* depth,
                                                             int32_t V, LevelSlot* slot) {
  unsigned long long sum = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < V; i += stride)
    if (depth[i] >= 0) sum += uint64_t(ptr[i + 1] - ptr[i]);
  unsigned long long v[4] = {sum, 0, 0, 0};
  block_sum4(v);
  if (threadIdx.x == 0 && v[0]) atomicAdd(&slot->s[blockIdx.x % kStripes].edges, v[0]);
}

__global__ void k_zero_slot(LevelSlot* slot) {
  for (int k = threadIdx.x; k < kStripes; k += blockDim.x) zero_stripe(slot->s[k]);
}

__global__ __launch_bounds__(kThreads) void k_check_offsets(const int32_t* ptr, int32_t V, int64_t nnz,
                                                            int32_t* err) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < V; i += stride) {
    if (ptr[i + 1] < ptr[i]) atomicOr(err, 1);
    if (i == 0 && ptr[0] != 0) atomicOr(err, 2);
    if (i == V - 1 && int64_t(ptr[V]) != nnz) atomicOr(err, 4);
  }
}

__global__ __launch_bounds__(kThreads) void k_check_indices(const int32_t* idx, int64_t nnz, int32_t V,
                                                            int32_t* err) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nnz; i += stride)
    if (idx[i] < 0 || idx[i] >= V) atomicOr(err, 8);
}

inline unsigned grid_for(int64_t n, int64_t per_block, int64_t cap = 65535) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

}  // namespace

hipError_t launch_bfs_init(hipStream_t s, const BfsArgs& a, int32_t source, int32_t dir0, hipEvent_t t0,
                          hipEvent_t t1) {
  const int64_t nflags = flag_entries(a.V);
  const int64_t n = std::max<int64_t>(std::max<int64_t>(a.V / 4 + 4, a.nwords), nflags);
  return launch_k(k_bfs_init, dim3(grid_for(n, kThreads, 8192)), s, t0, t1, a, source, dir0, nflags);
}

hipError_t launch_level_prep(hipStream_t s, const BfsArgs& a, int32_t level, int32_t forced_dir,
                            hipEvent_t t0, hipEvent_t t1) {
  return launch_k(k_level_prep, dim3(unsigned(scan_grid(a.V))), s, t0, t1, a, level, forced_dir);
}

hipError_t launch_step(hipStream_t s, const BfsArgs& a, int32_t step, hipEvent_t t0, hipEvent_t t1,
                       const StepReportArgs* rp) {
  const dim3 g(unsigned(main_blocks(a.nwords)));
  const StepReportArgs r = rp ? *rp : StepReportArgs{nullptr, 0u, 0, 0};
  if (a.early_exit) return launch_k(k_step<true>, g, s, t0, t1, a, step, r);
  return launch_k(k_step<false>, g, s, t0, t1, a, step, r);
}

hipError_t launch_steps(hipStream_t s, const BfsArgs& a, int32_t s_first, int32_t n, int32_t blocks,
                        uint32_t spin_limit, bool timing, const StepReportArgs& rp, hipEvent_t t0, hipEvent_t t1) {
  const dim3 g = dim3(static_cast<unsigned>(blocks));
  const StepReportArgs r = rp;
  const int32_t tm = timing ? 1 : 0;
  if (a.early_exit) return launch_k(k_steps<true>, g, s, t0, t1, a, s_first, n, spin_limit, tm, r);
  return launch_k(k_steps<false>, g, s, t0, t1, a, s_first, n, spin_limit, tm, r);
}

hipError_t persistent_capacity(int32_t* blocks) {
  int dev = 0, cus = 0, per_t = 0, per_f = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_t, k_steps<true>, kThreads, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_f, k_steps<false>, kThreads, 0);
  if (e != hipSuccess) return e;
  *blocks = cus * std::min(per_t, per_f);
  return hipSuccess;
}

hipError_t launch_step_report(hipStream_t s, const Ctrl* ctrl, int32_t s_first, int32_t n, int32_t rec_first,
                              HostReport* host, uint32_t seq) {
  hipLaunchKernelGGL(k_step_report, dim3(1), dim3(64), 0, s, ctrl, s_first, n, rec_first, host, seq);
  return hipGetLastError();
}

hipError_t launch_ctrl_init(hipStream_t s, Ctrl* ctrl, uint64_t* flags, int64_t nflags) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(grid_for(nflags, kThreads, 1024)), dim3(kThreads), 0, s,
                     ctrl, flags, nflags);
  return hipGetLastError();
}

hipError_t launch_scan_bits(hipStream_t s, const ScanBitsArgs& a) {
  hipLaunchKernelGGL(k_scan_bits, dim3(unsigned(scan_grid(a.V))), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_expand(hipStream_t s, const ExpandArgs& a, const uint32_t* m_dev,
                         const uint32_t* nf_dev) {
  hipLaunchKernelGGL(k_expand, dim3(unsigned(kExpandBlocks)), dim3(kThreads), 0, s, a, m_dev,
                     nf_dev);
  return hipGetLastError();
}

hipError_t launch_pull(hipStream_t s, const PullArgs& a) {
  const unsigned g = unsigned(pull_tiles(a.nwords));
  if (a.early_exit)
    hipLaunchKernelGGL(k_pull<true>, dim3(g), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_pull<false>, dim3(g), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill(hipStream_t s, uint32_t* p, int64_t n, uint32_t v) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kThreads * 4, 4096)), dim3(kThreads), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_s2d(hipStream_t s, const int32_t* idx, int32_t n, int32_t V, uint32_t* bits) {
  hipLaunchKernelGGL(k_s2d, dim3(grid_for(n, kThreads * 4, 4096)), dim3(kThreads), 0, s, idx, n, V,
                     bits);
  return hipGetLastError();
}

hipError_t launch_mxv_finalize(hipStream_t s, uint32_t* y, const uint32_t* r, int32_t nwords,
                               int32_t V, int accum, LevelSlot* slot) {
  hipLaunchKernelGGL(k_mxv_finalize, dim3(grid_for(nwords, kThreads, 1u << 30)), dim3(kThreads),
                     0, s, y, r, nwords, V, accum, slot);
  return hipGetLastError();
}

hipError_t launch_nz_bits(hipStream_t s, const int32_t* ptr, int32_t V, uint32_t* bits, int32_t min_len) {
  hipLaunchKernelGGL(k_nz_bits, dim3(grid_for(words_of(V), kThreads, 1u << 30)), dim3(kThreads),
                     0, s, ptr, V, bits, min_len);
  return hipGetLastError();
}

hipError_t launch_slab(hipStream_t s, const int32_t* ptr, const int32_t* ind, int32_t V, int4* slab,
                       int32_t* head) {
  hipLaunchKernelGGL(k_slab, dim3(grid_for(V, kThreads, 8192)), dim3(kThreads), 0, s, ptr, ind, V,
                     slab, head);
  return hipGetLastError();
}

hipError_t launch_max_degree(hipStream_t s, const int32_t* ptr, int32_t V, uint32_t* out) {
  hipLaunchKernelGGL(k_max_degree, dim3(grid_for(V, kThreads, 1024)), dim3(kThreads), 0, s, ptr, V, out);
  return hipGetLastError();
}

hipError_t launch_reached_degree(hipStream_t s, const int32_t* ptr, const int32_t* depth, int32_t V,
                                 LevelSlot* slot) {
  hipLaunchKernelGGL(k_zero_slot, dim3(1), dim3(64), 0, s, slot);
  hipLaunchKernelGGL(k_reached_degree, dim3(grid_for(V, kThreads * 8, 512)), dim3(kThreads), 0, s, ptr,
                     depth, V, slot);
  return hipGetLastError();
}


hipError_t launch_check_offsets(hipStream_t s, const int32_t* ptr, int32_t V, int64_t nnz,
                                int32_t* err) {
  hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(V, kThreads, 4096)), dim3(kThreads), 0, s,
                     ptr, V, nnz, err);
  return hipGetLastError();
}

hipError_t launch_check_indices(hipStream_t s, const int32_t* idx, int64_t nnz, int32_t V,
                                int32_t* err) {
  hipLaunchKernelGGL(k_check_indices, dim3(grid_for(nnz, kThreads, 4096)), dim3(kThreads), 0, s,
                     idx, nnz, V, err);
  return hipGetLastError();
}

}  // namespace dobfs
