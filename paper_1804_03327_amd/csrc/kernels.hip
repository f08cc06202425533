// HIP kernels of libdobfs for gfx950 (CDNA4, wave64).
//
// One BFS level is the Boolean masked matvec f' = A^T f .* not(v)
// (Algorithm 1). Push computes it column by column from the frontier list
// (Equation 5, Section 6.2); pull computes it row by row over the rows the
// mask lets through, stopping at the first hit (Equation 4, Algorithm 2,
// Sections 5.2-5.4). Everything is integer / bitwise: no MFMA.
//
// Memory layout (HBM): CSR(A) and CSC(A) int32 arrays; bit vectors as uint32
// words (bit i = word i>>5, bit i&31); frontier lists as int32.
//
// Rates that shaped these kernels (measured on MI355X): random 4-byte loads
// from a 512 KiB L2-resident bitmap ~270 G/s; atomics on distinct words
// ~27 G/s; atomics on one address ~0.09 G/s (serialized); streaming reads
// ~6.4 TB/s. So the bitmaps are read with plain loads first, per-level
// counters are striped over kStripes lines, and list appends are batched per
// block in LDS.

#include "dobfs_internal.h"

#include <algorithm>

namespace dobfs {
namespace {

constexpr uint32_t kStatusAgg = 1, kStatusPrefix = 2;

__device__ __forceinline__ int lane() { return int(__lane_id()); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane()) - 1ull; }

__device__ __forceinline__ uint32_t get_bit(const uint32_t* b, int32_t i) {
  return (b[i >> 5] >> (i & 31)) & 1u;
}

// Bits of word w that are inside [0, V).
__device__ __forceinline__ uint32_t valid_bits(int32_t w, int32_t V) {
  const int32_t lo = w * 32;
  if (lo + 32 <= V) return 0xffffffffu;
  if (lo >= V) return 0u;
  return (1u << (V - lo)) - 1u;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d, 64);
    if (lane() >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Exclusive scan over the 256 threads of a block; *total gets the block sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t s_w[kThreads / 64];
  const int wv = threadIdx.x >> 6;
  uint32_t incl = uint32_t(wave_incl_scan(int(v)));
  if (lane() == 63) s_w[wv] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kThreads / 64; ++k) {
    uint32_t t = s_w[k];
    before += (k < wv) ? t : 0u;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// Block-wide sums of four 64-bit values (one barrier pair).
__device__ __forceinline__ void block_sum4(unsigned long long v[4]) {
  __shared__ unsigned long long s_w[4][kThreads / 64];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = wave_sum64(v[k]);
  if (lane() == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s_w[k][threadIdx.x >> 6] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += s_w[k][w];
    v[k] = t;
  }
  __syncthreads();
}

// Adds a block's totals into its stripe of the level slot (thread 0 only).
__device__ __forceinline__ void stripe_add(LevelSlot* slot, unsigned long long count,
                                           unsigned long long aux, unsigned long long edges,
                                           unsigned long long mnew, unsigned long long insub) {
  Stripe* st = &slot->s[blockIdx.x % kStripes];
  if (count) atomicAdd(&st->count, uint32_t(count));
  if (aux) atomicAdd(&st->aux, uint32_t(aux));
  if (edges) atomicAdd(&st->edges, edges);
  if (mnew) atomicAdd(&st->mnew, mnew);
  if (insub) atomicAdd(&st->insub, insub);
}

__device__ __forceinline__ void zero_stripe(Stripe& st) {
  st.count = 0;
  st.aux = 0;
  st.edges = 0;
  st.mnew = 0;
  st.insub = 0;
}

// Zero the counters of the next level (block 0), before any of its kernels runs.
__device__ __forceinline__ void reset_slot(Ctrl* ctrl, LevelSlot* r, int32_t r_level) {
  if (!r || blockIdx.x != 0) return;
  for (int k = threadIdx.x; k < kStripes; k += blockDim.x) zero_stripe(r->s[k]);
  if (threadIdx.x == 0 && ctrl) {
    ctrl->qcount[r_level] = 0;
    ctrl->mf[r_level] = 0;
  }
}

// ---- single-pass tile prefix (decoupled look-back) ----
// Tile descriptors are one 64-bit word: [epoch:30][status:2][value:32], so a
// single atomic store publishes status and value together. Tiles are numbered
// by a ticket taken at block start, so every tile a block waits on belongs to
// a block that is already running and publishes without waiting itself.
__device__ __forceinline__ uint64_t pack_flag(uint32_t epoch, uint32_t status, uint32_t value) {
  return (uint64_t(epoch) << 34) | (uint64_t(status) << 32) | uint64_t(value);
}

__device__ __forceinline__ uint32_t take_ticket(Ctrl* ctrl, unsigned long long base) {
  __shared__ uint32_t s_tile;
  if (threadIdx.x == 0) s_tile = uint32_t(atomicAdd(&ctrl->ticket, 1ull) - base);
  __syncthreads();
  return s_tile;
}

// Returns the sum of all values of tiles before `tile` (called by every thread).
__device__ uint32_t tile_exclusive_prefix(uint64_t* flags, uint32_t tile, uint32_t epoch,
                                          uint32_t aggregate) {
  __shared__ uint32_t s_excl;
  if (threadIdx.x < 64) {
    if (tile == 0) {
      if (lane() == 0) {
        __hip_atomic_store(&flags[0], pack_flag(epoch, kStatusPrefix, aggregate), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        s_excl = 0;
      }
    } else {
      if (lane() == 0)
        __hip_atomic_store(&flags[tile], pack_flag(epoch, kStatusAgg, aggregate), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      uint32_t excl = 0;
      int64_t pos = int64_t(tile) - 1;
      while (true) {
        const int64_t idx = pos - lane();
        uint64_t f = 0;
        uint32_t st = kStatusPrefix;  // lanes before tile 0 never matter: tile 0 is a prefix
        if (idx >= 0) {
          f = __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          st = (uint32_t(f >> 34) == epoch) ? uint32_t(f >> 32) & 3u : 0u;
        }
        while (__any(st == 0)) {
          __builtin_amdgcn_s_sleep(1);
          if (st == 0) {
            f = __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st = (uint32_t(f >> 34) == epoch) ? uint32_t(f >> 32) & 3u : 0u;
          }
        }
        const uint32_t v = (idx >= 0) ? uint32_t(f) : 0u;
        const uint64_t pm = __ballot(st == kStatusPrefix);
        if (pm) {
          const int first = __ffsll((unsigned long long)pm) - 1;
          excl += wave_sum(lane() <= first ? v : 0u);
          break;
        }
        excl += wave_sum(v);
        pos -= 64;
      }
      if (lane() == 0) {
        __hip_atomic_store(&flags[tile], pack_flag(epoch, kStatusPrefix, excl + aggregate),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_excl = excl;
      }
    }
  }
  __syncthreads();
  return s_excl;
}

// ---------------------------------------------------------------- init
// Algorithm 1 initialisation: depth/parent unreached except the source,
// visited = {s}, frontier list = [s]; also clears the control block and the
// scan tile descriptors of this call.
__global__ __launch_bounds__(kThreads) void k_bfs_init(int32_t V, int32_t nwords, int32_t source,
                                                       const int32_t* rowptr, const int32_t* colptr,
                                                       int32_t* depth, int32_t* parent,
                                                       uint32_t* vis, int32_t* Q, Ctrl* ctrl,
                                                       uint64_t* flags, int64_t nflags) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  // 16-byte stores when both outputs allow them
  const bool vec = (reinterpret_cast<uintptr_t>(depth) % 16 == 0) &&
                   (!parent || reinterpret_cast<uintptr_t>(parent) % 16 == 0);
  const int64_t nvec = vec ? V / 4 : 0;
  int4* d4 = reinterpret_cast<int4*>(depth);
  int4* p4 = reinterpret_cast<int4*>(parent);
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
    if (parent) p4[i] = p;
  }
  for (int64_t i = nvec * 4 + t0; i < V; i += stride) {
    depth[i] = (i == source) ? 0 : -1;
    if (parent) parent[i] = (i == source) ? source : -1;
  }
  for (int64_t w = t0; w < nwords; w += stride)
    vis[w] = (w == (source >> 5)) ? (1u << (source & 31)) : 0u;
  for (int64_t k = t0; k < nflags; k += stride) flags[k] = 0;
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < kSlots * kStripes; k += blockDim.x)
      zero_stripe(ctrl->slot[k / kStripes].s[k % kStripes]);
    if (threadIdx.x == 0) {
      Q[0] = source;
      ctrl->ticket = 0;
      ctrl->mf32 = 0;
      ctrl->d2s_count = 0;
      ctrl->src_outdeg = rowptr[source + 1] - rowptr[source];
      ctrl->src_indeg = colptr[source + 1] - colptr[source];
      for (int s = 0; s < kSlots; ++s) {
        ctrl->qcount[s] = 0;
        ctrl->mf[s] = 0;
      }
    }
  }
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
      ctrl->ticket = 0;
      ctrl->mf32 = 0;
      ctrl->d2s_count = 0;
      ctrl->src_outdeg = 0;
      ctrl->src_indeg = 0;
      for (int s = 0; s < kSlots; ++s) {
        ctrl->qcount[s] = 0;
        ctrl->mf[s] = 0;
      }
    }
  }
}

// ----------------------------------------------------------- push: scan
// Out-degree of every frontier vertex and its exclusive prefix sum (the
// "length" and "scan" steps of the column-based matvec, Section 6.2): S[k] is
// where vertex Q[k]'s adjacency starts in the concatenated expansion, R[k] its
// row start in CSR(A). Every vertex whose adjacency segment contains the
// first edge of a kExpandChunk-edge chunk records itself as that chunk's
// first vertex, which is all the expand kernel needs to find its work (the
// load-balanced gather). The last tile stores m_f = nnz(m_f^+).
__global__ __launch_bounds__(kThreads) void k_push_scan(const int32_t* __restrict__ Q, int32_t nf_arg,
                                                        const uint32_t* nf_dev,
                                                        const int32_t* __restrict__ rowptr,
                                                        int32_t* __restrict__ S,
                                                        int32_t* __restrict__ R,
                                                        int32_t* __restrict__ chunk_first,
                                                        Ctrl* ctrl, unsigned long long ticket_base,
                                                        uint32_t epoch, uint64_t* flags,
                                                        int32_t level_slot, LevelSlot* reset,
                                                        int32_t reset_level) {
  reset_slot(ctrl, reset, reset_level);
  const int32_t nf = nf_dev ? int32_t(*nf_dev) : nf_arg;
  const uint32_t tile = take_ticket(ctrl, ticket_base);
  const int64_t first = int64_t(tile) * kScanTile;
  if (first >= nf && tile != 0) return;  // beyond the list: nobody waits for this tile
  const int64_t base = first + int64_t(threadIdx.x) * kScanIPT;
  int32_t deg[kScanIPT], st[kScanIPT];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanIPT; ++k) {
    deg[k] = 0;
    st[k] = 0;
    if (base + k < nf) {
      const int32_t u = Q[base + k];
      const int32_t b = rowptr[u], e = rowptr[u + 1];
      deg[k] = e - b;
      st[k] = b;
      sum += uint32_t(e - b);
    }
  }
  uint32_t agg;
  const uint32_t excl = block_excl_scan(sum, &agg);
  const uint32_t tile_excl = tile_exclusive_prefix(flags, tile, epoch, agg);
  uint32_t run = tile_excl + excl;
#pragma unroll
  for (int k = 0; k < kScanIPT; ++k) {
    if (base + k < nf) {
      S[base + k] = int32_t(run);
      R[base + k] = st[k];
      if (deg[k] > 0) {
        // chunks whose first edge lies in [run, run + deg)
        const uint32_t c0 = (run + kExpandChunk - 1) / kExpandChunk;
        const uint32_t c1 = (run + uint32_t(deg[k]) - 1) / kExpandChunk;
        for (uint32_t c = c0; c <= c1; ++c) chunk_first[c] = int32_t(base + k);
      }
      run += uint32_t(deg[k]);
    }
  }
  const bool last = (nf == 0) ? (tile == 0) : (tile == uint32_t((nf - 1) / kScanTile));
  if (last && threadIdx.x == 0) {
    ctrl->mf32 = tile_excl + agg;
    ctrl->mf[level_slot] = uint64_t(tile_excl + agg);
  }
}

__device__ __forceinline__ int32_t thread_search(const int32_t* S, int32_t lo, int32_t hi, uint32_t e) {
  while (hi - lo > 1) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (uint32_t(S[mid]) <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// --------------------------------------------------------- push: expand
// Load-balanced gather over the concatenated adjacency of the frontier: a
// block takes chunks of kExpandChunk consecutive edges; each edge finds its
// frontier vertex by a search over the scan (the interval-gather step of
// Section 6.2), so supervertices spread over many blocks and adjacent lanes
// read adjacent column indices. Each thread carries kExpandEPT edges at once
// so their loads overlap. The merge + mask filter of the paper's sort-based
// version is one atomicOr per edge whose target still looks unvisited: the
// first setter of a bit owns the vertex (Boolean OR makes any winner exact),
// which both deduplicates and applies the mask not(v). Winners are buffered
// in LDS and appended to the next frontier list with one atomic per flush.
__global__ __launch_bounds__(kThreads) void k_push_expand(ExpandArgs a) {
  __shared__ int32_t sS[kExpandWin], sR[kExpandWin], sQ[kExpandWin];
  __shared__ int32_t s_buf[kExpandBuf];
  __shared__ uint32_t s_nbuf, s_base;
  reset_slot(a.ctrl, a.reset, a.reset_level);
  const int32_t nf = a.nf_dev ? int32_t(*a.nf_dev) : a.nf;
  const uint32_t m = a.ctrl->mf32;
  if (nf <= 0 || m == 0) return;
  const uint32_t nchunks = (m + kExpandChunk - 1) / kExpandChunk;
  if (blockIdx.x >= nchunks) return;
  if (threadIdx.x == 0) s_nbuf = 0;
  unsigned long long won_total = 0, mnew = 0, insub = 0;
  const uint32_t cflip = a.complement ? 1u : 0u;

  auto flush = [&]() {  // all threads; callers are past a barrier
    const uint32_t nb = s_nbuf;
    if (nb == 0) return;
    if (threadIdx.x == 0) s_base = atomicAdd(&a.ctrl->qcount[a.qslot], nb);
    __syncthreads();
    const uint32_t b = s_base;
    for (uint32_t k = threadIdx.x; k < nb; k += kThreads) a.Qout[b + k] = s_buf[k];
    __syncthreads();
    if (threadIdx.x == 0) s_nbuf = 0;
    __syncthreads();
  };

  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const uint32_t e0 = c * kExpandChunk;
    const uint32_t e1 = min(e0 + uint32_t(kExpandChunk), m);
    const int32_t k0 = a.chunk_first[c];
    const int32_t k1 = (c + 1 < nchunks) ? a.chunk_first[c + 1] : nf - 1;
    const int32_t n = k1 - k0 + 1;
    const bool in_lds = n <= kExpandWin;
    __syncthreads();  // previous chunk's LDS readers are done, s_nbuf is settled
    if (a.Qout && s_nbuf + kExpandChunk > kExpandBuf) flush();
    if (in_lds) {
      for (int32_t i = threadIdx.x; i < n; i += kThreads) {
        sS[i] = a.S[k0 + i];
        sR[i] = a.R[k0 + i];
        sQ[i] = a.Q[k0 + i];
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
          const int32_t kk = thread_search(sS, 0, n, e);
          s = sS[kk]; rs = sR[kk]; u[t] = sQ[kk];
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
        if (a.out_rowptr) mnew += uint64_t(a.out_rowptr[w[t] + 1] - a.out_rowptr[w[t]]);
        if (a.in_colptr) insub += uint64_t(a.in_colptr[w[t] + 1] - a.in_colptr[w[t]]);
      }
      if (a.Qout) {
        const uint64_t bal = __ballot(won[t]);
        if (bal) {
          const int cnt = __popcll(bal);
          const int leader = __ffsll((unsigned long long)bal) - 1;
          uint32_t p = 0;
          if (lane() == leader) p = atomicAdd(&s_nbuf, uint32_t(cnt));
          p = __shfl(p, leader, 64);
          if (won[t]) s_buf[p + __popcll(bal & lanemask_lt())] = w[t];
        }
      }
    }
  }
  __syncthreads();
  if (a.Qout) flush();
  unsigned long long v[4] = {won_total, mnew, insub, 0};
  block_sum4(v);
  if (threadIdx.x == 0) {
    // every edge of a chunk is read exactly once; the block's chunks sum to its edges
    unsigned long long edges = 0;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x)
      edges += min(uint32_t(kExpandChunk), m - c * kExpandChunk);
    stripe_add(a.slot, v[0], 0, edges, v[1], v[2]);
  }
}

// ------------------------------------------------------------------ pull
// Row-based masked matvec (Algorithm 2) over CSC(A). A block owns 64 bitmap
// words (2048 rows): it lists the rows its mask lets through (output
// sparsity, Section 5.2), lets one thread check the first kPullFirst
// in-neighbours of each row in stored order and stop at the first hit
// (early exit, Section 5.3), and hands longer unresolved rows to a whole
// wave, which checks 64 in-neighbours per step and keeps the lowest hit, so
// the reported parent is always the first in stored order. A thread works on
// kPullBatch rows at once so their loads overlap. Results gather in LDS and
// the block writes its words of the output vector whole, so no atomics touch
// the output bitmap. `x` (the input vector) is never written here, which
// keeps the visited snapshot exact when x = visited (operand reuse,
// Section 5.4).
template <bool EE>
__global__ __launch_bounds__(kThreads) void k_pull(PullArgs a) {
  __shared__ uint16_t s_cand[kPullTileV];
  __shared__ uint16_t s_long[kPullTileV];
  __shared__ uint32_t s_found[kPullTileWords];
  __shared__ int32_t s_ncand, s_nlong;
  reset_slot(a.ctrl, a.reset, a.reset_level);
  const int tid = threadIdx.x;
  const int32_t w0 = blockIdx.x * kPullTileWords;
  const int32_t v0 = w0 * 32;
  const uint32_t cflip = a.complement ? 0xffffffffu : 0u;

  if (tid < 64) {  // wave 0 lists the candidate rows of the tile in order
    const int32_t w = w0 + tid;
    uint32_t cand = 0;
    s_found[tid] = 0;
    if (w < a.nwords) {
      const uint32_t pass = a.mask ? (a.mask[w] ^ cflip) : 0xffffffffu;
      cand = (a.mask_after ? 0xffffffffu : pass) & a.nz[w] & valid_bits(w, a.V);
    }
    const int c = __popc(cand);
    const int incl = wave_incl_scan(c);
    int pos = incl - c;
    uint32_t bits = cand;
    while (bits) {
      const int b = __ffs(bits) - 1;
      s_cand[pos++] = uint16_t(tid * 32 + b);
      bits &= bits - 1;
    }
    if (tid == 63) {
      s_ncand = incl;
      s_nlong = 0;
    }
  }
  __syncthreads();
  const int32_t ncand = s_ncand;
  unsigned long long checks = 0, insub = 0;

  auto record = [&](int32_t off, int32_t j, int32_t indeg) {
    const int32_t i = v0 + off;
    if (a.mask_after && a.mask && !(get_bit(a.mask, i) ^ (cflip & 1u))) return;
    atomicOr(&s_found[off >> 5], 1u << (off & 31));
    if (a.depth) a.depth[i] = a.level + 1;
    if (a.parent) a.parent[i] = j;
    if (a.edge_rule) insub += uint64_t(indeg);
  };

  for (int32_t base = 0; base < ncand; base += kPullBatch * kThreads) {
    int32_t off[kPullBatch], beg[kPullBatch], end[kPullBatch], j[kPullBatch];
    bool hit[kPullBatch];
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) {
      const int32_t idx = base + t * kThreads + tid;
      off[t] = idx < ncand ? int32_t(s_cand[idx]) : -1;
    }
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) {
      beg[t] = off[t] >= 0 ? a.colptr[v0 + off[t]] : 0;
      end[t] = off[t] >= 0 ? a.colptr[v0 + off[t] + 1] : 0;
    }
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) j[t] = beg[t] < end[t] ? a.rowind[beg[t]] : 0;
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) hit[t] = beg[t] < end[t] && get_bit(a.x, j[t]);
#pragma unroll
    for (int t = 0; t < kPullBatch; ++t) {
      if (off[t] < 0) continue;
      const int32_t lim = min(end[t], beg[t] + kPullFirst);
      int32_t h = hit[t] ? j[t] : -1, p = beg[t];
      if (!hit[t]) {
        for (p = beg[t] + 1; p < lim; ++p) {
          const int32_t jj = a.rowind[p];
          if (get_bit(a.x, jj)) { h = jj; break; }
        }
      }
      if (EE) {
        checks += uint64_t(h >= 0 ? p - beg[t] + 1 : lim - beg[t]);
        if (h >= 0) record(off[t], h, end[t] - beg[t]);
        else if (end[t] > lim) s_long[atomicAdd(&s_nlong, 1)] = uint16_t(base + t * kThreads + tid);
      } else {
        // no early exit: every in-neighbour is examined; the first hit is kept
        checks += uint64_t(lim - beg[t]);
        if (h >= 0) record(off[t], h, end[t] - beg[t]);
        if (end[t] > lim)
          s_long[atomicAdd(&s_nlong, 1)] = uint16_t((base + t * kThreads + tid) | (h >= 0 ? 0x8000 : 0));
      }
    }
  }
  __syncthreads();

  const int32_t nlong = s_nlong;
  const int wv = tid >> 6;
  for (int32_t r = wv; r < nlong; r += kThreads / 64) {
    const uint16_t ent = s_long[r];
    const bool done = (ent & 0x8000) != 0;
    const int32_t off = s_cand[ent & 0x7fff];
    const int32_t i = v0 + off;
    const int32_t beg0 = a.colptr[i], end = a.colptr[i + 1];
    const int32_t beg = beg0 + kPullFirst;
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
      if (hit >= 0) record(off, hit, end - beg0);
    }
  }
  __syncthreads();

  unsigned long long nfound = 0, nout = 0;
  if (tid < kPullTileWords) {
    const int32_t w = w0 + tid;
    if (w < a.nwords) {
      const uint32_t f = s_found[tid];
      const uint32_t o = ((a.out_base ? a.out_base[w] : 0u) | f) & valid_bits(w, a.V);
      a.out[w] = o;
      if (a.found_out) a.found_out[w] = f;
      nfound = __popc(f);
      nout = a.count_out ? __popc(o) : 0;
    }
  }
  unsigned long long v[4] = {nfound, nout, checks, insub};
  block_sum4(v);
  if (tid == 0) stripe_add(a.slot, v[0], v[1], v[2], 0, v[3]);
}

// ------------------------------------------------- dense-to-sparse convert
// Set bits of (a AND NOT b_not) as an ascending index list (DENSE2SPARSE of
// Section 6.3): popcount per word, block scan, tile prefix, write.
__global__ __launch_bounds__(kThreads) void k_d2s(const uint32_t* __restrict__ a,
                                                  const uint32_t* __restrict__ b_not,
                                                  int32_t nwords, int32_t V,
                                                  int32_t* __restrict__ out, Ctrl* ctrl,
                                                  unsigned long long ticket_base, uint32_t epoch,
                                                  uint64_t* flags, uint32_t* count_out) {
  const uint32_t tile = take_ticket(ctrl, ticket_base);
  const int32_t wbase = int32_t(tile) * kD2STile + threadIdx.x * kD2SWPT;
  uint32_t bits[kD2SWPT];
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kD2SWPT; ++k) {
    const int32_t w = wbase + k;
    bits[k] = 0;
    if (w < nwords) bits[k] = a[w] & (b_not ? ~b_not[w] : 0xffffffffu) & valid_bits(w, V);
    c += __popc(bits[k]);
  }
  uint32_t agg;
  const uint32_t excl = block_excl_scan(c, &agg);
  const uint32_t tile_excl = tile_exclusive_prefix(flags, tile, epoch, agg);
  uint32_t pos = tile_excl + excl;
#pragma unroll
  for (int k = 0; k < kD2SWPT; ++k) {
    uint32_t b = bits[k];
    while (b) {
      const int i = __ffs(b) - 1;
      out[pos++] = (wbase + k) * 32 + i;
      b &= b - 1;
    }
  }
  const uint32_t ntiles = uint32_t((nwords + kD2STile - 1) / kD2STile);
  if (tile == ntiles - 1 && threadIdx.x == 0) *count_out = tile_excl + agg;
}

// --------------------------------------------------------------- helpers
__global__ __launch_bounds__(kThreads) void k_fill(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// SPARSE2DENSE: scatter an index list into a (zeroed) bit vector.
__global__ __launch_bounds__(kThreads) void k_s2d(const int32_t* idx, int32_t n_arg,
                                                  const uint32_t* n_dev, int32_t V,
                                                  uint32_t* bits) {
  const int32_t n = n_dev ? int32_t(*n_dev) : n_arg;
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
__global__ __launch_bounds__(kThreads) void k_nz_bits(const int32_t* ptr, int32_t V, uint32_t* bits) {
  const int32_t w = blockIdx.x * kThreads + threadIdx.x;
  const int32_t nwords = (V + 31) / 32;
  if (w >= nwords) return;
  uint32_t b = 0;
  for (int k = 0; k < 32; ++k) {
    const int32_t i = w * 32 + k;
    if (i < V && ptr[i + 1] > ptr[i]) b |= 1u << k;
  }
  bits[w] = b;
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

hipError_t launch_bfs_init(hipStream_t s, int32_t V, int32_t nwords, int32_t source,
                           const int32_t* rowptr, const int32_t* colptr, int32_t* depth,
                           int32_t* parent, uint32_t* vis, int32_t* Q, Ctrl* ctrl, uint64_t* flags,
                           int64_t nflags) {
  const int64_t n = std::max<int64_t>(std::max<int64_t>(V / 4 + 4, nwords), nflags);
  hipLaunchKernelGGL(k_bfs_init, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s, V,
                     nwords, source, rowptr, colptr, depth, parent, vis, Q, ctrl, flags, nflags);
  return hipGetLastError();
}

hipError_t launch_ctrl_init(hipStream_t s, Ctrl* ctrl, uint64_t* flags, int64_t nflags) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(grid_for(nflags, kThreads, 1024)), dim3(kThreads), 0, s,
                     ctrl, flags, nflags);
  return hipGetLastError();
}

hipError_t launch_push_scan(hipStream_t s, int64_t tiles, const int32_t* Q, int32_t nf,
                            const uint32_t* nf_dev, const int32_t* rowptr, int32_t* S, int32_t* R,
                            int32_t* chunk_first, Ctrl* ctrl, unsigned long long ticket_base,
                            uint32_t epoch, uint64_t* flags, int32_t level_slot, LevelSlot* reset,
                            int32_t reset_level) {
  hipLaunchKernelGGL(k_push_scan, dim3(unsigned(tiles)), dim3(kThreads), 0, s, Q, nf, nf_dev,
                     rowptr, S, R, chunk_first, ctrl, ticket_base, epoch, flags, level_slot, reset,
                     reset_level);
  return hipGetLastError();
}

hipError_t launch_push_expand(hipStream_t s, int32_t blocks, const ExpandArgs& a) {
  hipLaunchKernelGGL(k_push_expand, dim3(unsigned(blocks)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pull(hipStream_t s, bool early_exit, const PullArgs& a) {
  const unsigned g = unsigned((a.nwords + kPullTileWords - 1) / kPullTileWords);
  if (early_exit)
    hipLaunchKernelGGL(k_pull<true>, dim3(g), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_pull<false>, dim3(g), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_d2s(hipStream_t s, const uint32_t* a, const uint32_t* b_not, int32_t nwords,
                      int32_t V, int32_t* out, Ctrl* ctrl, unsigned long long ticket_base,
                      uint32_t epoch, uint64_t* flags, uint32_t* count_out) {
  hipLaunchKernelGGL(k_d2s, dim3(unsigned(d2s_tiles(nwords))), dim3(kThreads), 0, s, a, b_not,
                     nwords, V, out, ctrl, ticket_base, epoch, flags, count_out);
  return hipGetLastError();
}

hipError_t launch_fill(hipStream_t s, uint32_t* p, int64_t n, uint32_t v) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kThreads * 4, 4096)), dim3(kThreads), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_s2d(hipStream_t s, const int32_t* idx, int32_t n, const uint32_t* n_dev,
                      int32_t V, uint32_t* bits) {
  const int64_t cover = n_dev ? int64_t(V) : int64_t(n);
  hipLaunchKernelGGL(k_s2d, dim3(grid_for(cover, kThreads * 4, 4096)), dim3(kThreads), 0, s, idx,
                     n, n_dev, V, bits);
  return hipGetLastError();
}

hipError_t launch_mxv_finalize(hipStream_t s, uint32_t* y, const uint32_t* r, int32_t nwords,
                               int32_t V, int accum, LevelSlot* slot) {
  hipLaunchKernelGGL(k_mxv_finalize, dim3(grid_for(nwords, kThreads, 1u << 30)), dim3(kThreads),
                     0, s, y, r, nwords, V, accum, slot);
  return hipGetLastError();
}

hipError_t launch_nz_bits(hipStream_t s, const int32_t* ptr, int32_t V, uint32_t* bits) {
  hipLaunchKernelGGL(k_nz_bits, dim3(grid_for(words_of(V), kThreads, 1u << 30)), dim3(kThreads),
                     0, s, ptr, V, bits);
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
