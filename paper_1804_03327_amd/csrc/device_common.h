// Device helpers shared by the single-source and the multi-source kernels:
// wave and block reductions, striped level counters, the single-pass tile
// prefix (decoupled look-back) and the frontier scans that turn a list or a
// bitmap into the degree prefix the load-balanced expansion reads. Every
// translation unit that includes this gets its own copy (anonymous namespace).
#pragma once

#include "dobfs_internal.h"

#include <hip/hip_ext.h>

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

// Cross-lane steps by DPP (GFX9 data-parallel primitives: shift right within
// a row of 16 lanes, broadcast lane 15 / 31 to the next rows), a few cycles
// each, where a lane shuffle goes through the LDS crossbar. The sequence is
// the wave's inclusive scan; lane 63 ends with the whole wave's total. A
// lane reading outside its row, or a row the mask leaves out, adds the
// identity 0 (the values are unsigned). Every lane of the wave must be active.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), kCtrl, kRowMask, 0xf, false));
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  return uint64_t(dpp32<kCtrl, kRowMask>(uint32_t(v))) | (uint64_t(dpp32<kCtrl, kRowMask>(uint32_t(v >> 32))) << 32);
}
struct OpAdd {
  template <class T> __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
  template <class T> __device__ __forceinline__ T operator()(T a, T b) const { return a > b ? a : b; }
};
struct OpOr {
  template <class T> __device__ __forceinline__ T operator()(T a, T b) const { return a | b; }
};
template <class Op>
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t v, Op op) {
  v = op(v, dpp32<kDppRowShr1, 0xf>(v));
  v = op(v, dpp32<kDppRowShr2, 0xf>(v));
  v = op(v, dpp32<kDppRowShr4, 0xf>(v));
  v = op(v, dpp32<kDppRowShr8, 0xf>(v));
  v = op(v, dpp32<kDppRowBcast15, 0xa>(v));
  v = op(v, dpp32<kDppRowBcast31, 0xc>(v));
  return v;
}
template <class Op>
__device__ __forceinline__ uint64_t wave_scan_dpp(uint64_t v, Op op) {
  v = op(v, dpp64<kDppRowShr1, 0xf>(v));
  v = op(v, dpp64<kDppRowShr2, 0xf>(v));
  v = op(v, dpp64<kDppRowShr4, 0xf>(v));
  v = op(v, dpp64<kDppRowShr8, 0xf>(v));
  v = op(v, dpp64<kDppRowBcast15, 0xa>(v));
  v = op(v, dpp64<kDppRowBcast31, 0xc>(v));
  return v;
}
__device__ __forceinline__ uint32_t lane63(uint32_t v) { return uint32_t(__builtin_amdgcn_readlane(int(v), 63)); }
__device__ __forceinline__ uint64_t lane63(uint64_t v) {
  return uint64_t(lane63(uint32_t(v))) | (uint64_t(lane63(uint32_t(v >> 32))) << 32);
}

__device__ __forceinline__ int wave_incl_scan(int v) { return int(wave_scan_dpp(uint32_t(v), OpAdd{})); }
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return lane63(wave_scan_dpp(v, OpAdd{})); }
__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
  return lane63(wave_scan_dpp(uint64_t(v), OpAdd{}));
}
// Launch with optional kernel start / end events (hipExtLaunchKernel).
template <class K, class... Args>
hipError_t launch_k(K kernel, dim3 grid, hipStream_t s, hipEvent_t t0, hipEvent_t t1, Args... args) {
  if (t0 || t1)
    hipExtLaunchKernelGGL(kernel, grid, dim3(kThreads), 0, s, t0, t1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, dim3(kThreads), 0, s, args...);
  return hipGetLastError();
}

// A value every lane holds alike, moved to scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
  return uint64_t(lo) | (uint64_t(hi) << 32);
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
  st.fbits = 0;
  st.mu = 0;
  st.maxdeg = 0;
  st.tilemax = 0;
}

// Raises a block's stripe's largest discovered out-degree (thread 0 only).
__device__ __forceinline__ void stripe_max(LevelSlot* slot, uint32_t deg) {
  if (deg) atomicMax(&slot->s[blockIdx.x % kStripes].maxdeg, deg);
}

__device__ __forceinline__ uint32_t wave_max32(uint32_t v) { return lane63(wave_scan_dpp(v, OpMax{})); }
// Largest value over the 256 threads of a block (every thread gets it).
__device__ __forceinline__ uint32_t block_max32(uint32_t v) {
  __shared__ uint32_t s_m[kThreads / 64];
  v = wave_max32(v);
  if (lane() == 0) s_m[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t t = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) t = max(t, s_m[w]);
  __syncthreads();
  return t;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) { return lane63(wave_scan_dpp(v, OpOr{})); }
// OR over the 256 threads of a block (every thread gets the result).
__device__ __forceinline__ uint64_t block_or64(uint64_t v) {
  __shared__ uint64_t s_o[kThreads / 64];
  v = wave_or64(v);
  if (lane() == 0) s_o[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t t = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) t |= s_o[w];
  __syncthreads();
  return t;
}

// ORs a block's discovered source bits into its stripe (thread 0 only).
__device__ __forceinline__ void stripe_or(LevelSlot* slot, uint64_t bits) {
  if (bits) atomicOr((unsigned long long*)&slot->s[blockIdx.x % kStripes].fbits, (unsigned long long)bits);
}

// ---- single-pass tile prefix (decoupled look-back) ----
// Tile descriptors are one 64-bit word: [epoch:30][status:2][value:32], so a
// single atomic store publishes status and value together. Tiles are numbered
// by tickets taken when a block is ready to work on one, so every tile a
// block waits on belongs to a running block that publishes without waiting.
__device__ __forceinline__ uint64_t pack_flag(uint32_t epoch, uint32_t status, uint32_t value) {
  return (uint64_t(epoch) << 34) | (uint64_t(status) << 32) | uint64_t(value);
}

__device__ __forceinline__ uint32_t take_ticket(unsigned long long* ticket) {
  __shared__ uint32_t s_tile;
  __syncthreads();  // every thread is done with the previous tile's s_tile
  if (threadIdx.x == 0) s_tile = uint32_t(atomicAdd(ticket, 1ull));
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

// Chunks of kExpandChunk edges whose first edge lies in [run, run + deg):
// the vertex at list position k is their first vertex.
__device__ __forceinline__ void mark_chunks(int32_t* chunk_first, uint32_t run, int32_t deg, int32_t k) {
  if (deg <= 0) return;
  const uint32_t c0 = (run + kExpandChunk - 1) / kExpandChunk;
  const uint32_t c1 = (run + uint32_t(deg) - 1) / kExpandChunk;
  for (uint32_t c = c0; c <= c1; ++c) chunk_first[c] = k;
}

// --------------------------------------------------- frontier list scans
// Out-degree of every frontier vertex and its exclusive prefix sum (the
// "length" and "scan" steps of the column-based matvec, Section 6.2): S[k] is
// where vertex Q[k]'s adjacency starts in the concatenated expansion, R[k] its
// row start in CSR(A), and every chunk of kExpandChunk edges records its
// first vertex, which is all the expand step needs to find its work (the
// load-balanced gather). Blocks take tiles by ticket until the list is done.
__device__ void scan_list(const int32_t* __restrict__ Q, int32_t nf, const int32_t* __restrict__ rowptr,
                          int32_t* __restrict__ S, int32_t* __restrict__ R,
                          int32_t* __restrict__ chunk_first, uint64_t* flags, uint32_t epoch,
                          unsigned long long* ticket, uint32_t* mf_out) {
  const uint32_t ntiles = uint32_t(nf > 0 ? (nf + kScanTile - 1) / kScanTile : 1);
  if (blockIdx.x >= ntiles) return;  // no tile for this block: take no ticket
  const bool one_each = ntiles <= gridDim.x;
  for (bool first = true;; first = false) {
    if (one_each && !first) return;  // every tile has a block of its own
    const uint32_t tile = take_ticket(ticket);
    if (tile >= ntiles) return;
    const int64_t base = int64_t(tile) * kScanTile + int64_t(threadIdx.x) * kScanIPT;
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
        mark_chunks(chunk_first, run, deg[k], int32_t(base + k));
        run += uint32_t(deg[k]);
      }
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) *mf_out = tile_excl + agg;
  }
}

// The set bits of (a AND NOT b_not) as an ascending list (DENSE2SPARSE of
// Section 6.3), fused with the same degree prefix when rowptr is given: two
// look-back chains, one over vertex counts and one over degree sums.
__device__ void scan_bits(const ScanBitsArgs& a) {
  const uint32_t ntiles = uint32_t((a.nwords + kBitsTile - 1) / kBitsTile);
  if (blockIdx.x >= ntiles) return;  // no tile for this block: take no ticket
  const bool one_each = ntiles <= gridDim.x;
  for (bool first = true;; first = false) {
    if (one_each && !first) return;  // every tile has a block of its own
    const uint32_t tile = take_ticket(a.ticket);
    if (tile >= ntiles) return;
    const int32_t wbase = int32_t(tile) * kBitsTile + threadIdx.x * kBitsWPT;
    uint32_t bits[kBitsWPT];
    uint32_t c = 0, d = 0;
#pragma unroll
    for (int k = 0; k < kBitsWPT; ++k) {
      const int32_t w = wbase + k;
      bits[k] = 0;
      if (w < a.nwords)
        bits[k] = a.a[w] & (a.b_not ? ~a.b_not[w] : 0xffffffffu) & valid_bits(w, a.V);
      c += __popc(bits[k]);
      if (a.rowptr) {
        uint32_t b = bits[k];
        while (b) {
          const int32_t v = w * 32 + __ffs(b) - 1;
          d += uint32_t(a.rowptr[v + 1] - a.rowptr[v]);
          b &= b - 1;
        }
      }
    }
    if (a.mu_slot) {  // in-edges of the rows nobody has reached yet (m_u of the edge-count rule)
      unsigned long long mu[4] = {0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < kBitsWPT; ++k) {
        const int32_t w = wbase + k;
        uint32_t u = w < a.nwords ? (a.unv_nz[w] & ~a.unv_vis[w] & valid_bits(w, a.V)) : 0u;
        while (u) {
          const int32_t v = w * 32 + __ffs(u) - 1;
          mu[0] += uint64_t(a.colptr[v + 1] - a.colptr[v]);
          u &= u - 1;
        }
      }
      block_sum4(mu);
      if (threadIdx.x == 0 && mu[0]) atomicAdd(&a.mu_slot->s[blockIdx.x % kStripes].mu, mu[0]);
    }
    uint32_t agg_c, agg_d = 0;
    const uint32_t excl_c = block_excl_scan(c, &agg_c);
    uint32_t excl_d = 0;
    if (a.rowptr) excl_d = block_excl_scan(d, &agg_d);
    const uint32_t pc = tile_exclusive_prefix(a.flagsA, tile, a.epochA, agg_c);
    uint32_t pd = 0;
    if (a.rowptr) pd = tile_exclusive_prefix(a.flagsB, tile, a.epochB, agg_d);
    uint32_t pos = pc + excl_c, run = pd + excl_d;
#pragma unroll
    for (int k = 0; k < kBitsWPT; ++k) {
      uint32_t b = bits[k];
      while (b) {
        const int32_t v = (wbase + k) * 32 + __ffs(b) - 1;
        a.Qout[pos] = v;
        if (a.rowptr) {
          const int32_t rb = a.rowptr[v], deg = a.rowptr[v + 1] - rb;
          a.S[pos] = int32_t(run);
          a.R[pos] = rb;
          mark_chunks(a.chunk_first, run, deg, int32_t(pos));
          run += uint32_t(deg);
        }
        ++pos;
        b &= b - 1;
      }
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) {
      *a.nf_out = pc + agg_c;
      if (a.mf_out) *a.mf_out = pd + agg_d;
    }
  }
}

__device__ __forceinline__ int32_t thread_search(const int32_t* S, int32_t lo, int32_t hi, uint32_t e) {
  while (hi - lo > 1) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (uint32_t(S[mid]) <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// Whether the scan of a push that follows a pull recounts m_u (see scan_bits):
// the single-source traversal under the edge-count rule. Its pulls then skip
// the in-degrees of the rows they find.
__device__ __forceinline__ bool recounts_mu(const BfsArgs& a) { return a.edge_rule != 0; }
__device__ __forceinline__ bool recounts_mu(const BatchArgs&) { return false; }
// The multi-source traversal also needs the (vertex, source) pair counts and the source bits.
__host__ __device__ constexpr bool is_batch(const BfsArgs&) { return false; }
__host__ __device__ constexpr bool is_batch(const BatchArgs&) { return true; }

// The state entering level L, from the state entering L-1 and the counters
// L-1 left: the direction rule of Section 6.3 (or Beamer's edge form),
// forced directions and mode overrides, buffer parities. Every thread
// computes it from uniform addresses, which the compiler serves with scalar
// loads; this measured several microseconds faster per launch than one wave
// computing it and broadcasting it through LDS. All blocks of a level_prep
// compute the same state.
// The counters one level left, spread over the lanes for the wave reductions: every block's
// waves read them at the start of a step, so the read is laid out for the fewest cache lines
// per load. Lane j reads bytes 16 (j % 4) .. 16 (j % 4) + 15 of stripes j / 4 and 16 + j / 4
// (the 56 bytes of counters start every 128-byte stripe): two 16-byte loads touching 16 lines
// each, where one stripe per lane and field took seven loads of 32 lines. A lane holds the
// combined value of its two stripes for the fields in its quarter, zero for the others.
static_assert(kStripes == 32 && sizeof(Stripe) == 128, "two loads of 16 stripes");
static_assert(offsetof(Stripe, edges) == 8 && offsetof(Stripe, mnew) == 16 && offsetof(Stripe, insub) == 24 &&
                  offsetof(Stripe, fbits) == 32 && offsetof(Stripe, mu) == 40 &&
                  offsetof(Stripe, maxdeg) == 48 && offsetof(Stripe, tilemax) == 52,
              "stripe counters in four 16-byte quarters");
struct StripeLanes {
  uint64_t count, aux, edges, mnew, insub, fbits, mu;
  uint32_t maxdeg, tilemax;
};
__device__ __forceinline__ StripeLanes load_stripes(const LevelSlot& sl) {
  const int k = lane();
  const int q = k & 3;
  const ulonglong2 x0 = reinterpret_cast<const ulonglong2*>(&sl.s[k >> 2])[q];
  const ulonglong2 x1 = reinterpret_cast<const ulonglong2*>(&sl.s[16 + (k >> 2)])[q];
  StripeLanes x;
  x.count = q == 0 ? (x0.x & 0xffffffffull) + (x1.x & 0xffffffffull) : 0ull;
  x.aux = q == 0 ? (x0.x >> 32) + (x1.x >> 32) : 0ull;
  x.edges = q == 0 ? x0.y + x1.y : 0ull;
  x.mnew = q == 1 ? x0.x + x1.x : 0ull;
  x.insub = q == 1 ? x0.y + x1.y : 0ull;
  x.fbits = q == 2 ? (x0.x | x1.x) : 0ull;
  x.mu = q == 2 ? x0.y + x1.y : 0ull;
  x.maxdeg = q == 3 ? max(uint32_t(x0.x), uint32_t(x1.x)) : 0u;
  x.tilemax = q == 3 ? max(uint32_t(x0.x >> 32), uint32_t(x1.x >> 32)) : 0u;
  return x;
}
// The wave's total of a count whose total is below 2^32, as a scalar.
__device__ __forceinline__ uint64_t wave_total(uint64_t v) {
  return uint64_t(__builtin_amdgcn_readfirstlane(wave_sum(uint32_t(v))));
}
// Marks the counters as needed here, so that their loads go out together with the load of
// the previous state (the compiler would otherwise sink them into the branch that starts a
// level, a round trip later).
__device__ __forceinline__ void stripes_needed(const StripeLanes& x) {
  asm volatile("" ::"v"(x.count), "v"(x.mnew), "v"(x.fbits), "v"(x.maxdeg));
}

// The state entering level L from the state entering L-1 (prev) and the
// counters L-1 left (x): the direction rule of Section 6.3 (or Beamer's edge
// form), forced directions and mode overrides, buffer parities, and whether
// a push can share out its own work.
// prev_slot: the counter slot of the step that ended level L-1 (multi-source: its m_f tells
// whether that push listed its winners or marked them).
template <class Args>
__device__ LevelState next_state(const Args& a, int32_t L, int32_t forced, const LevelState& prev,
                                 const StripeLanes& x, int32_t prev_slot, LevelTotals* tot_out) {
  LevelTotals t{0, 0, 0, 0, 0, 0};
  LevelState st = prev;
  st.level = L;
  if (!prev.done) {
    // each cross-lane reduction costs a few hundred cycles in every wave of a launch every
    // level runs, so only the totals this traversal and level use are formed (the branches
    // are uniform): the ones that decide the level in every block, the record's (edges,
    // pairs) only in block 0, which publishes it. Vertex and edge totals are below 2^31
    // (int32 vertex ids and CSR offsets), so they add up in 32 bits.
    constexpr bool batch = is_batch(Args{});
    const bool record = blockIdx.x == 0;
    t.count = wave_total(x.count);
    t.mnew = wave_total(x.mnew);
    if (record) t.edges = wave_total(x.edges);
    if (batch && record) t.aux = uniform64(wave_sum64(x.aux));
    if (a.edge_rule) t.insub = wave_total(x.insub);
    if (t.count == 0) {
      st.done = 1;
      st.levels = L;
    } else {
      const int64_t n_new = int64_t(t.count);
      // m_u loses the in-edges of each push level's winners; pulls leave it alone, and the
      // push that follows a pull recounts it (single source)
      const bool recounted = recounts_mu(a) && prev.dir == 0 && !prev.list_valid;
      if (recounted) t.mu = wave_total(x.mu);
      const int64_t m_u = (recounted ? int64_t(t.mu) : prev.m_u) - (a.edge_rule ? int64_t(t.insub) : 0);
      int32_t next = next_direction_rule(a.heuristic, a.alpha, a.beta, prev.dir, a.V, prev.nf, n_new,
                                         int64_t(t.mnew), m_u);
      if (a.mode == 1) next = 0;  // push only
      if (a.mode == 5) next = 1;  // pull only
      if (forced >= 0) next = forced;
      st.dir = next;
      st.nf = int32_t(n_new);
      // a push level appended its winners to Q[L % 2], unless (multi-source) it marked them
      st.list_valid = (prev.dir == 0 && !(batch && mb_push_marks(a.ctrl->mf[prev_slot]))) ? 1 : 0;
      st.vis_idx = prev.dir == 1 ? (prev.vis_idx ^ 1) : prev.vis_idx;
      st.m_u = m_u;
      st.active = batch ? uniform64(wave_or64(x.fbits)) : 0ull;
      // a push needs no global scan when its frontier's edges can be shared out inside
      // blocks: a list from a push whose sizes local_fits() accepts (local 1), or the bits a
      // pull left when no tile found more than sched.bitmap_rows rows and none of high
      // out-degree (local 2: every block expands its own slice of the bitmap)
      st.local = 0;
      st.share = 1;
      if (a.local_push && next == 0) {
        if (prev.dir == 0) {
          // a push's winners' out-degrees are tracked unless the graph is low-degree and the
          // rule needs no m_f; then kLocalDeg bounds them
          const bool tracked = a.edge_rule || !a.low_degree;
          const int64_t mf_b = tracked ? int64_t(t.mnew) : INT64_MAX;
          const int64_t md_b = tracked ? int64_t(__builtin_amdgcn_readfirstlane(wave_max32(x.maxdeg))) : int64_t(kLocalDeg);
          const int64_t G = main_blocks(a.nwords);
          if (a.low_degree || local_fits(n_new, mf_b, md_b, G, a.sched.local_unit, a.sched.local_chunks)) {
            st.local = 1;
            st.share = local_share(n_new, mf_b, md_b, G, a.sched.local_unit);
          }
        } else {
          const uint32_t tm = __builtin_amdgcn_readfirstlane(wave_max32(x.tilemax));
          st.local = tm <= uint32_t(a.sched.bitmap_rows) ? 2 : 0;
        }
      }
      st.phase = (next == 0 && !st.local) ? kPhaseScan : kPhaseWhole;
    }
  }
  *tot_out = t;
  return st;
}

// The state entering level L (level loops with one slot per level): every
// thread computes it from uniform addresses, which the compiler serves with
// scalar loads; the previous state and the counters come in one round trip.
// All blocks of a launch compute the same state.
template <class Args>
__device__ LevelState level_state(const Args& a, int32_t L, int32_t forced, LevelTotals* tot_out,
                                  LevelState* prev_out) {
  const Ctrl* c = a.ctrl;
  if (L == 0) {
    LevelState st = c->ring[0];
    if (forced >= 0) st.dir = forced;
    *tot_out = LevelTotals{0, 0, 0, 0, 0, 0};
    *prev_out = st;
    return st;
  }
  const StripeLanes x = load_stripes(c->slot[(L - 1) % kSlots]);
  const LevelState prev = c->ring[(L - 1) % kRing];
  *prev_out = prev;
  return next_state(a, L, forced, prev, x, (L - 1) % kSlots, tot_out);
}

// Block 0 of level L's first kernel: publish the level's state and the
// record of level L-1, and clear the counters level L+1 will add into
// (nothing reads them before the next kernel boundary).
__device__ void publish_level(Ctrl* c, int32_t L, const LevelState& st, const LevelState& prev,
                              const LevelTotals& tot) {
  if (blockIdx.x != 0) return;
  if (threadIdx.x == 0) {
    c->ring[L % kRing] = st;
    if (L >= 1) {
      if (!prev.done) {
        LevelRecord r;
        r.dir = prev.dir;
        r.nf = prev.nf;
        r.n_new = int32_t(tot.count);
        r.variant = prev.dir == 0 ? prev.local : 0;
        r.edges = int64_t(tot.edges);
        // a scanned push level's m_f comes from its scan; a local one reads exactly its m_f edges
        r.m_f = prev.dir == 0 ? (prev.local ? int64_t(tot.edges) : int64_t(c->mf[(L - 1) % kSlots])) : 0;
        r.mnew = tot.mnew;
        r.insub = tot.insub;
        r.aux = tot.aux;
        c->rec[(L - 1) % kRing] = r;
      }
    }
    c->qcount[(L + 1) % kSlots] = 0;
    c->mf[(L + 1) % kSlots] = 0;
    c->ticket[(L + 1) % 2] = 0;
  }
  for (int k = threadIdx.x; k < kStripes; k += blockDim.x) zero_stripe(c->slot[(L + 1) % kSlots].s[k]);
}

// The record of the level before the one step s starts (prev is that level's state).
__device__ __forceinline__ LevelRecord step_record(const Ctrl* c, int32_t s, const LevelState& prev,
                                                   const LevelTotals& tot) {
  LevelRecord r;
  r.dir = prev.dir;
  r.nf = prev.nf;
  r.n_new = int32_t(tot.count);
  r.variant = prev.dir == 0 ? prev.local : 0;
  r.edges = int64_t(tot.edges);
  // a scanned push level's m_f comes from its scan; a local one reads exactly its m_f edges
  r.m_f = prev.dir == 0 ? (prev.local ? int64_t(tot.edges) : int64_t(c->mf[(s - 1) % kSlots])) : 0;
  r.mnew = tot.mnew;
  r.insub = tot.insub;
  r.aux = tot.aux;
  return r;
}

// Block 0: publish step s's state and, when it starts a level, the record of
// the level before; clear what step s + 2 will count into.
__device__ __forceinline__ void publish_step(Ctrl* c, int32_t s, const LevelState& st, const LevelState& prev,
                             const LevelTotals& tot, bool new_level) {
  if (threadIdx.x == 0) {
    c->ring[s % kRing] = st;
    if (new_level) c->rec[(st.level - 1) % kRing] = step_record(c, s, prev, tot);
    c->qcount[(s + 2) % kSlots] = 0;
    c->ticket[(s + 1) % 2] = 0;
  }
  for (int k = threadIdx.x; k < kStripes; k += blockDim.x) zero_stripe(c->slot[(s + 2) % kSlots].s[k]);
}

// Waits until every block of the launch has arrived (see GridBar). Agent-scope
// fences are whole-cache operations (write back / invalidate the XCD's L2), so
// only thread 0 of a block issues them: every wave first waits for its own
// memory operations to complete, then thread 0 releases before its block
// arrives and acquires once after the wait (the polls themselves are relaxed);
// the block barrier after it orders the other waves' reads behind that.
// Returns false when the wait gave up (spin limit, or another block gave up).
__device__ __forceinline__ bool grid_barrier(GridBar* bar, uint32_t target, uint32_t spin_limit) {
  __shared__ int s_ok;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's loads and stores are complete
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the block's writes reach memory
    const uint32_t G = gridDim.x;
    const uint32_t groups = G < uint32_t(kBarGroups) ? G : uint32_t(kBarGroups);
    const uint32_t g = blockIdx.x % groups;
    const uint32_t members = (G - g + groups - 1) / groups;  // blocks b < G with b % groups == g
    const unsigned long long o = __hip_atomic_fetch_add(&bar->group[g].n, 1ull, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
    if ((o + 1) % members == 0) {
      const unsigned long long o2 = __hip_atomic_fetch_add(&bar->top.n, 1ull, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
      if ((o2 + 1) % groups == 0) __hip_atomic_store(&bar->gen, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    uint32_t polls = 0;
    while (int32_t(__hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (++polls > spin_limit) {
        __hip_atomic_fetch_or(&bar->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // released, but another block gave up: it will not arrive again
    if (ok && __hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // drop stale cache lines
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

}  // namespace
}  // namespace dobfs
