// Multi-source BFS kernels of libdobfs for gfx950: up to 64 traversals at
// once, one bit of a uint64 per source. A level is the masked Boolean
// matrix product F' = A^T F .* not(Vis) over (OR, AND), the matvec of
// Algorithm 1 with the frontier vector widened to 64 columns (Section 3
// notes that the masked matvec generalises to a masked matrix product in
// the same way). Push scatters each frontier vertex's source bits along its
// out-edges with atomicOr (Equation 5 per column); pull ORs the visited words
// of a row's in-neighbours until every source still missing is found, the
// early exit of Section 5.3 taken per row once the whole missing set is
// covered. Operand reuse (Section 5.4) holds bit by bit: for every source the
// visited set read by the pull stands in for that source's frontier.
//
// Levels are laid out as in the single-source path: mb_prep decides the
// direction on the device and, for push, lists the frontier vertices with
// their degree prefix; mb_main runs the expansion or the pull. Levels of
// discovery are kept vertex-major ([V][k] uint16, one 128-byte line per
// vertex at k = 64) so a vertex's new bits land in one line; mb_depth turns
// them into the [k][V] int32 depth rows at the end.

#include "device_common.h"

namespace dobfs {
namespace {

__device__ __forceinline__ uint64_t* mb_frontier(const BatchArgs& a, int32_t L) {
  return a.Fs + int64_t(mb_frontier_slot(L)) * a.V;
}

// Level L+1 for every source bit in `bits` of vertex v, where level L+1's
// frontier is not kept (its words are the record of the levels below kMbSnap).
__device__ __forceinline__ void stamp_levels(uint16_t* lvl, int32_t k, int32_t v, uint64_t bits,
                                             int32_t level) {
  if (level + 1 < kMbSnap) return;
  uint16_t* row = lvl + int64_t(v) * k;
  while (bits) {
    const int b = __ffsll((unsigned long long)bits) - 1;
    row[b] = uint16_t(level + 1);
    bits &= bits - 1;
  }
}

// ----------------------------------------------------------------- init
// Visited and level-0 frontier words hold the source bits (the frontier of
// level 0 records that every source is at depth 0), and the control block
// starts a push level whose list is the distinct sources.
__global__ __launch_bounds__(kThreads) void k_mb_init(BatchArgs a, int32_t dir0, int64_t nflags) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t v = t0; v < a.V; v += stride) {
    uint64_t m = 0;
    if ((a.src_filter[(v >> 6) & 15] >> (v & 63)) & 1ull)  // almost no vertex passes the filter
      for (int b = 0; b < a.k; ++b) m |= (a.src[b] == v) ? (1ull << b) : 0ull;
    a.vis[0][v] = m;
    a.Fs[v] = m;  // mb_frontier(a, 0)
  }
  for (int64_t k = t0; k < nflags; k += stride) {
    a.flagsA[k] = 0;
    a.flagsB[k] = 0;
  }
  if (blockIdx.x == 0) {
    Ctrl* c = a.ctrl;
    for (int k = threadIdx.x; k < kSlots * kStripes; k += blockDim.x)
      zero_stripe(c->slot[k / kStripes].s[k % kStripes]);
    for (int k = threadIdx.x; k < a.nuniq; k += blockDim.x) a.Q[0][k] = a.uniq[k];
    if (threadIdx.x == 0) {
      c->ticket[0] = 0;
      c->ticket[1] = 0;
      c->mf32 = 0;
      c->nf32 = 0;
      c->src_outdeg = 0;
      c->src_indeg = 0;
      for (int s = 0; s < kSlots; ++s) {
        c->qcount[s] = 0;
        c->mf[s] = 0;
      }
      LevelState st;
      st.dir = dir0;
      st.done = 0;
      st.list_valid = 1;
      st.vis_idx = 0;
      st.nf = a.nuniq;
      st.levels = 0;
      st.level = 0;
      st.local = 0;
      st.share = 1;
      st.m_u = a.nnz;  // in-edges of vertices some source has not reached yet
      st.active = a.active;
      c->ring[0] = st;
    }
  }
}

// ----------------------------------------------------------------- push
struct MbExpandShared {
  int32_t sS[kExpandWin], sR[kExpandWin], sQ[kExpandWin];
  int32_t buf[kExpandBuf];
  uint32_t nbuf, base;
};

// Column-based product: every edge u -> w of the frontier's concatenated
// adjacency carries F[u]'s source bits to w. The bits w has not seen are
// claimed with one 64-bit atomicOr on Vis[w]; the bits a thread newly set are
// its own, so it stamps their level and adds them to the next frontier word
// of w. The thread whose add made that word nonzero lists w for the next
// level. The chunked, load-balanced walk over the edges is the one of the
// single-source expansion.
__device__ void mb_expand_body(const BatchArgs& a, int32_t L, const LevelState& st, MbExpandShared& sh) {
  const int32_t nf = st.nf;
  const uint32_t m = a.ctrl->mf[L % kSlots];
  if (nf <= 0 || m == 0) return;
  const uint32_t nchunks = (m + kExpandChunk - 1) / kExpandChunk;
  if (blockIdx.x >= nchunks) return;
  const int32_t* Q = a.Q[L % 2];
  int32_t* Qout = a.Q[(L + 1) % 2];
  const uint64_t* Fc = mb_frontier(a, L);
  uint64_t* Fn = mb_frontier(a, L + 1);
  uint64_t* vis = a.vis[st.vis_idx];
  uint32_t* qcount = &a.ctrl->qcount[(L + 1) % kSlots];
  const uint64_t active = a.active;
  if (threadIdx.x == 0) sh.nbuf = 0;
  unsigned long long nvert = 0, nbits = 0, mnew = 0, insub = 0;
  uint64_t fbits = 0;

  auto flush = [&]() {
    const uint32_t nb = sh.nbuf;
    if (nb == 0) return;
    if (threadIdx.x == 0) sh.base = atomicAdd(qcount, nb);
    __syncthreads();
    const uint32_t b = sh.base;
    for (uint32_t k = threadIdx.x; k < nb; k += kThreads) Qout[b + k] = sh.buf[k];
    __syncthreads();
    if (threadIdx.x == 0) sh.nbuf = 0;
    __syncthreads();
  };

  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const uint32_t e0 = c * kExpandChunk;
    const uint32_t e1 = min(e0 + uint32_t(kExpandChunk), m);
    const int32_t k0 = a.chunk_first[c];
    const int32_t k1 = (c + 1 < nchunks) ? a.chunk_first[c + 1] : nf - 1;
    const int32_t n = k1 - k0 + 1;
    const bool in_lds = n <= kExpandWin;
    __syncthreads();
    if (sh.nbuf + kExpandChunk > kExpandBuf) flush();
    if (in_lds) {
      for (int32_t i = threadIdx.x; i < n; i += kThreads) {
        sh.sS[i] = a.S[k0 + i];
        sh.sR[i] = a.R[k0 + i];
        sh.sQ[i] = Q[k0 + i];
      }
    }
    __syncthreads();
    int32_t w[kExpandEPT], u[kExpandEPT], pos[kExpandEPT];
    bool valid[kExpandEPT];
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
          s = a.S[kk]; rs = a.R[kk]; u[t] = Q[kk];
        }
        pos[t] = rs + int32_t(e - uint32_t(s));
      }
    }
    uint64_t x[kExpandEPT];
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) w[t] = valid[t] ? a.colind[pos[t]] : 0;
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) x[t] = valid[t] ? (Fc[u[t]] & active & ~vis[w[t]]) : 0ull;
    bool listed[kExpandEPT];
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      listed[t] = false;
      if (x[t]) {
        const uint64_t old = atomicOr((unsigned long long*)(vis + w[t]), (unsigned long long)x[t]);
        const uint64_t nb = x[t] & ~old;
        if (nb) {
          const uint64_t oldf = atomicOr((unsigned long long*)(Fn + w[t]), (unsigned long long)nb);
          stamp_levels(a.lvl, a.k, w[t], nb, L);
          nbits += uint64_t(__popcll(nb));
          fbits |= nb;
          if (oldf == 0) {
            listed[t] = true;
            ++nvert;
            if (a.edge_rule) mnew += uint64_t(a.rowptr[w[t] + 1] - a.rowptr[w[t]]);
          }
          if (a.edge_rule && ((old | nb) & active) == active)  // this claim completed w
            insub += uint64_t(a.colptr[w[t] + 1] - a.colptr[w[t]]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      const uint64_t bal = __ballot(listed[t]);
      if (bal) {
        const int cnt = __popcll(bal);
        const int leader = __ffsll((unsigned long long)bal) - 1;
        uint32_t p = 0;
        if (lane() == leader) p = atomicAdd(&sh.nbuf, uint32_t(cnt));
        p = __shfl(p, leader, 64);
        if (listed[t]) sh.buf[p + __popcll(bal & lanemask_lt())] = w[t];
      }
    }
  }
  __syncthreads();
  flush();
  unsigned long long v4[4] = {nvert, nbits, mnew, insub};
  block_sum4(v4);
  fbits = block_or64(fbits);
  if (threadIdx.x == 0) {
    stripe_or(&a.ctrl->slot[L % kSlots], fbits);
    unsigned long long edges = 0;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x)
      edges += min(uint32_t(kExpandChunk), m - c * kExpandChunk);
    stripe_add(&a.ctrl->slot[L % kSlots], v4[0], v4[1], edges, v4[2], v4[3]);
  }
}

// ----------------------------------------------------------------- pull
struct MbPullShared {
  uint16_t cand[kMbTileV];
  uint16_t lng[kMbLong];
  uint64_t lacc[kMbLong];
  uint32_t nzf[kMbTileWords];
  int32_t ncand, nlong;
};

// Row-based product over one tile of kMbTileV rows: rows that a still-expanding
// source has not reached (the mask, Section 5.2) and that have in-neighbours
// are listed; each ORs the visited words of its in-neighbours in stored order
// and stops once every missing source bit is found (early exit, Section 5.3).
// A thread takes a row's slab (first kSlab in-neighbours, one read), then the
// row up to kMbMid in-neighbours, then a wave finishes it, 64 per step. The
// tile's new visited words (old | found), next-frontier words and nonzero
// bits are written whole; no atomics touch them.
__device__ void mb_pull_body(const BatchArgs& a, int32_t L, const LevelState& st, int32_t tile,
                             MbPullShared& sh) {
  const int tid = threadIdx.x;
  const int32_t w0 = tile * kMbTileWords;
  const int32_t v0 = w0 * 32;
  const uint64_t* vin = a.vis[st.vis_idx];
  uint64_t* vout = a.vis[st.vis_idx ^ 1];
  uint64_t* Fn = mb_frontier(a, L + 1);
  const uint64_t active = st.active;  // a source with an empty frontier finds nothing more
  if (tid < kMbTileWords) sh.nzf[tid] = 0;
  if (tid == 0) {
    sh.ncand = 0;
    sh.nlong = 0;
  }
  __syncthreads();
  for (int r0 = 0; r0 < kMbTileV; r0 += kThreads) {
    const int r = r0 + tid;
    const int32_t v = v0 + r;
    bool cand = false;
    if (v < a.V) {
      const uint64_t m = vin[v];
      cand = ((~m & active) != 0) && get_bit(a.nz_in, v);
      if (!cand) {
        vout[v] = m;
        Fn[v] = 0;
      }
    }
    const uint64_t bal = __ballot(cand);
    if (bal) {
      const int leader = __ffsll((unsigned long long)bal) - 1;
      int p = 0;
      if (lane() == leader) p = atomicAdd(&sh.ncand, __popcll(bal));
      p = __shfl(p, leader, 64);
      if (cand) sh.cand[p + __popcll(bal & lanemask_lt())] = uint16_t(r);
    }
  }
  __syncthreads();
  const int32_t ncand = sh.ncand;
  unsigned long long nvert = 0, nbits = 0, checks = 0, mnew = 0, insub = 0;
  uint64_t fbits = 0;

  auto finish = [&](int r, uint64_t m, uint64_t found) {
    const int32_t v = v0 + r;
    vout[v] = m | found;
    Fn[v] = found;
    if (!found) return;
    atomicOr(&sh.nzf[r >> 5], 1u << (r & 31));
    stamp_levels(a.lvl, a.k, v, found, L);
    ++nvert;
    nbits += uint64_t(__popcll(found));
    fbits |= found;
    if (a.edge_rule) {
      mnew += uint64_t(a.rowptr[v + 1] - a.rowptr[v]);
      if (((m | found) & a.active) == a.active) insub += uint64_t(a.colptr[v + 1] - a.colptr[v]);
    }
  };

  for (int32_t idx = tid; idx < ncand; idx += kThreads) {
    const int r = sh.cand[idx];
    const int32_t v = v0 + r;
    const uint64_t m = vin[v];
    const uint64_t need = ~m & active;
    // the slab: the row's first kSlab in-neighbours from one coalesced read
    const int4 hd = a.slab[v];
    const int32_t e[kSlab] = {hd.x, hd.y, hd.z, hd.w};
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < kSlab; ++q) {
      if (e[q] >= 0) {
        acc |= vin[e[q]];
        ++checks;
      }
    }
    if ((acc & need) == need || hd.w < 0) {
      finish(r, m, acc & need);
      continue;
    }
    const int32_t beg = a.colptr[v], end = a.colptr[v + 1];
    const int32_t lim = min(end, beg + kMbMid);
    int32_t p = beg + kSlab;
    while (p < lim && (acc & need) != need) {
      int32_t j[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) j[q] = p + q < lim ? a.rowind[p + q] : -1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (j[q] < 0 || (acc & need) == need) continue;
        acc |= vin[j[q]];
        ++checks;
      }
      p += 4;
    }
    if ((acc & need) != need && lim < end) {
      const int slot = atomicAdd(&sh.nlong, 1);
      if (slot < kMbLong) {
        sh.lng[slot] = uint16_t(r);
        sh.lacc[slot] = acc;
        continue;
      }
      for (int32_t q = lim; q < end && (acc & need) != need; ++q) {  // wave list full: finish here
        acc |= vin[a.rowind[q]];
        ++checks;
      }
    }
    finish(r, m, acc & need);
  }
  __syncthreads();
  const int32_t nlong = min(sh.nlong, kMbLong);
  for (int32_t i = tid >> 6; i < nlong; i += kThreads / 64) {
    const int r = sh.lng[i];
    const int32_t v = v0 + r;
    const uint64_t m = vin[v];
    const uint64_t need = ~m & active;
    const int32_t beg = a.colptr[v] + kMbMid, end = a.colptr[v + 1];
    uint64_t acc = sh.lacc[i];
    unsigned long long n = 0;
    for (int32_t p = beg; p < end; p += 64) {
      const int32_t q = p + lane();
      const uint64_t x = q < end ? vin[a.rowind[q]] : 0ull;
      acc |= wave_or64(x);
      n += uint64_t(min(64, end - p));
      if ((acc & need) == need) break;
    }
    if (lane() == 0) {
      checks += n;
      finish(r, m, acc & need);
    }
  }
  __syncthreads();
  if (tid < kMbTileWords && w0 + tid < a.nwords) a.nzF[w0 + tid] = sh.nzf[tid];
  unsigned long long v4[4] = {nvert, nbits, checks, mnew};
  block_sum4(v4);
  unsigned long long i4[4] = {insub, 0, 0, 0};
  block_sum4(i4);
  fbits = block_or64(fbits);
  if (tid == 0) {
    stripe_add(&a.ctrl->slot[L % kSlots], v4[0], v4[1], v4[2], v4[3], i4[0]);
    stripe_or(&a.ctrl->slot[L % kSlots], fbits);
  }
}

// --------------------------------------------------------- level kernels
// First kernel of level L: the state (direction rule on vertex counts and
// edge counts of the whole batch), the previous level's record, and for a
// push level the frontier list with its degree prefix. Before a push level
// adds into the next frontier buffer, the buffer is cleared: densely when it
// is one of this traversal's fresh buffers, else (it holds the frontier of
// two levels back) sparsely through that level's list when it has one.
__global__ __launch_bounds__(kThreads) void k_mb_prep(BatchArgs a, int32_t L, int32_t forced) {
  Ctrl* c = a.ctrl;
  LevelTotals tot;
  LevelState prev;
  const LevelState st = level_state(a, L, forced, &tot, &prev);
  publish_level(c, L, st, prev, tot);
  if (st.done || st.dir != 0) return;
  uint64_t* Fn = mb_frontier(a, L + 1);
  {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (mb_frontier_recycled(L + 1) && (prev.list_valid || prev.dir == 0)) {
      // a push level always had its frontier as a list
      const int32_t* Qp = a.Q[(L + 1) % 2];
      for (int64_t i = t0; i < prev.nf; i += stride) Fn[Qp[i]] = 0;
    } else {
      for (int64_t v = t0; v < a.V; v += stride) Fn[v] = 0;
    }
  }
  uint32_t* mf_out = &c->mf[L % kSlots];
  if (st.list_valid) {
    scan_list(a.Q[L % 2], st.nf, a.rowptr, a.S, a.R, a.chunk_first, a.flagsA, uint32_t(2 * L + 1),
              &c->ticket[L % 2], mf_out);
  } else {
    ScanBitsArgs sb{};
    sb.a = a.nzF;
    sb.b_not = nullptr;
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
    scan_bits(sb);
  }
}

union MbShared {
  MbExpandShared e;
  MbPullShared p;
};

__global__ __launch_bounds__(kThreads) void k_mb_main(BatchArgs a, int32_t L) {
  __shared__ MbShared sh;
  const LevelState st = a.ctrl->ring[L % kRing];
  if (st.done) return;
  if (st.dir == 0) {
    mb_expand_body(a, L, st, sh.e);
  } else {
    const int32_t ntiles = (a.nwords + kMbTileWords - 1) / kMbTileWords;
    for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
      __syncthreads();  // LDS of the previous tile is no longer read
      mb_pull_body(a, L, st, t, sh.p);
    }
  }
}

// rows.row[b][v] = level at which source b reached v, or -1: 64 vertices per
// block step. The kept frontier words of levels below kMbSnap give those
// depths: bit b of level L's word. Four threads per vertex fold the vertex's
// kept words into bit planes of the depth (plane i = OR of the words of the
// levels with bit i set; each reached pair sits in exactly one level's word)
// and write 16 entries each of the block's [v][k] level table in LDS, 0xffff
// where the source never reached the vertex; the level table in memory is
// read only for pairs first reached at level kMbSnap or later. The depth
// rows are then written as coalesced runs, four vertices per 16-byte store.
constexpr int kMbDepthV = 64;
static_assert(kMbSnap <= 16, "depths of the kept levels are folded into four bit planes");
static_assert(kThreads == 4 * kMbDepthV, "four threads per vertex of a block step");
__global__ __launch_bounds__(kThreads) void k_mb_depth(BatchArgs a, int32_t level, DepthRows rows) {
  __shared__ __align__(16) uint16_t s_l[kMbDepthV * kMaxSources];
  const LevelState end = a.ctrl->ring[level % kRing];
  if (!end.done) return;  // not over yet: a later batch's transpose writes the rows
  const uint64_t* vis = a.vis[end.vis_idx];
  const int32_t k = a.k;
  const int32_t nsnap = min(end.levels, kMbSnap);  // kept frontiers: levels 0 .. nsnap-1
  const int64_t nblk = (int64_t(a.V) + kMbDepthV - 1) / kMbDepthV;
  const int32_t j = threadIdx.x >> 2, b0 = (threadIdx.x & 3) * 16;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t v0 = blk * kMbDepthV;
    const int32_t nv = int32_t(min(int64_t(kMbDepthV), int64_t(a.V) - v0));
    __syncthreads();  // the previous step's table is no longer read
    if (j < nv && b0 < k) {
      const int64_t v = v0 + j;
      const uint64_t reached = vis[v];
      uint64_t kept = 0, p0 = 0, p1 = 0, p2 = 0, p3 = 0;
#pragma unroll
      for (int32_t L = 0; L < kMbSnap; ++L) {
        if (L < nsnap) {
          const uint64_t f = a.Fs[int64_t(L) * a.V + v];  // mb_frontier(a, L)
          kept |= f;
          if (L & 1) p0 |= f;
          if (L & 2) p1 |= f;
          if (L & 4) p2 |= f;
          if (L & 8) p3 |= f;
        }
      }
      const uint64_t deep = reached & ~kept;
      const int32_t nb = min(16, k - b0);
      const bool vec = nb == 16 && (k % 8) == 0;  // this thread's 16 entries are one aligned 32-byte piece
      union Piece {
        uint4 x[2];
        uint16_t h[16];
      };
      Piece lv, d;
      lv.x[0] = lv.x[1] = make_uint4(0u, 0u, 0u, 0u);
      const uint16_t* lrow = a.lvl + v * k + b0;
      if ((deep >> b0) & 0xffffull) {  // some of these pairs were reached at a level >= kMbSnap
        if (vec) {
          lv.x[0] = reinterpret_cast<const uint4*>(lrow)[0];
          lv.x[1] = reinterpret_cast<const uint4*>(lrow)[1];
        } else {
#pragma unroll
          for (int32_t q = 0; q < 16; ++q)
            if (q < nb) lv.h[q] = lrow[q];
        }
      }
#pragma unroll
      for (int32_t q = 0; q < 16; ++q) {
        const int32_t b = b0 + q;
        uint16_t x = 0xffff;
        if ((deep >> b) & 1ull) {
          x = lv.h[q];
        } else if ((reached >> b) & 1ull) {
          x = uint16_t(((p0 >> b) & 1ull) | (((p1 >> b) & 1ull) << 1) | (((p2 >> b) & 1ull) << 2) |
                       (((p3 >> b) & 1ull) << 3));
        }
        d.h[q] = x;
      }
      uint16_t* dst = s_l + j * k + b0;
      if (vec) {
        reinterpret_cast<uint4*>(dst)[0] = d.x[0];
        reinterpret_cast<uint4*>(dst)[1] = d.x[1];
      } else {
#pragma unroll
        for (int32_t q = 0; q < 16; ++q)
          if (q < nb) dst[q] = d.h[q];
      }
    }
    __syncthreads();
    auto depth_at = [&](int32_t i) -> int32_t {
      const uint16_t d = s_l[i];
      return d == 0xffff ? -1 : int32_t(d);
    };
    if (nv == kMbDepthV) {
      // four consecutive vertices of one depth row per item: one 16-byte store where the row allows
      constexpr int kQ = kMbDepthV / 4;
      for (int32_t it = threadIdx.x; it < k * kQ; it += kThreads) {
        const int32_t b = it / kQ, jj = (it % kQ) * 4;
        int32_t d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = depth_at((jj + q) * k + b);
        int32_t* out = rows.row[b] + v0 + jj;
        if ((reinterpret_cast<uintptr_t>(out) & 15) == 0) {
          *reinterpret_cast<int4*>(out) = make_int4(d[0], d[1], d[2], d[3]);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) out[q] = d[q];
        }
      }
    } else {
      for (int32_t i = threadIdx.x; i < nv * k; i += kThreads) {
        const int32_t b = i / nv, jj = i - b * nv;
        rows.row[b][v0 + jj] = depth_at(jj * k + b);
      }
    }
  }
}

}  // namespace

hipError_t launch_mb_init(hipStream_t s, const BatchArgs& a, int32_t dir0, int64_t nflags, hipEvent_t t0,
                         hipEvent_t t1) {
  const int64_t n = std::max<int64_t>(a.V, nflags);
  const unsigned g = unsigned(std::min<int64_t>((n + kThreads - 1) / kThreads, 8192));
  return launch_k(k_mb_init, dim3(g > 0 ? g : 1), s, t0, t1, a, dir0, nflags);
}

hipError_t launch_mb_prep(hipStream_t s, const BatchArgs& a, int32_t level, int32_t forced_dir,
                         hipEvent_t t0, hipEvent_t t1) {
  return launch_k(k_mb_prep, dim3(unsigned(scan_grid(a.V))), s, t0, t1, a, level, forced_dir);
}

hipError_t launch_mb_main(hipStream_t s, const BatchArgs& a, int32_t level, hipEvent_t t0, hipEvent_t t1) {
  const int64_t tiles = (int64_t(a.nwords) + kMbTileWords - 1) / kMbTileWords;
  const dim3 g(unsigned(std::max<int64_t>(kExpandBlocks, tiles)));
  return launch_k(k_mb_main, g, s, t0, t1, a, level);
}

hipError_t launch_mb_depth(hipStream_t s, const BatchArgs& a, int32_t level, const DepthRows& rows) {
  const int64_t nblk = (int64_t(a.V) + kMbDepthV - 1) / kMbDepthV;
  const unsigned g = unsigned(std::min<int64_t>(nblk, 4096));
  hipLaunchKernelGGL(k_mb_depth, dim3(g > 0 ? g : 1), dim3(kThreads), 0, s, a, level, rows);
  return hipGetLastError();
}

}  // namespace dobfs
