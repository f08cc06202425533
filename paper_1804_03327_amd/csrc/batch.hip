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
// Levels run as steps, one launch each, as in the single-source path: a pull
// level is one step, a push level two (the scan step lists the frontier
// vertices with their degree prefix, the expansion step pushes). Every block
// of a step derives the step's state from the state the step before published
// and the counters it left, so the direction is decided on the device inside
// the level's own kernel. The frontier
// words of a level are exactly the (vertex, source) pairs first reached at
// that level, so those of the first kMbSnap levels are kept and are the depth
// record; deeper levels stamp a vertex-major [V][k] uint16 level table.
// mb_depth turns both into the [k][V] int32 depth rows at the end.

#include "device_common.h"

namespace dobfs {
namespace {

__device__ __forceinline__ uint64_t* mb_frontier(const BatchArgs& a, int32_t L) {
  return a.Fs + int64_t(mb_frontier_slot(L)) * a.fstride;
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
// Visited and level-0/1 frontier words start cleared (16-byte stores), then
// take the source bits (depth 0): bit b of Vis and of level 0's frontier at
// sources[b]. The thread that cleared a source's pair of words sets its bit,
// after its own clear, so no other thread's store can come between. The
// control block starts level 0 (a push whose list is the distinct sources,
// unless the level is forced to pull).
__global__ __launch_bounds__(kThreads) void k_mb_init(BatchArgs a, int32_t dir0, int64_t nflags) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const ulonglong2 z = make_ulonglong2(0ull, 0ull);
  ulonglong2* vis2 = reinterpret_cast<ulonglong2*>(a.vis[0]);
  ulonglong2* f0 = reinterpret_cast<ulonglong2*>(a.Fs);              // mb_frontier(a, 0)
  ulonglong2* f1 = reinterpret_cast<ulonglong2*>(a.Fs + a.fstride);  // mb_frontier(a, 1)
  const int64_t npair = int64_t(a.V) / 2;
  for (int64_t i = t0; i < npair; i += stride) {
    vis2[i] = z;
    f0[i] = z;
    f1[i] = z;
  }
  if ((a.V & 1) && t0 == 0) {
    a.vis[0][a.V - 1] = 0ull;
    a.Fs[a.V - 1] = 0ull;
    a.Fs[a.fstride + a.V - 1] = 0ull;
  }
  // The grid is a power of two, so the thread that cleared pair i is i mod stride (pair
  // npair is the last vertex of an odd V, which thread 0 cleared). Lane b of every wave takes
  // source b and the wave picks out the sources whose clearing thread is one of its own lanes;
  // those few are set one by one, each by its clearing lane.
  const int64_t mask = stride - 1;
  auto owner_of = [&](int32_t v) -> int64_t {
    const int64_t pair = int64_t(v) / 2;
    return pair < npair ? (pair & mask) : 0;
  };
  const int ln = lane();
  const int32_t sv = ln < a.k ? a.src[ln] : 0;
  uint64_t here = __ballot(ln < a.k && (owner_of(sv) >> 6) == (t0 >> 6));
  while (here) {
    const int b = __ffsll((unsigned long long)here) - 1;
    here &= here - 1;
    const int32_t v = __shfl(sv, b, 64);
    if (owner_of(v) == t0) {
      a.vis[0][v] |= 1ull << b;
      a.Fs[v] |= 1ull << b;
    }
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
      c->bar.abort = 0;  // the persistent loop's grid barrier starts idle
      c->bar.t_end = 0;
      c->bar.gen = 0;
      c->bar.top.n = 0;
      for (int g = 0; g < kBarGroups; ++g) c->bar.group[g].n = 0;
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
      st.phase = dir0 == 0 ? kPhaseScan : kPhaseWhole;
      st.m_u = a.nnz;  // in-edges of vertices some source has not reached yet
      st.active = a.active;
      st.t0 = 0;
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
// adjacency carries F[u]'s source bits to w. The bits w had not seen when the
// level began are claimed with one 64-bit atomicOr on w's next-frontier word
// (Vis is not written during the level: the next frontier is exactly what it
// gains, merged in by the next level's first step); the bits a thread newly set are
// its own to count, and the thread whose add made the word nonzero lists w
// for the next level. The chunked, load-balanced walk over the edges is the
// one of the single-source expansion.
// The expansion step s of level st.level: m_f from the scan step before it, counters into
// slot s.
__device__ __forceinline__ void mb_expand_body(const BatchArgs& a, const LevelState& st, int32_t s, MbExpandShared& sh) {
  const int32_t L = st.level;
  const int32_t nf = st.nf;
  const uint32_t m = a.ctrl->mf[s % kSlots];
  if (nf <= 0 || m == 0) return;
  const uint32_t nchunks = (m + kExpandChunk - 1) / kExpandChunk;
  if (blockIdx.x >= nchunks) return;
  const int32_t* Q = a.Q[L % 2];
  int32_t* Qout = a.Q[(L + 1) % 2];
  const uint64_t* Fc = mb_frontier(a, L);
  uint64_t* Fn = mb_frontier(a, L + 1);
  uint64_t* vis = a.vis[st.vis_idx];
  uint32_t* qcount = &a.ctrl->qcount[s % kSlots];
  uint32_t* nzn = a.nzF[(L + 1) % 2];
  const bool marks = mb_push_marks(m);  // winners go to the non-zero bitmap, not the list
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
    if (!marks && sh.nbuf + kExpandChunk > kExpandBuf) flush();
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
    uint64_t x[kExpandEPT], seen[kExpandEPT];
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) w[t] = valid[t] ? a.colind[pos[t]] : 0;
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      seen[t] = valid[t] ? vis[w[t]] : ~0ull;
      x[t] = valid[t] ? (Fc[u[t]] & active & ~seen[t]) : 0ull;
    }
    bool listed[kExpandEPT];
#pragma unroll
    for (int t = 0; t < kExpandEPT; ++t) {
      listed[t] = false;
      if (x[t]) {
        // the next frontier word collects exactly the bits w gains at this level, so it is the
        // only word claimed here; the visited words take them in the next level's first step
        const uint64_t oldf = atomicOr((unsigned long long*)(Fn + w[t]), (unsigned long long)x[t]);
        const uint64_t nb = x[t] & ~oldf;
        if (nb) {
          stamp_levels(a.lvl, a.k, w[t], nb, L);
          nbits += uint64_t(__popcll(nb));
          fbits |= nb;
          if (oldf == 0) {
            listed[t] = !marks;
            if (marks) atomicOr(nzn + (w[t] >> 5), 1u << (w[t] & 31));
            ++nvert;
            if (a.edge_rule) mnew += uint64_t(a.rowptr[w[t] + 1] - a.rowptr[w[t]]);
          }
          if (a.edge_rule && ((seen[t] | oldf | nb) & active) == active)  // this claim completed w
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
  if (!marks) flush();
  unsigned long long v4[4] = {nvert, nbits, mnew, insub};
  block_sum4(v4);
  fbits = block_or64(fbits);
  if (threadIdx.x == 0) {
    stripe_or(&a.ctrl->slot[s % kSlots], fbits);
    unsigned long long edges = 0;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x)
      edges += min(uint32_t(kExpandChunk), m - c * kExpandChunk);
    stripe_add(&a.ctrl->slot[s % kSlots], v4[0], v4[1], edges, v4[2], v4[3]);
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
// bits are written whole; no atomics touch them. Step s's counters go to slot s.
__device__ __forceinline__ void mb_pull_body(const BatchArgs& a, const LevelState& st, int32_t s, int32_t tile,
                             MbPullShared& sh) {
  const int tid = threadIdx.x;
  const int32_t L = st.level;
  const int32_t w0 = tile * kMbTileWords;
  const int32_t v0 = w0 * 32;
  const uint64_t* vin = a.vis[st.vis_idx];
  uint64_t* vout = a.vis[st.vis_idx ^ 1];
  uint64_t* Fn = mb_frontier(a, L + 1);
  const uint64_t active = st.active;  // a source with an empty frontier finds nothing more
  // after a push, vin lacks this level's frontier words (the merge is left to this pull):
  // a row's own word is vin | Fc, and the in-neighbours' words are read from Fc, which for
  // every source bit a row still needs holds the same bits as the merged words (a source's
  // visited in-neighbour of a row it has not reached was reached at this level, Section 5.4)
  const bool merge = st.local == 1;
  const uint64_t* Fc = mb_frontier(a, L);
  const uint64_t* xin = merge ? Fc : vin;
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
      const uint64_t m = merge ? (vin[v] | Fc[v]) : vin[v];
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
    const uint64_t m = merge ? (vin[v] | Fc[v]) : vin[v];
    const uint64_t need = ~m & active;
    // the slab: the row's first kSlab in-neighbours from one coalesced read
    const int4 hd = a.slab[v];
    const int32_t e[kSlab] = {hd.x, hd.y, hd.z, hd.w};
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < kSlab; ++q) {
      if (e[q] >= 0) {
        acc |= xin[e[q]];
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
        acc |= xin[j[q]];
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
        acc |= xin[a.rowind[q]];
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
    const uint64_t m = merge ? (vin[v] | Fc[v]) : vin[v];
    const uint64_t need = ~m & active;
    const int32_t beg = a.colptr[v] + kMbMid, end = a.colptr[v + 1];
    uint64_t acc = sh.lacc[i];
    unsigned long long n = 0;
    for (int32_t p = beg; p < end; p += 64) {
      const int32_t q = p + lane();
      const uint64_t x = q < end ? xin[a.rowind[q]] : 0ull;
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
  if (tid < kMbTileWords && w0 + tid < a.nwords) a.nzF[(L + 1) % 2][w0 + tid] = sh.nzf[tid];
  unsigned long long v4[4] = {nvert, nbits, checks, mnew};
  block_sum4(v4);
  unsigned long long i4[4] = {insub, 0, 0, 0};
  block_sum4(i4);
  fbits = block_or64(fbits);
  if (tid == 0) {
    stripe_add(&a.ctrl->slot[s % kSlots], v4[0], v4[1], v4[2], v4[3], i4[0]);
    stripe_or(&a.ctrl->slot[s % kSlots], fbits);
  }
}

// ---------------------------------------------------------- step loop
// One launch per step. Every block derives step s's state from the state step
// s-1 published and the counters it left (one round trip): the expansion that
// a scan step prepared, or a new level, whose direction the rule of Section
// 6.3 (or the edge form) decides on the counts of the whole batch. The
// counters of step s gather in slot s % kSlots; step s clears slot
// (s + 2) % kSlots, which nothing touches until step s + 2.
__device__ __forceinline__ LevelState mb_step_state(const BatchArgs& a, int32_t s, LevelTotals* tot,
                                                    LevelState* prev_out, bool* new_level) {
  const Ctrl* c = a.ctrl;
  *new_level = false;
  *tot = LevelTotals{0, 0, 0, 0, 0, 0};
  if (s == 0) {  // level 0 as the init kernel left it
    const LevelState st = c->ring[0];
    *prev_out = st;
    return st;
  }
  // (the counters' loads are left where the compiler puts them, after the state's: holding
  // them from the start costs this kernel registers, 6 waves per SIMD instead of 7)
  const StripeLanes x = load_stripes(c->slot[(s - 1) % kSlots]);
  const LevelState prev = c->ring[(s - 1) % kRing];
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
  LevelState st = next_state(a, L, forced, prev, x, (s - 1) % kSlots, tot);
  // a pull after a push merges the push's winners into the visited words itself
  st.local = (!st.done && st.dir == 1 && prev.dir == 0) ? 1 : 0;
  return st;
}

// The scan step of push level L = st.level (prev: the state of level L-1). A push leaves Vis
// as its level began, so before another push what it found is merged in, through its list
// when it made a short one, else in one dense pass (random lines of two arrays cost more than
// a sweep). The next frontier's buffer and non-zero bitmap are cleared: the buffer densely
// when it is one of this traversal's fresh buffers, else (it holds the frontier of two levels
// back) sparsely through that level's list. Then the frontier list with its degree prefix
// (Section 6.2), from the list the push before left or from the non-zero bitmap; m_f goes
// where the expansion step reads it.
__device__ __forceinline__ void mb_scan_step(const BatchArgs& a, const LevelState& st, const LevelState& prev, int32_t s) {
  Ctrl* c = a.ctrl;
  const int32_t L = st.level;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (L >= 1 && prev.dir == 0) {
    const int32_t* Qc = a.Q[L % 2];
    const uint64_t* Fc = mb_frontier(a, L);
    uint64_t* vis = a.vis[st.vis_idx];
    if (!st.list_valid || int64_t(st.nf) * kMbDenseMerge >= int64_t(a.V)) {
      const ulonglong2* F2 = reinterpret_cast<const ulonglong2*>(Fc);
      ulonglong2* V2 = reinterpret_cast<ulonglong2*>(vis);
      const int64_t n2 = int64_t(a.V) / 2;
      for (int64_t i = t0; i < n2; i += stride) {
        const ulonglong2 f = F2[i];
        if (f.x | f.y) {
          ulonglong2 m = V2[i];
          m.x |= f.x;
          m.y |= f.y;
          V2[i] = m;
        }
      }
      if ((a.V & 1) && t0 == 0) vis[a.V - 1] |= Fc[a.V - 1];
    } else {
      constexpr int kU = 4;  // independent entries per thread in flight
      for (int64_t i0 = t0; i0 < st.nf; i0 += stride * kU) {
        int32_t v[kU];
        uint64_t f[kU], m[kU];
#pragma unroll
        for (int q = 0; q < kU; ++q) v[q] = i0 + q * stride < st.nf ? Qc[i0 + q * stride] : -1;
#pragma unroll
        for (int q = 0; q < kU; ++q) {
          f[q] = v[q] >= 0 ? Fc[v[q]] : 0ull;
          m[q] = v[q] >= 0 ? vis[v[q]] : 0ull;
        }
#pragma unroll
        for (int q = 0; q < kU; ++q)
          if (v[q] >= 0) vis[v[q]] = m[q] | f[q];
      }
    }
  }
  {  // the non-zero bitmap of the next frontier, in case this push marks its winners there
    uint32_t* nzn = a.nzF[(L + 1) % 2];
    for (int32_t w = blockIdx.x * kThreads + threadIdx.x; w < a.nwords; w += gridDim.x * kThreads) nzn[w] = 0;
  }
  uint64_t* Fn = mb_frontier(a, L + 1);
  if (L >= 1) {  // level 1's buffer is cleared by the init kernel
    if (mb_frontier_recycled(L + 1) && (prev.list_valid || prev.dir == 0)) {
      // a push level always had its frontier as a list
      const int32_t* Qp = a.Q[(L + 1) % 2];
      for (int64_t i = t0; i < prev.nf; i += stride) Fn[Qp[i]] = 0;
    } else {  // 16-byte stores: the buffer is 256-byte aligned and padded to an even length
      ulonglong2* F2 = reinterpret_cast<ulonglong2*>(Fn);
      const ulonglong2 z = make_ulonglong2(0ull, 0ull);
      for (int64_t i = t0; i < (int64_t(a.V) + 1) / 2; i += stride) F2[i] = z;
    }
  }
  uint32_t* mf_out = &c->mf[(s + 1) % kSlots];
  if (st.list_valid) {
    scan_list(a.Q[L % 2], st.nf, a.rowptr, a.S, a.R, a.chunk_first, a.flagsA, uint32_t(2 * s + 1),
              &c->ticket[s % 2], mf_out);
  } else {
    ScanBitsArgs sb{};
    sb.a = a.nzF[L % 2];
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
    sb.epochA = uint32_t(2 * s + 1);
    sb.epochB = uint32_t(2 * s + 2);
    sb.ticket = &c->ticket[s % 2];
    sb.nf_out = &c->nf32;
    sb.mf_out = mf_out;
    scan_bits(sb);
  }
}

union MbShared {
  MbExpandShared e;
  MbPullShared p;
};

// The work of step s (state st, prev: the state before it) over the launch's grid.
__device__ __forceinline__ void mb_step_body(const BatchArgs& a, const LevelState& st, const LevelState& prev,
                                             int32_t s, MbShared& sh) {
  if (st.phase == kPhaseScan) {
    mb_scan_step(a, st, prev, s);
  } else if (st.dir == 0) {
    mb_expand_body(a, st, s, sh.e);
  } else {
    const int32_t ntiles = (a.nwords + kMbTileWords - 1) / kMbTileWords;
    for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
      __syncthreads();  // LDS of the previous tile is no longer read
      mb_pull_body(a, st, s, t, sh.p);
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_mb_step(BatchArgs a, int32_t s) {
  __shared__ MbShared sh;
  LevelTotals tot;
  LevelState prev;
  bool new_level;
  const LevelState st = mb_step_state(a, s, &tot, &prev, &new_level);
  if (blockIdx.x == 0) publish_step(a.ctrl, s, st, prev, tot, new_level);
  if (st.done) return;
  mb_step_body(a, st, prev, s, sh);
}

// The persistent form of the step loop: steps s_first .. s_first + n - 1 in
// one launch of co-resident blocks, a grid barrier between consecutive steps
// in place of a kernel boundary. Every body already strides over the grid it
// is given (expansion chunks, pull tiles, scan tiles by ticket), so the blocks
// run each step's body once. Block 0 publishes every state (with its start
// time when timing); when the traversal ends early the launch's remaining
// states read as the final one, as steps enqueued past the end publish it.
// A barrier wait that gives up raises the abort flag, which the report
// passes on; every block then leaves.
__global__ __launch_bounds__(kThreads) void k_mb_steps(BatchArgs a, int32_t s_first, int32_t n, uint32_t spin_limit,
                                                       int32_t timing) {
  __shared__ MbShared sh;
  __shared__ uint32_t s_gen;
  GridBar* bar = &a.ctrl->bar;
  if (threadIdx.x == 0)  // no barrier of this traversal is in progress between launches
    s_gen = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const uint32_t gen0 = s_gen;
  for (int32_t k = 0; k < n; ++k) {
    const int32_t s = s_first + k;
    LevelTotals tot;
    LevelState prev;
    bool new_level;
    LevelState st = mb_step_state(a, s, &tot, &prev, &new_level);
    if (blockIdx.x == 0) {
      if (timing) st.t0 = wall_clock64();
      publish_step(a.ctrl, s, st, prev, tot, new_level);
      if (st.done)
        for (int32_t j = 1 + int32_t(threadIdx.x); j < n - k; j += kThreads) a.ctrl->ring[(s + j) % kRing] = st;
    }
    if (st.done) break;
    __syncthreads();  // LDS of the previous step is no longer read
    mb_step_body(a, st, prev, s, sh);
    if (k == n - 1) break;  // the kernel boundary ends the last step
    if (!grid_barrier(bar, gen0 + uint32_t(k) + 1u, spin_limit)) break;
  }
  if (timing) {
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_max(&bar->t_end, (unsigned long long)wall_clock64(), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

// rows.row[b][v] = level at which source b reached v, or -1. A thread takes
// four consecutive vertices and folds their kept frontier words (levels below
// kMbSnap: bit b of level L's word) into bit planes of the depth, plane i
// being the OR of the words of the levels with bit i set (each reached pair
// sits in exactly one level's word). It then walks the sources, writing each
// depth row's four entries with one 16-byte non-temporal store, so a wave
// writes 1 KB runs of a row. The level table in memory is read, eight entries at a time,
// only where a pair was first reached at level kMbSnap or later.
constexpr int kMbDepthVPT = 4;
static_assert(kMbSnap <= 16, "depths of the kept levels are folded into four bit planes");
__global__ __launch_bounds__(kThreads) void k_mb_depth(BatchArgs a, int32_t step, DepthRows rows) {
  const LevelState end = a.ctrl->ring[step % kRing];
  if (!end.done) return;  // not over yet: a later batch's transpose writes the rows
  // the final visited words: the state that found the end keeps the last level's direction and
  // buffer index, and a last pull wrote its result to the other buffer (merged with what the push
  // before it found, which its input may lack)
  const uint64_t* vis = a.vis[end.dir == 1 ? (end.vis_idx ^ 1) : end.vis_idx];
  const int32_t k = a.k;
  const int32_t nsnap = min(end.levels, kMbSnap);  // kept frontiers: levels 0 .. nsnap-1
  const int64_t ngroups = (int64_t(a.V) + kMbDepthVPT - 1) / kMbDepthVPT;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < ngroups; g += stride) {
    const int64_t v0 = g * kMbDepthVPT;
    const int32_t nv = int32_t(min(int64_t(kMbDepthVPT), int64_t(a.V) - v0));
    uint64_t reached[4], kept[4], p0[4], p1[4], p2[4], p3[4];
    // v0 is a multiple of 4 and every word array is 256-byte aligned: two 16-byte loads each
    auto load4 = [&](const uint64_t* base, uint64_t out[4]) {
      if (nv == 4) {
        const ulonglong2 x = reinterpret_cast<const ulonglong2*>(base + v0)[0];
        const ulonglong2 y = reinterpret_cast<const ulonglong2*>(base + v0)[1];
        out[0] = x.x; out[1] = x.y; out[2] = y.x; out[3] = y.y;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = q < nv ? base[v0 + q] : 0ull;
      }
    };
    load4(vis, reached);
#pragma unroll
    for (int q = 0; q < 4; ++q) kept[q] = p0[q] = p1[q] = p2[q] = p3[q] = 0ull;
#pragma unroll
    for (int32_t L = 0; L < kMbSnap; ++L) {
      if (L < nsnap) {
        uint64_t f[4];
        load4(a.Fs + int64_t(L) * a.fstride, f);  // mb_frontier(a, L)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          kept[q] |= f[q];
          if (L & 1) p0[q] |= f[q];
          if (L & 2) p1[q] |= f[q];
          if (L & 4) p2[q] |= f[q];
          if (L & 8) p3[q] |= f[q];
        }
      }
    }
    uint64_t deep[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) deep[q] = reached[q] & ~kept[q];
    const bool any_deep = (deep[0] | deep[1] | deep[2] | deep[3]) != 0ull;
    for (int32_t b8 = 0; b8 < k; b8 += 8) {
      union Piece {
        uint4 x;
        uint16_t h[8];
      };
      Piece lv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        lv[q].x = make_uint4(0u, 0u, 0u, 0u);
        if (any_deep && ((deep[q] >> b8) & 0xffull)) {  // some pair reached at a level >= kMbSnap
          const uint16_t* row = a.lvl + (v0 + q) * k + b8;
          if ((k % 8) == 0) {
            lv[q].x = *reinterpret_cast<const uint4*>(row);
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
              if (b8 + j < k) lv[q].h[j] = row[j];
          }
        }
      }
#pragma unroll
      for (int32_t j = 0; j < 8; ++j) {
        const int32_t b = b8 + j;
        if (b >= k) break;
        int32_t d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t plane = uint32_t((p0[q] >> b) & 1ull) | (uint32_t((p1[q] >> b) & 1ull) << 1) |
                                 (uint32_t((p2[q] >> b) & 1ull) << 2) | (uint32_t((p3[q] >> b) & 1ull) << 3);
          d[q] = !((reached[q] >> b) & 1ull) ? -1 : (((deep[q] >> b) & 1ull) ? int32_t(lv[q].h[j]) : int32_t(plane));
        }
        int32_t* out = rows.row[b] + v0;
        if (nv == 4 && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
          // non-temporal: the rows are the call's output, not read again on the device, and
          // 256 MB of them left in the caches would evict what the next traversal works on
          typedef int32_t v4i __attribute__((ext_vector_type(4)));
          const v4i x = {d[0], d[1], d[2], d[3]};
          __builtin_nontemporal_store(x, reinterpret_cast<v4i*>(out));
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (q < nv) out[q] = d[q];
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_mb_init(hipStream_t s, const BatchArgs& a, int32_t dir0, int64_t nflags, hipEvent_t t0,
                         hipEvent_t t1) {
  const int64_t n = std::max<int64_t>(int64_t(a.V) / 2 + 1, nflags);
  const int64_t want = std::min<int64_t>((n + kThreads - 1) / kThreads, 8192);
  unsigned g = 1;  // a power of two (the kernel finds a source's clearing thread with a mask)
  while (int64_t(g) < want) g *= 2;
  return launch_k(k_mb_init, dim3(g), s, t0, t1, a, dir0, nflags);
}

// By default a block per pull tile, at most 8192: every block of every step derives the step's
// state first, which on graphs of millions of vertices costs more than a second tile per block.
hipError_t launch_mb_step(hipStream_t s, const BatchArgs& a, int32_t step, int64_t blocks, hipEvent_t t0,
                          hipEvent_t t1) {
  const int64_t tiles = (int64_t(a.nwords) + kMbTileWords - 1) / kMbTileWords;
  const int64_t full = std::max<int64_t>(kExpandBlocks, std::min<int64_t>(tiles, 8192));
  const dim3 g(unsigned(blocks > 0 && blocks < full ? blocks : full));
  return launch_k(k_mb_step, g, s, t0, t1, a, step);
}

hipError_t launch_mb_steps(hipStream_t s, const BatchArgs& a, int32_t s_first, int32_t n, int32_t blocks,
                           uint32_t spin_limit, bool timing, hipEvent_t t0, hipEvent_t t1) {
  return launch_k(k_mb_steps, dim3(static_cast<unsigned>(blocks)), s, t0, t1, a, s_first, n, spin_limit,
                  int32_t(timing ? 1 : 0));
}

hipError_t persistent_capacity_mb(int32_t* blocks) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_mb_steps, kThreads, 0);
  if (e != hipSuccess) return e;
  *blocks = cus * per;
  return hipSuccess;
}

hipError_t launch_mb_depth(hipStream_t s, const BatchArgs& a, int32_t step, const DepthRows& rows) {
  const int64_t groups = (int64_t(a.V) + kMbDepthVPT - 1) / kMbDepthVPT;
  const unsigned g = unsigned(std::min<int64_t>((groups + kThreads - 1) / kThreads, 4096));
  hipLaunchKernelGGL(k_mb_depth, dim3(g > 0 ? g : 1), dim3(kThreads), 0, s, a, step, rows);
  return hipGetLastError();
}

}  // namespace dobfs
