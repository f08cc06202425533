// Sort-based push BFS of libdobfs (modes DOBFS_MODE_PUSH_SORT and _KEYS): the
// column-based masked matvec the way Algorithm 3 prints it and Table 2's
// "Baseline" row measures it. Every level gathers the frontier's adjacency
// lists as (neighbour, frontier vertex) pairs, sorts them by neighbour with a
// key-value radix sort (rocPRIM's device radix sort, as the paper uses CUB's),
// keeps the first pair of every run of equal keys (the segmented reduce that
// merges duplicates) and filters it by the mask not(visited). The winner of a
// run is the parent. The host reads each level's frontier and edge counts
// back, as the paper's loop does, since the sort takes its size on the host.
// The key-only form (Table 2's "Structure only") gathers the neighbours alone,
// sorts keys only and keeps each distinct key: depths without parents.
// Kept for the ablation; the default push merges by atomic claim instead.

#include <algorithm>
#include <cstring>

#include "device_common.h"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

namespace dobfs {
namespace {

// The gather step: edge e of the concatenated expansion becomes
// (colind[e'], frontier vertex). Chunks and their windows are those of the
// frontier scan, as in the atomic push.
struct GatherShared {
  int32_t sS[kExpandWin], sR[kExpandWin], sQ[kExpandWin];
};

__global__ __launch_bounds__(kThreads) void k_sort_gather(ExpandArgs a, uint32_t* keys, int32_t* vals) {
  __shared__ GatherShared sh;
  const int32_t nf = a.nf;
  const uint32_t m = a.m;
  if (nf <= 0 || m == 0) return;
  const uint32_t nchunks = (m + kExpandChunk - 1) / kExpandChunk;
  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const uint32_t e0 = c * kExpandChunk;
    const uint32_t e1 = min(e0 + uint32_t(kExpandChunk), m);
    const int32_t k0 = a.chunk_first[c];
    const int32_t k1 = (c + 1 < nchunks) ? a.chunk_first[c + 1] : nf - 1;
    const int32_t n = k1 - k0 + 1;
    const bool in_lds = n <= kExpandWin;
    __syncthreads();
    if (in_lds) {
      for (int32_t i = threadIdx.x; i < n; i += kThreads) {
        sh.sS[i] = a.S[k0 + i];
        sh.sR[i] = a.R[k0 + i];
        sh.sQ[i] = a.Q[k0 + i];
      }
    }
    __syncthreads();
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
      int32_t s, rs, u;
      if (in_lds) {
        const int32_t kk = thread_search(sh.sS, 0, n, e);
        s = sh.sS[kk]; rs = sh.sR[kk]; u = sh.sQ[kk];
      } else {
        const int32_t kk = thread_search(a.S, k0, k1 + 1, e);
        s = a.S[kk]; rs = a.R[kk]; u = a.Q[kk];
      }
      keys[e] = uint32_t(a.colind[rs + int32_t(e - uint32_t(s))]);
      if (vals) vals[e] = u;
    }
  }
}

// Segmented reduce + mask filter over the sorted pairs: the first pair of a
// run of equal keys stands for the run (Boolean OR of the run); it survives
// if its key is not visited. Survivors get depth and parent, their visited
// bit, and a place in the next frontier list (buffered per block, one atomic
// per flush).
struct FilterShared {
  int32_t buf[kExpandBuf];
  uint32_t nbuf, base;
};

__global__ __launch_bounds__(kThreads) void k_sort_filter(const uint32_t* keys, const int32_t* vals, uint32_t m,
                                                          uint32_t* vis, int32_t* depth, int32_t* parent,
                                                          int32_t level, int32_t* Qout, uint32_t* qcount,
                                                          LevelSlot* slot) {
  __shared__ FilterShared sh;
  const int tid = threadIdx.x;
  const uint32_t per = (m + gridDim.x - 1) / gridDim.x;  // a contiguous slice per block
  const uint32_t i0 = min(m, blockIdx.x * per), i1 = min(m, i0 + per);
  if (tid == 0) sh.nbuf = 0;
  unsigned long long found = 0;
  auto flush = [&]() {
    const uint32_t nb = sh.nbuf;
    if (nb == 0) return;
    if (tid == 0) sh.base = atomicAdd(qcount, nb);
    __syncthreads();
    const uint32_t b = sh.base;
    for (uint32_t k = tid; k < nb; k += kThreads) Qout[b + k] = sh.buf[k];
    __syncthreads();
    if (tid == 0) sh.nbuf = 0;
    __syncthreads();
  };
  for (uint32_t t0 = i0; t0 < i1; t0 += kThreads) {
    __syncthreads();
    if (sh.nbuf + kThreads > uint32_t(kExpandBuf)) flush();
    const uint32_t i = t0 + tid;
    bool win = false;
    uint32_t k = 0;
    if (i < i1) {
      k = keys[i];
      const bool first = i == 0 || keys[i - 1] != k;
      if (first && !((vis[k >> 5] >> (k & 31)) & 1u)) {
        win = true;
        atomicOr(vis + (k >> 5), 1u << (k & 31));  // keys are unique among survivors; words are shared
        depth[k] = level + 1;
        if (parent) parent[k] = vals[i];
        ++found;
      }
    }
    const uint64_t bal = __ballot(win);
    if (bal) {
      const int leader = __ffsll((unsigned long long)bal) - 1;
      uint32_t p = 0;
      if (lane() == leader) p = atomicAdd(&sh.nbuf, uint32_t(__popcll(bal)));
      p = __shfl(p, leader, 64);
      if (win) sh.buf[p + __popcll(bal & lanemask_lt())] = int32_t(k);
    }
  }
  __syncthreads();
  flush();
  unsigned long long v[4] = {found, 0, 0, 0};
  block_sum4(v);
  if (tid == 0) stripe_add(slot, v[0], 0, uint64_t(i1 - i0), 0, 0);
}

// Sort key of CSC entry p: larger out-degree of its row first (maxdeg - deg).
__global__ __launch_bounds__(kThreads) void k_hub_keys(const int32_t* rowind, const int32_t* rowptr, int64_t nnz,
                                                       uint32_t maxdeg, uint32_t* keys) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < nnz; p += stride) {
    const int32_t r = rowind[p];
    keys[p] = maxdeg - uint32_t(rowptr[r + 1] - rowptr[r]);
  }
}

}  // namespace

hipError_t hubs_first(hipStream_t s, const int32_t* rowptr, const int32_t* colptr, const int32_t* rowind_in,
                      int32_t* rowind_out, int32_t V, int64_t nnz, uint32_t maxdeg) {
  if (nnz <= 0) return hipSuccess;
  int bits = 1;
  while (bits < 32 && (uint64_t(1) << bits) <= maxdeg) ++bits;
  uint32_t *kin = nullptr, *kout = nullptr;
  void* tmp = nullptr;
  size_t tb = 0;
  hipError_t e = hipMalloc(&kin, size_t(nnz) * 4);
  if (e == hipSuccess) e = hipMalloc(&kout, size_t(nnz) * 4);
  if (e == hipSuccess) {
    const unsigned g = unsigned(std::min<int64_t>((nnz + kThreads - 1) / kThreads, 8192));
    hipLaunchKernelGGL(k_hub_keys, dim3(g), dim3(kThreads), 0, s, rowind_in, rowptr, nnz, maxdeg, kin);
    e = hipGetLastError();
  }
  // a stable sort within each column: equal degrees keep their stored (ascending id) order
  if (e == hipSuccess)
    e = rocprim::segmented_radix_sort_pairs(nullptr, tb, kin, kout, rowind_in, rowind_out, unsigned(nnz),
                                            unsigned(V), colptr, colptr + 1, 0, unsigned(bits), s);
  if (e == hipSuccess) e = hipMalloc(&tmp, std::max<size_t>(tb, 1));
  if (e == hipSuccess)
    e = rocprim::segmented_radix_sort_pairs(tmp, tb, kin, kout, rowind_in, rowind_out, unsigned(nnz),
                                            unsigned(V), colptr, colptr + 1, 0, unsigned(bits), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (kin) (void)hipFree(kin);
  if (kout) (void)hipFree(kout);
  if (tmp) (void)hipFree(tmp);
  return e;
}

size_t sort_push_bytes(int64_t nnz) {
  size_t tmp = 0, tk = 0;
  const unsigned n = unsigned(nnz > 0 ? nnz : 1);
  (void)rocprim::radix_sort_pairs(nullptr, tmp, static_cast<const uint32_t*>(nullptr),
                                  static_cast<uint32_t*>(nullptr), static_cast<const int32_t*>(nullptr),
                                  static_cast<int32_t*>(nullptr), n, 0, 32);
  (void)rocprim::radix_sort_keys(nullptr, tk, static_cast<const uint32_t*>(nullptr),
                                 static_cast<uint32_t*>(nullptr), n, 0, 32);
  return std::max(tmp, tk);
}

hipError_t launch_sort_gather(hipStream_t s, const ExpandArgs& a, uint32_t* keys, int32_t* vals) {
  const uint32_t nchunks = (a.m + kExpandChunk - 1) / kExpandChunk;
  const unsigned g = unsigned(std::max<uint32_t>(1, std::min<uint32_t>(nchunks, 4096)));
  hipLaunchKernelGGL(k_sort_gather, dim3(g), dim3(kThreads), 0, s, a, keys, vals);
  return hipGetLastError();
}

hipError_t sort_pairs(hipStream_t s, void* tmp, size_t tmp_bytes, const uint32_t* kin, uint32_t* kout,
                      const int32_t* vin, int32_t* vout, uint32_t m, int bits) {
  size_t tb = tmp_bytes;
  return rocprim::radix_sort_pairs(tmp, tb, kin, kout, vin, vout, m, 0, bits, s);
}

hipError_t sort_keys(hipStream_t s, void* tmp, size_t tmp_bytes, const uint32_t* kin, uint32_t* kout, uint32_t m,
                     int bits) {
  size_t tb = tmp_bytes;
  return rocprim::radix_sort_keys(tmp, tb, kin, kout, m, 0, bits, s);
}

hipError_t launch_sort_filter(hipStream_t s, const uint32_t* keys, const int32_t* vals, uint32_t m, uint32_t* vis,
                              int32_t* depth, int32_t* parent, int32_t level, int32_t* Qout, uint32_t* qcount,
                              LevelSlot* slot) {
  const unsigned g = unsigned(std::max<uint32_t>(1, std::min<uint32_t>((m + kThreads - 1) / kThreads, 2048)));
  hipLaunchKernelGGL(k_sort_filter, dim3(g), dim3(kThreads), 0, s, keys, vals, m, vis, depth, parent, level, Qout,
                     qcount, slot);
  return hipGetLastError();
}

}  // namespace dobfs
