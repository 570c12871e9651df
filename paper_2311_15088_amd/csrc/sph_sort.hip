// sph_sort.hip -- cell keys and the deterministic counting sort of fluid
// particles and agents (Sections "Neighborhood Search" and "Neighbor Search
// with Sorting" of the paper).
//
// Per set (the fluid or the agents of one scene):
//   k_key_count   key = hash(get_cell(x)); rank = atomic slot in the cell
//                 (one atomic per run of equal keys in a wavefront: the input
//                 is the previous step's cell order, so runs are long)
//   k_scan_*      exclusive prefix sum of the cell counts -> first slot of
//                 each cell; the counters are cleared for the next step
//   k_scatter     slot = off[key] + rank; record (source, id) at the slot
//   k_fixup       the atomics leave the order inside a cell arbitrary; each
//                 slot is re-ranked by id inside its cell, which makes the
//                 order the (key, id) order -- a pure function of the state --
//                 and the particle is gathered into cell-ordered SoA arrays.
// Many sets share one launch: a thread finds its set by binary search over
// the prefix of set sizes.
#include "sph_device.hpp"
#include "sph_internal.hpp"

namespace sph {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kChunk = kScanThreads * kScanPer;  // cells per scan block

__global__ void __launch_bounds__(256) k_key_count(const SortSet* __restrict__ sets, int nsets,
                                                   const uint32_t* __restrict__ prefix, uint32_t total) {
  const uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const bool valid = gi < total;
  int s = 0;
  uint32_t li = 0, key = 0xFFFFFFFFu;
  if (valid) {
    s = find_set(prefix, nsets, gi);
    li = gi - prefix[s];
    const SortSet& S = sets[s];
    int cx, cy, cz;
    cell_of(S.g, S.x[li], S.y[li], S.z[li], cx, cy, cz);
    key = hash3(S.g, cx, cy, cz);
    S.key[li] = key;
  }
  // runs of equal (set, key) in consecutive lanes share one atomic
  const uint32_t pkey = __shfl_up(key, 1);
  const int ps = __shfl_up(s, 1);
  const bool head = !valid || lane == 0 || pkey != key || ps != s;
  const uint64_t heads = __ballot(head);
  const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const int start = 63 - __clzll(heads & upto);
  const uint64_t after = heads & ~upto;
  const int end = after ? (__ffsll((long long)after) - 1) : 64;
  uint32_t base = 0;
  if (valid && lane == start) base = atomicAdd(&sets[s].cnt[key], (uint32_t)(end - start));
  base = __shfl(base, start);
  if (valid) sets[s].rank[li] = base + (uint32_t)(lane - start);
}

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds_wave, uint32_t& total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t t = __shfl_up(inc, d);
    if (lane >= d) inc += t;
  }
  if (lane == kWave - 1) lds_wave[wave] = inc;
  __syncthreads();
  uint32_t woff = 0, tot = 0;
  const int nw = blockDim.x / kWave;
  for (int w = 0; w < nw; ++w) {
    uint32_t t = lds_wave[w];
    if (w < wave) woff += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return woff + inc - v;
}

// Phase 1: per-chunk totals.
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const SortSet* __restrict__ sets, int nsets,
                                                              const uint32_t* __restrict__ chunk_prefix,
                                                              uint32_t* __restrict__ bsum) {
  __shared__ uint32_t lw[kScanThreads / kWave];
  const uint32_t b = blockIdx.x;
  const int s = find_set(chunk_prefix, nsets, b);
  const SortSet& S = sets[s];
  const uint32_t c0 = (b - chunk_prefix[s]) * kChunk;
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    uint32_t c = c0 + k * kScanThreads + threadIdx.x;
    if (c < S.g.ncells) acc += S.cnt[c];
  }
  uint32_t tot;
  block_exclusive_scan(acc, lw, tot);
  if (threadIdx.x == 0) bsum[b] = tot;
}

// Phase 2: exclusive scan of the chunk totals of each set (one block per set).
__global__ void __launch_bounds__(kScanThreads) k_scan_sets(int nsets, const uint32_t* __restrict__ chunk_prefix,
                                                            uint32_t* __restrict__ bsum, uint32_t* counters) {
  __shared__ uint32_t lw[kScanThreads / kWave];
  const int s = blockIdx.x;
  // the work counters of this step's tiled passes start from zero
  if (s == 0 && threadIdx.x < kWorkCounters && counters) counters[threadIdx.x] = 0u;
  if (s >= nsets) return;
  const uint32_t b0 = chunk_prefix[s], b1 = chunk_prefix[s + 1];
  uint32_t carry = 0;
  for (uint32_t base = b0; base < b1; base += kScanThreads) {
    uint32_t b = base + threadIdx.x;
    uint32_t v = (b < b1) ? bsum[b] : 0u;
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(v, lw, tot);
    if (b < b1) bsum[b] = carry + ex;
    carry += tot;
  }
}

// Phase 3: offsets of every cell; clears the counters; writes off[cells] = n.
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const SortSet* __restrict__ sets, int nsets,
                                                             const uint32_t* __restrict__ chunk_prefix,
                                                             const uint32_t* __restrict__ bsum) {
  __shared__ uint32_t lw[kScanThreads / kWave];
  const uint32_t b = blockIdx.x;
  const int s = find_set(chunk_prefix, nsets, b);
  const SortSet& S = sets[s];
  const uint32_t nc = S.g.ncells;
  // each thread owns kScanPer consecutive cells
  const uint32_t c0 = (b - chunk_prefix[s]) * kChunk + threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    uint32_t c = c0 + k;
    v[k] = (c < nc) ? S.cnt[c] : 0u;
    acc += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(acc, lw, tot) + bsum[b];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    uint32_t c = c0 + k;
    if (c < nc) {
      S.off[c] = ex;
      S.cnt[c] = 0u;
    }
    ex += v[k];
  }
  if (b + 1 == chunk_prefix[s + 1] && threadIdx.x == 0) S.off[nc] = bsum[b] + tot;
}

__global__ void __launch_bounds__(256) k_scatter(const SortSet* __restrict__ sets, int nsets,
                                                 const uint32_t* __restrict__ prefix, uint32_t total) {
  const uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= total) return;
  const int s = find_set(prefix, nsets, gi);
  const uint32_t li = gi - prefix[s];
  const SortSet& S = sets[s];
  const uint32_t pos = S.off[S.key[li]] + S.rank[li];
  S.tsrc[pos] = li;
  S.tid[pos] = S.id[li];
}

__global__ void __launch_bounds__(256) k_fixup(const SortSet* __restrict__ sets, int nsets,
                                               const uint32_t* __restrict__ prefix, uint32_t total) {
  const uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= total) return;
  const int s = find_set(prefix, nsets, gi);
  const uint32_t slot = gi - prefix[s];
  const SortSet& S = sets[s];
  const uint32_t src = S.tsrc[slot];
  const uint32_t myid = S.tid[slot];
  const uint32_t c = S.key[src];
  const uint32_t a = S.off[c], e = S.off[c + 1];
  uint32_t r = 0;
  for (uint32_t t = a; t < e; ++t) r += (S.tid[t] < myid) ? 1u : 0u;
  const uint32_t dst = a + r;
  S.sx[dst] = S.x[src];
  S.sy[dst] = S.y[src];
  S.sz[dst] = S.z[src];
  S.svx[dst] = S.vx[src];
  S.svy[dst] = S.vy[src];
  S.svz[dst] = S.vz[src];
  S.sid[dst] = myid;
}

static inline uint32_t blocks_for(uint32_t n, int bs) { return (n + bs - 1) / bs; }

void launch_sort_phase(const SortPlan& P, int phase, hipStream_t st) {
  switch (phase) {
    case 0:
      if (P.total > 0)
        hipLaunchKernelGGL(k_key_count, dim3(blocks_for(P.total, 256)), dim3(256), 0, st, P.sets, P.nsets, P.prefix, P.total);
      break;
    case 1:
      hipLaunchKernelGGL(k_scan_reduce, dim3(P.nchunks), dim3(kScanThreads), 0, st, P.sets, P.nsets, P.chunk_prefix, P.bsum);
      break;
    case 2:
      hipLaunchKernelGGL(k_scan_sets, dim3(P.nsets), dim3(kScanThreads), 0, st, P.nsets, P.chunk_prefix, P.bsum,
                         P.counters);
      break;
    case 3:
      hipLaunchKernelGGL(k_scan_apply, dim3(P.nchunks), dim3(kScanThreads), 0, st, P.sets, P.nsets, P.chunk_prefix, P.bsum);
      break;
    case 4:
      if (P.total > 0)
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(P.total, 256)), dim3(256), 0, st, P.sets, P.nsets, P.prefix, P.total);
      break;
    case 5:
      if (P.total > 0)
        hipLaunchKernelGGL(k_fixup, dim3(blocks_for(P.total, 256)), dim3(256), 0, st, P.sets, P.nsets, P.prefix, P.total);
      break;
  }
}

void launch_sort(const SortPlan& P, hipStream_t st) {
  for (int ph = 0; ph < kSortPhases; ++ph) launch_sort_phase(P, ph, st);
}

uint32_t scan_chunks(uint32_t ncells) { return (ncells + kChunk - 1) / kChunk; }

}  // namespace sph
