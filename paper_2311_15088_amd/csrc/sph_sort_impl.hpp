// sph_sort_impl.hpp -- bodies of the counting-sort phases (Sections
// "Neighborhood Search" and "Neighbor Search with Sorting" of the paper) as
// device functions of one block, shared by the per-phase kernels and the
// fused step kernel.
//
// Per set (the fluid or the agents of one scene):
//   key_count   key = hash(get_cell(x)); rank = atomic slot in the cell
//               (one atomic per run of equal keys in a wavefront: the input
//               is the previous step's cell order, so runs are long)
//   scan_*      exclusive prefix sum of the cell counts -> first slot of
//               each cell; the counters are cleared for the next step
//   scatter     slot = off[key] + rank; record (source, id) at the slot
//   fixup       the atomics leave the order inside a cell arbitrary; each
//               slot is re-ranked by id inside its cell, which makes the
//               order the (key, id) order -- a pure function of the state --
//               and the particle is gathered into cell-ordered SoA arrays.
// Element phases give every set whole blocks (block prefix over sets), so the
// set of a block is uniform and its descriptor is read with scalar loads.
#pragma once
#include "sph_device.hpp"
#include "sph_internal.hpp"

namespace sph {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kChunk = kScanThreads * kScanPer;  // cells per scan block

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void key_count_block(const SortSet* __restrict__ sets, int nsets,
                                                       const uint32_t* __restrict__ bprefix, uint32_t blk) {
  const int s = (int)uni(find_set(bprefix, nsets, blk));
  const SortSet& S = sets[s];
  const uint32_t li = (blk - bprefix[s]) * kSortBD + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const bool valid = li < S.n;
  uint32_t key = 0xFFFFFFFFu;
  if (valid) {
    int cx, cy, cz;
    cell_of(S.g, S.x[li], S.y[li], S.z[li], cx, cy, cz);
    key = hash3(S.g, cx, cy, cz);
    S.key[li] = key;
  }
  // runs of equal keys in consecutive lanes share one atomic
  const uint32_t pkey = __shfl_up(key, 1);
  const bool head = !valid || lane == 0 || pkey != key;
  const uint64_t heads = __ballot(head);
  const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const int start = 63 - __clzll(heads & upto);
  const uint64_t after = heads & ~upto;
  const int end = after ? (__ffsll((long long)after) - 1) : 64;
  uint32_t base = 0;
  if (valid && lane == start) base = atomicAdd(&S.cnt[key], (uint32_t)(end - start));
  base = __shfl(base, start);
  if (valid) S.rank[li] = base + (uint32_t)(lane - start);
}

// Exclusive scan of one value per thread across the block; returns the
// exclusive prefix and the block total.
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

// Phase 1: per-chunk totals (coalesced loads); block 0 also clears the work
// counters of this step's tiled passes.
__device__ __forceinline__ void scan_reduce_block(const SortSet* __restrict__ sets, int nsets,
                                                  const uint32_t* __restrict__ chunk_prefix,
                                                  uint32_t* __restrict__ bsum, uint32_t* counters, uint32_t blk) {
  __shared__ uint32_t lw[kScanThreads / kWave];
  const uint32_t b = blk;
  if (b == 0 && counters)
    for (int k = threadIdx.x; k < kWorkCounters; k += blockDim.x) counters[k] = 0u;
  const int s = (int)uni(find_set(chunk_prefix, nsets, b));
  const SortSet& S = sets[s];
  const uint32_t c0 = (b - chunk_prefix[s]) * kChunk;
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const uint32_t c = c0 + k * kScanThreads + threadIdx.x;
    if (c < S.g.ncells) acc += S.cnt[c];
  }
  uint32_t tot;
  block_exclusive_scan(acc, lw, tot);
  if (threadIdx.x == 0) bsum[b] = tot;
}

// Phase 2: offsets of every cell; clears the counters; writes off[cells] = n.
// A chunk's base is the sum of the totals of the set's earlier chunks, summed
// by the block itself.  Coalesced loads/stores, transposed through LDS so
// that every thread scans kScanPer consecutive cells.
__device__ __forceinline__ void scan_apply_block(const SortSet* __restrict__ sets, int nsets,
                                                             const uint32_t* __restrict__ chunk_prefix,
                                                             const uint32_t* __restrict__ bsum, uint32_t blk) {
  __shared__ uint32_t lw[kScanThreads / kWave];
  __shared__ uint4 lc[kScanThreads];
  const uint32_t b = blk;
  const int s = (int)uni(find_set(chunk_prefix, nsets, b));
  const SortSet& S = sets[s];
  const uint32_t nc = S.g.ncells;
  const uint32_t c0 = (b - chunk_prefix[s]) * kChunk;
  uint32_t* lflat = reinterpret_cast<uint32_t*>(lc);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const uint32_t e = k * kScanThreads + threadIdx.x;
    const uint32_t c = c0 + e;
    uint32_t v = 0;
    if (c < nc) {
      v = S.cnt[c];
      S.cnt[c] = 0u;
    }
    lflat[e] = v;
  }
  __syncthreads();
  uint32_t part = 0;
  for (uint32_t q = chunk_prefix[s] + threadIdx.x; q < b; q += kScanThreads) part += bsum[q];
  uint32_t base;
  block_exclusive_scan(part, lw, base);
  const uint4 v = lc[threadIdx.x];
  uint32_t tot;
  const uint32_t ex = block_exclusive_scan(v.x + v.y + v.z + v.w, lw, tot) + base;
  lc[threadIdx.x] = make_uint4(ex, ex + v.x, ex + v.x + v.y, ex + v.x + v.y + v.z);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const uint32_t e = k * kScanThreads + threadIdx.x;
    const uint32_t c = c0 + e;
    if (c < nc) S.off[c] = lflat[e];
  }
  if (b + 1 == chunk_prefix[s + 1] && threadIdx.x == 0) S.off[nc] = base + tot;
}

__device__ __forceinline__ void scatter_block(const SortSet* __restrict__ sets, int nsets,
                                                     const uint32_t* __restrict__ bprefix, uint32_t blk) {
  const int s = (int)uni(find_set(bprefix, nsets, blk));
  const SortSet& S = sets[s];
  const uint32_t li = (blk - bprefix[s]) * kSortBD + threadIdx.x;
  if (li >= S.n) return;
  const uint32_t pos = S.off[S.key[li]] + S.rank[li];
  S.tsrc[pos] = li;
  S.tid[pos] = S.id[li];
}

// ids staged in LDS per fix-up block: the cells of a block's 256 slots span
// this many slots at most when no cell holds more than 384 particles
constexpr uint32_t kFixStage = 1024;

__device__ __forceinline__ void fixup_block(const SortSet* __restrict__ sets, int nsets,
                                                   const uint32_t* __restrict__ bprefix, uint32_t blk) {
  __shared__ uint32_t s_ids[kFixStage];
  __shared__ uint32_t s_lo[kSortBD / kWave], s_hi[kSortBD / kWave];
  const int s = (int)uni(find_set(bprefix, nsets, blk));
  const SortSet& S = sets[s];
  const uint32_t first = (blk - bprefix[s]) * kSortBD;
  const uint32_t slot = first + threadIdx.x;
  const uint32_t w0 = first + (threadIdx.x & ~(kWave - 1));  // first slot of this wavefront
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const bool act = slot < S.n;
  uint32_t src = 0, myid = 0, a = 0, len = 0;
  if (act) {
    src = S.tsrc[slot];
    myid = S.tid[slot];
    const uint32_t c = S.key[src];
    a = S.off[c];
    len = S.off[c + 1] - a;
  }
  // rank = number of ids in the cell smaller than mine.  The slots of the
  // cells this block's slots lie in are staged in LDS when they fit (one
  // coalesced load per slot); otherwise ids of slots inside this wavefront
  // come from the other lanes and the rest from memory.
  uint32_t maxlen = len, lo = act ? a : 0xffffffffu, hi = act ? a + len : 0u;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    maxlen = max(maxlen, (uint32_t)__shfl_xor(maxlen, d));
    lo = min(lo, (uint32_t)__shfl_xor(lo, d));
    hi = max(hi, (uint32_t)__shfl_xor(hi, d));
  }
  if (lane == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  uint32_t blo = 0xffffffffu, bhi = 0u;
#pragma unroll
  for (int w = 0; w < kSortBD / kWave; ++w) {
    blo = min(blo, s_lo[w]);
    bhi = max(bhi, s_hi[w]);
  }
  const bool staged = bhi > blo && bhi - blo <= kFixStage;  // the same for the whole block
  if (staged)
    for (uint32_t e = threadIdx.x; e < bhi - blo; e += kSortBD) s_ids[e] = S.tid[blo + e];
  __syncthreads();
  uint32_t r = 0;
  if (staged) {
    const uint32_t* __restrict__ cell = s_ids + (a - blo);
    for (uint32_t k = 0; k < maxlen; ++k)
      if (k < len) r += (cell[k] < myid) ? 1u : 0u;
  } else {
    for (uint32_t k = 0; k < maxlen; ++k) {
      const uint32_t t = a + k;
      uint32_t v = (uint32_t)__shfl(myid, (int)((t - w0) & (kWave - 1)));
      if (k < len) {
        if (t - w0 >= (uint32_t)kWave) v = S.tid[t];
        r += (v < myid) ? 1u : 0u;
      }
    }
  }
  __syncthreads();  // the shared words are reused by the next call
  if (!act) return;
  const uint32_t dst = a + r;
  S.sx[dst] = S.x[src];
  S.sy[dst] = S.y[src];
  S.sz[dst] = S.z[src];
  S.svx[dst] = S.vx[src];
  S.svy[dst] = S.vy[src];
  S.svz[dst] = S.vz[src];
  S.sid[dst] = myid;
}

}  // namespace sph
