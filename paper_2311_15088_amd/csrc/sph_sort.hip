// sph_sort.hip -- per-phase kernels of the counting sort up to the scatter (the
// fix-up is launched with the work-item list, sph_physics.hip); the bodies are
// in sph_sort_impl.hpp.
#include "sph_sort_impl.hpp"

namespace sph {

__global__ void __launch_bounds__(kSortBD) k_key_count(const SortSet* __restrict__ sets, int nsets,
                                                       const uint32_t* __restrict__ bprefix) {
  key_count_block(sets, nsets, bprefix, blockIdx.x);
}
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const SortSet* __restrict__ sets, int nsets,
                                                              const uint32_t* __restrict__ chunk_prefix,
                                                              uint32_t* __restrict__ bsum, uint32_t* counters) {
  scan_reduce_block(sets, nsets, chunk_prefix, bsum, counters, blockIdx.x);
}
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const SortSet* __restrict__ sets, int nsets,
                                                             const uint32_t* __restrict__ chunk_prefix,
                                                             const uint32_t* __restrict__ bsum) {
  scan_apply_block(sets, nsets, chunk_prefix, bsum, blockIdx.x);
}
__global__ void __launch_bounds__(kSortBD) k_scatter(const SortSet* __restrict__ sets, int nsets,
                                                     const uint32_t* __restrict__ bprefix) {
  scatter_block(sets, nsets, bprefix, blockIdx.x);
}

void launch_sort_phase(const SortPlan& P, int phase, hipStream_t st) {
  switch (phase) {
    case 0:
      if (P.nblocks) hipLaunchKernelGGL(k_key_count, dim3(P.nblocks), dim3(kSortBD), 0, st, P.sets, P.nsets, P.bprefix);
      break;
    case 1:
      hipLaunchKernelGGL(k_scan_reduce, dim3(P.nchunks), dim3(kScanThreads), 0, st, P.sets, P.nsets, P.chunk_prefix, P.bsum,
                         P.counters);
      break;
    case 2:
      hipLaunchKernelGGL(k_scan_apply, dim3(P.nchunks), dim3(kScanThreads), 0, st, P.sets, P.nsets, P.chunk_prefix, P.bsum);
      break;
    case 3:
      if (P.nblocks) hipLaunchKernelGGL(k_scatter, dim3(P.nblocks), dim3(kSortBD), 0, st, P.sets, P.nsets, P.bprefix);
      break;
  }
}

uint32_t scan_chunks(uint32_t ncells) { return (ncells + kChunk - 1) / kChunk; }

}  // namespace sph
