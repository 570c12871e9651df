// sph_fused.hip -- one persistent launch per time step for all scenes.
//
// The kernel runs every phase of the step (cell keys and counting sort,
// tile list, density, then agents and forces) with grid-wide barriers between
// phases, so a step of hundreds of scenes is one launch instead of eleven.
// The grid never exceeds the number of workgroups the device holds at once,
// so all of them are resident and a barrier only waits for running waves.
// Phase bodies are the same device functions the per-phase kernels run, in
// the same order, so both forms give bit-identical results.
//
// Barrier: a counter and a generation word in device memory.  Each block
// publishes its writes with one agent-scope release fence (the L2 of its XCD
// is written back), arrives with a relaxed atomic, and waits by polling the
// generation word with relaxed atomic loads; only after the wait does it take
// one agent-scope acquire fence.  An acquire on every poll would invalidate
// the XCD's L2 under the blocks that are still working.  A wait is bounded:
// after kSpinLimit polls the block raises a sticky abort flag and leaves;
// every later barrier and every later launch sees the flag and leaves at once,
// so the grid always drains.
#include "sph_api_internal.hpp"
#include "sph_agents_impl.hpp"
#include "sph_fluid_impl.hpp"
#include "sph_sort_impl.hpp"

namespace sph {

constexpr uint32_t kSpinLimit = 1u << 20;  // ~0.1 s of polling with s_sleep

// Returns false (uniformly across the block) when the step was aborted.
__device__ __forceinline__ bool grid_sync(uint32_t* bar, int* abort_flag, uint32_t& gen, int* s_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t g = gen;
    const uint32_t arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == gridDim.x - 1) {
      // last arrival: reset the counter, then open the barrier (the release
      // orders the reset before the new generation)
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || ++spins > kSpinLimit) {
          __hip_atomic_fetch_or(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    gen = g + 1;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

template <int CAPD, int CAPF>
__global__ void __launch_bounds__(kFusedBD) k_step_fused(FusedPlan F) {
  __shared__ int s_ok;
  const SortPlan& S = F.sort;
  const PhysPlan& P = F.phys;
  const uint32_t G = gridDim.x;
  if (threadIdx.x == 0) s_ok = __hip_atomic_load(F.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 0 : 1;
  __syncthreads();
  if (!s_ok) return;  // an earlier step aborted: leave at once
  uint32_t gen = __hip_atomic_load(&F.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  for (uint32_t b = blockIdx.x; b < S.nblocks; b += G) key_count_block(S.sets, S.nsets, S.bprefix, b);
  if (!grid_sync(F.bar, F.abort_flag, gen, &s_ok)) return;
  for (uint32_t b = blockIdx.x; b < S.nchunks; b += G)
    scan_reduce_block(S.sets, S.nsets, S.chunk_prefix, S.bsum, S.counters, b);
  if (!grid_sync(F.bar, F.abort_flag, gen, &s_ok)) return;
  for (uint32_t b = blockIdx.x; b < S.nchunks; b += G) scan_apply_block(S.sets, S.nsets, S.chunk_prefix, S.bsum, b);
  if (!grid_sync(F.bar, F.abort_flag, gen, &s_ok)) return;
  for (uint32_t b = blockIdx.x; b < S.nblocks; b += G) scatter_block(S.sets, S.nsets, S.bprefix, b);
  if (!grid_sync(F.bar, F.abort_flag, gen, &s_ok)) return;
  for (uint32_t b = blockIdx.x; b < S.nblocks; b += G) fixup_block(S.sets, S.nsets, S.bprefix, b);
  if (!grid_sync(F.bar, F.abort_flag, gen, &s_ok)) return;
  if (P.nf) {
    for (uint32_t b = blockIdx.x; b < (P.ntiles + 255) / 256; b += G) tile_list_block(P, b);
    if (!grid_sync(F.bar, F.abort_flag, gen, &s_ok)) return;
    fluid_tiles<false, kFusedBD, CAPD>(P);
  }
  if (!grid_sync(F.bar, F.abort_flag, gen, &s_ok)) return;
  // agents and fluid forces touch disjoint arrays: no barrier between them
  const uint32_t agents_per_block = kFusedBD / kWave;
  for (uint32_t b = blockIdx.x; b < (P.na + agents_per_block - 1) / agents_per_block; b += G)
    agents_block<kFusedBD>(P, b);
  if (P.nf) fluid_tiles<true, kFusedBD, CAPF>(P);
}

using FusedFn = void (*)(FusedPlan);

struct FusedVariant {
  const void* fn;
  const char* name;
};

static const FusedVariant* fused_variants() {
  static const FusedVariant v[] = {
      {(const void*)k_step_fused<512, 512>, "fused_win512_512"},
      {(const void*)k_step_fused<1024, 512>, "fused_win1024_512"},
      {(const void*)k_step_fused<256, 256>, "fused_win256_256"},
  };
  return v;
}

int fused_variant_count() { return 3; }
const char* fused_variant_name(int v) {
  return (v >= 0 && v < fused_variant_count()) ? fused_variants()[v].name : nullptr;
}

// Largest grid whose workgroups are all resident at once.
int fused_grid(int variant) {
  static int grids[8];
  const int v = (variant >= 0 && variant < fused_variant_count()) ? variant : 0;
  if (!grids[v]) {
    int dev = 0, ncu = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fused_variants()[v].fn, kFusedBD, 0) != hipSuccess)
      per = 1;
    grids[v] = std::max(1, ncu) * std::max(1, per);
  }
  return grids[v];
}

void launch_step_fused(const FusedPlan& F, int variant, hipStream_t st) {
  const int v = (variant >= 0 && variant < fused_variant_count()) ? variant : 0;
  void* args[] = {(void*)&F};
  (void)hipLaunchKernel(fused_variants()[v].fn, dim3(fused_grid(v)), dim3(kFusedBD), args, 0, st);
}

}  // namespace sph
