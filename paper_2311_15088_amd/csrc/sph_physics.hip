// sph_physics.hip -- per-phase kernels of the fluid and agent passes and their
// launch configurations; the bodies are in sph_fluid_impl.hpp.
#include <hip/hip_ext.h>

#include "sph_agents_impl.hpp"
#include "sph_fluid_impl.hpp"
#include "sph_sort_impl.hpp"

namespace sph {

// The sort's fix-up and the work-item list of the fluid passes share one
// launch.  The list reads only the cell offsets of this step, so it does not
// wait for the fix-up; its blocks come first in the grid, so that its long
// per-lane walks over dense tiles start while the fix-up fills the machine.
static_assert(kSortBD == 256, "one block size for both parts");
__global__ void __launch_bounds__(256) k_fixup_tiles(const SortSet* __restrict__ sets, int nsets,
                                                     const uint32_t* __restrict__ bprefix, uint32_t tile_blocks,
                                                     PhysPlan P) {
  if (blockIdx.x < tile_blocks) tile_list_block(P, blockIdx.x);
  else fixup_block(sets, nsets, bprefix, blockIdx.x - tile_blocks);
}

template <bool FORCE, int BD, int CAP, bool UNIT_H = false, int TXM = 32, int TY = 1>
__global__ void __launch_bounds__(BD) k_fluid(PhysPlan P) {
  fluid_tiles<FORCE, BD, CAP, UNIT_H, TXM, TY>(P);
}

template <int BD>
__global__ void __launch_bounds__(BD) k_agents(PhysPlan P) {
  agents_block<BD>(P, blockIdx.x);
}

// ----------------------------------------------------------------------------
// Launch configurations of the fluid passes: block size and LDS window of the
// density pass, of the force pass (a halo row longer than the window is staged
// in pieces), and the most own particles per work item.  They are
// instantiations of the one kernel above; every one produces bit-identical
// results (the candidate order of each particle does not depend on them).
struct FluidVariant {
  const void* density;
  const void* density_unit;  // the density pass when every scene has h^2 <= 1
  const void* force;
  int bd_density, bd_force, item_max, tile_max, tile_y;
  const char* name;
};

// TXM: widest tile of the variant; TY: its grid rows per tile along y.
template <int BDD, int CD, int BDF, int CF, int TXM = 32, int TY = 1>
static FluidVariant make_variant(int item_max, const char* name) {
  return FluidVariant{(const void*)k_fluid<false, BDD, CD, false, TXM, TY>,
                      (const void*)k_fluid<false, BDD, CD, true, TXM, TY>,
                      (const void*)k_fluid<true, BDF, CF, false, TXM, TY>, BDD, BDF, item_max, TXM, TY, name};
}

static const FluidVariant* variants() {
  // On a fluid at rest density the density pass runs fastest with 512-thread
  // blocks (variant 0); over a dam break's 1,000 steps, as the column
  // compresses, 256-thread blocks in both passes (variant 1, the default:
  // 0.33 against 0.34 ms per step at 1,048,576 particles).  The force pass
  // (more registers and LDS per thread) prefers 256 threads; items of at most
  // 256 own particles suit both.
  static const FluidVariant v[] = {
      make_variant<512, 512, 256, 512>(256, "d512_f256_win512"),
      make_variant<256, 512, 256, 512>(256, "bd256_win512_512"),
      make_variant<128, 512, 128, 256>(128, "bd128_win512_256"),
      make_variant<512, 512, 512, 512>(512, "bd512_win512_512"),
      make_variant<256, 1024, 256, 1024>(256, "bd256_win1024_1024"),
      make_variant<256, 256, 256, 256>(256, "bd256_win256_256"),
      make_variant<512, 1024, 256, 512>(256, "d512_win1024_f256_win512"),
      make_variant<1024, 1024, 256, 512>(256, "d1024_win1024_f256_win512"),
      // more than one own particle per thread: work items of up to two or
      // four blocks' worth of particles (each thread takes particles i,
      // i + BD, ...), so a dense tile re-stages its halo rows less often
      make_variant<512, 512, 256, 512>(512, "d512_f256_ppt2"),
      make_variant<256, 512, 256, 512>(512, "bd256_ppt2"),
      make_variant<256, 512, 256, 512>(1024, "bd256_ppt4"),
      // both passes with 512 threads on tiles of up to 64 cells: at rest
      // density a tile then holds about 512 particles, one per thread of
      // either pass (config 1, first 100 steps: 0.250 against 0.255 ms per
      // step for the default; over 1,000 steps, as the column compresses,
      // 0.398 against 0.375)
      make_variant<512, 512, 512, 512, 64>(512, "bd512_tx64"),
      // tiles of two grid rows along y: twelve halo rows staged for two
      // rows of own particles instead of nine per row (a third fewer
      // stagings per own particle); each lane skips the three rows outside
      // its own stencil
      make_variant<512, 512, 256, 512, 32, 2>(256, "d512_f256_ty2"),
      make_variant<512, 512, 512, 512, 32, 2>(512, "bd512_ty2"),
  };
  return v;
}
constexpr int kNumVariants = 14;
constexpr int kAgentBD = 256;

int fluid_variants() { return kNumVariants; }
int fluid_default_variant() { return 1; }

int fluid_item_max(int fused, int variant) {
  if (fused) return kFusedBD;
  return variants()[(variant >= 0 && variant < kNumVariants) ? variant : 0].item_max;
}
const char* fluid_variant_name(int v) { return (v >= 0 && v < kNumVariants) ? variants()[v].name : nullptr; }

int fluid_tile_y(int fused, int variant) {
  if (fused) return 1;
  return (variant >= 0 && variant < kNumVariants) ? variants()[variant].tile_y : 1;
}

int fluid_tile_max(int fused, int variant) {
  if (fused) return 32;  // the fused kernel's tables
  return (variant >= 0 && variant < kNumVariants) ? variants()[variant].tile_max : 0;
}

static int persistent_blocks(const void* fn, int bd) {
  static int ncu = 0;
  if (!ncu) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu <= 0) ncu = 256;
  }
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, bd, 0) != hipSuccess || per <= 0) per = 1;
  return ncu * per;
}

// start / stop (may be null): events recorded when the kernel itself starts
// and ends (hipExtLaunchKernel), without the gaps between launches.
static void launch_fluid(const PhysPlan& P, bool force, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  static int grids[kNumVariants][3];
  const int v = (P.variant >= 0 && P.variant < kNumVariants) ? P.variant : 0;
  const FluidVariant& V = variants()[v];
  const int form = force ? 2 : (P.unit_h ? 1 : 0);
  const void* fn = force ? V.force : (P.unit_h ? V.density_unit : V.density);
  const int bd = force ? V.bd_force : V.bd_density;
  int& grid = grids[v][form];
  if (!grid) grid = persistent_blocks(fn, bd);
  const uint32_t g = std::min<uint32_t>((uint32_t)grid, P.ntiles);
  void* args[] = {(void*)&P};
  if (start || stop) (void)hipExtLaunchKernel(fn, dim3(g), dim3(bd), args, 0, st, start, stop, 0);
  else (void)hipLaunchKernel(fn, dim3(g), dim3(bd), args, 0, st);
}

void launch_fixup_tiles(const SortPlan& S, const PhysPlan& P, hipStream_t st, bool with_tiles) {
  const uint32_t tb = (P.nf && with_tiles) ? (P.ntiles + 255) / 256 : 0u;
  if (tb + S.nblocks)
    hipLaunchKernelGGL(k_fixup_tiles, dim3(tb + S.nblocks), dim3(256), 0, st, S.sets, S.nsets, S.bprefix, tb, P);
}

void launch_density(const PhysPlan& P, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  if (!P.nf) return;
  launch_fluid(P, false, st, start, stop);
}

void launch_force(const PhysPlan& P, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  if (!P.nf) return;
  launch_fluid(P, true, st, start, stop);
}

void launch_agents(const PhysPlan& P, hipStream_t st) {
  if (!P.na) return;
  const uint32_t waves_per_block = kAgentBD / kWave;
  hipLaunchKernelGGL(k_agents<kAgentBD>, dim3((P.na + waves_per_block - 1) / waves_per_block), dim3(kAgentBD), 0, st,
                     P);
}

uint32_t fluid_tiles(const DGrid& g, int tx, int ty) { return tiles_of(g, tx, ty); }

}  // namespace sph
