// sph_internal.hpp -- host-side launch plans shared by the translation units
// of libsph.so (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sph_device.hpp"

namespace sph {

// Device tables describing one batched counting sort over several sets.
constexpr int kSortBD = 256;  // block size of the per-element sort kernels

struct SortPlan {
  const SortSet* sets;         // [nsets]
  int nsets;
  const uint32_t* bprefix;     // [nsets + 1] prefix of kSortBD-element blocks per set
  uint32_t nblocks;
  const uint32_t* chunk_prefix;// [nsets + 1] scan-chunk prefix
  uint32_t nchunks;
  uint32_t* bsum;              // [nchunks]
  uint32_t* counters;          // [kWorkCounters] work counters of the tiled passes, cleared by the scan
};

// closure controller state words: step counter, mode (1 = surrogate), use
// the surrogate this step, check step, checks, failed checks, steps taken with
// the surrogate / the exact gather, surrogate needed this step (use || check)
constexpr int kClStep = 0, kClMode = 1, kClUse = 2, kClCheck = 3, kClChecks = 4, kClFallbacks = 5,
              kClSurrogateSteps = 6, kClExactSteps = 7, kClNeed = 8, kClWords = 9;

// Work counters of the tiled passes.  Each pass hands its work items out
// from kItemQueues counters, each on a cache line of its own; queue q serves
// the workgroups b with b mod nq == q (nq = min(grid, kItemQueues)), which
// the hardware dispatches to one XCD.  One counter for the whole grid
// serialised every fetch of every workgroup at one address.
// A queue hands its items out in runs of kQueueRun consecutive list entries
// (queue q: entries q R .. q R + R - 1, then (nq + q) R .., R = kQueueRun):
// consecutive entries are neighbouring tiles whose halo rows overlap, so the
// workgroups of one XCD re-read them from that XCD's L2.  Runs of 16 took the
// L2 hit rate of the fluid passes from 35 / 15 % to 61 / 57 % (density /
// force) and their HBM reads from 110 / 334 MB to 47 / 155 MB per launch at
// config 1.
constexpr int kItemQueues = 8, kQueueStride = 32;  // 32 words = 128 bytes apart
constexpr uint32_t kQueueRun = 16;
constexpr int kCounterList = 0;
constexpr int kCounterDensity = kQueueStride, kCounterForce = kCounterDensity + kItemQueues * kQueueStride;
constexpr int kWorkCounters = kCounterForce + kItemQueues * kQueueStride;
// slots of the pair counter (each workgroup adds its count into slot
// blockIdx mod kPairSlots; a read sums them)
constexpr int kPairSlots = 64;
constexpr int kTXMax = 64;  // most cells per fluid tile (kernel variants may allow fewer)

// Device arrays of the physics kernels (all scenes concatenated).
struct PhysPlan {
  const DScene* scenes;
  int nscenes;
  const uint32_t* fprefix;     // [nscenes + 1] fluid element prefix (unpadded)
  uint32_t nf;
  const uint32_t* aprefix;     // [nscenes + 1] agent element prefix
  uint32_t na;
  // fluid, cell order
  const float *sx, *sy, *sz, *svx, *svy, *svz;
  const uint32_t* off;
  float* rho;
  uint32_t* nbr;
  uint32_t* nmask;             // [9][6][nf] neighbours among each halo row's candidates, 32 per word (density -> force)
  uint32_t* rowcode;           // [nf] each halo row's candidate cells, 3 bits per row (density -> force)
  unsigned long long* pairs;   // running sum of neighbour counts
  // tiles: runs of tx cells along x in one grid row (all scenes concatenated)
  const uint32_t* tprefix;     // [nscenes + 1] tile prefix
  uint32_t ntiles;
  int tx;                      // cells per tile along x (<= kTXMax)
  int ty;                      // grid rows per tile along y (the kernel variant's; 1 in the fused step)
  int variant;                 // kernel variant (block size, particles per thread, LDS capacity)
  int unit_h;                  // every scene has h^2 <= 1 (a density-pass form relies on it)
  unsigned long long* tile_list;  // [cells] work items of this step (tile << 16 | first cell << 8 | last cell)
  uint32_t item_max;           // particles per work item before a tile is cut
  uint32_t* counters;          // [kWorkCounters]
  // fluid, next-step storage (written by the force kernel)
  float *px, *py, *pz, *vx, *vy, *vz;
  // agents: state in id order (updated in place), sorted copies, offsets
  float *agx, *agy, *agz, *aux, *auy, *auz;
  const float *asx, *asy, *asz, *asvx, *asvy, *asvz;
  const uint32_t* asid;
  const uint32_t* aoff;
  // learned closure (nullptr = none): surrogate forces, controller state,
  // per-agent error terms at check steps
  const float* cl_fhat;
  const uint32_t* cl_state;
  float* cl_err;
  // obstacle grid on the agent grid (nullptr = no obstacles): per cell the
  // mean normal of the obstacle-mesh vertices in it, w = 1 if it has any
  const float4* obst;
  float obst_w;                // weight of the avoidance steering
  // diagnostics (nullptr = off)
  float *d_aint, *d_acoup, *d_steer, *d_force;  // [n][3] / [a][3]
  uint32_t *d_touch, *d_acnt;                   // [n] / [a][4]
};

constexpr int kSortPhases = 5;  // key+count, scan reduce, scan apply, scatter, fix-up
// sort phases 0 .. kSortPhases - 2 (the fix-up is launched with the tile list)
void launch_sort_phase(const SortPlan& P, int phase, hipStream_t st);
uint32_t scan_chunks(uint32_t ncells);

// fix-up + work-item list, density, agents, force + integration
constexpr int kStepPhases = kSortPhases + 3;
uint32_t fluid_tiles(const DGrid& g, int tx, int ty = 1);
int fluid_variants();
// Kernel variant of the per-phase form a context starts with.
int fluid_default_variant();
// particles per work item of the fluid passes: the block size of the form
int fluid_item_max(int fused, int variant);
// Widest tile (cells along x) a kernel variant's LDS tables hold.
int fluid_tile_max(int fused, int variant);
// Grid rows per tile along y of a kernel variant (1 for the fused step).
int fluid_tile_y(int fused, int variant);
const char* fluid_variant_name(int v);
// The sort's fix-up and the fluid passes' work-item list in one launch (the
// list needs only the cell offsets, so it overlaps the fix-up).
// with_tiles = false: the fix-up alone (the list forms need no work items)
void launch_fixup_tiles(const SortPlan& S, const PhysPlan& P, hipStream_t st, bool with_tiles = true);
// start / stop: optional events recorded at the fluid kernel's own start and end
void launch_density(const PhysPlan& P, hipStream_t st, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
void launch_agents(const PhysPlan& P, hipStream_t st);
void launch_force(const PhysPlan& P, hipStream_t st, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

// Neighbour-list forms of the fluid passes (the paper's list-based neighbour
// search), kept beside the tiled gather as ablations.  Mode: the tiled gather,
// the sorted list (count, scan, fill on the counting-sorted particles) or the
// bucket list (fixed-capacity cell buckets, 27 x capacity entries per particle).
constexpr int kSearchTiles = 0, kSearchSortedList = 1, kSearchBucketList = 2;
constexpr int kBucketOverflow = 0, kListOverflow = 1, kListStatusWords = 2;
struct ListPlan {
  int mode;
  uint32_t cap;          // bucket list: particles per cell bucket
  uint64_t list_cap;     // entries of the list buffer
  uint32_t* lcnt;        // [nf] list length per particle (the particle itself included)
  uint32_t* loff;        // [nf + 1] sorted list: first entry of each particle
  uint32_t* lsum;        // sorted list: scan chunk sums
  uint32_t* list;        // sorted indices: packed (sorted list) or [nf][27 cap] (bucket list)
  uint32_t* bcnt;        // [ncells] bucket fill counts
  uint32_t* bucket;      // [ncells][cap]
  uint32_t ncells;       // fluid cells of all scenes (scene s from its cbase)
  uint32_t* status;      // [kListStatusWords] sticky overflow flags
};
uint32_t list_scan_chunks(uint32_t n);
// the list of this step (after the sort's fix-up), the passes over it
void launch_list_build(const PhysPlan& P, const ListPlan& L, hipStream_t st);
void launch_list_density(const PhysPlan& P, const ListPlan& L, hipStream_t st, hipEvent_t start = nullptr,
                         hipEvent_t stop = nullptr);
void launch_list_force(const PhysPlan& P, const ListPlan& L, hipStream_t st, hipEvent_t start = nullptr,
                       hipEvent_t stop = nullptr);

// Voxel density at cube corners (single-scene contexts): the field of the
// state a step starts from, computed after its density pass.
struct VoxelPlan {
  float* phi;          // [n] corner values, x fastest (nullptr: off)
  uint32_t n;          // corners
  int dims[3];         // corners per axis
  float mn[3], gs;     // corner c at fl(mn + fl(c gs)) per axis
  float R2, inv_R2;    // R^2 (float32 of the double square), 1 / R^2
  float r;             // particle radius
  float reach;         // R with a margin for float32 rounding (cell ranges)
  int tile_ok;         // a 64 x 2 x 2 corner block reaches at most 64 cell rows
};
void launch_voxel(const PhysPlan& P, const VoxelPlan& V, hipStream_t st);

// One persistent launch per step (all phases, grid-wide barriers).
constexpr int kFusedBD = 256;
struct FusedPlan {
  SortPlan sort;
  PhysPlan phys;
  uint32_t* bar;    // [2] arrival counter, generation
  int* abort_flag;  // sticky: a barrier wait timed out
};
void launch_step_fused(const FusedPlan& F, int variant, hipStream_t st);
int fused_variant_count();
const char* fused_variant_name(int v);

}  // namespace sph
