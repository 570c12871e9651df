// sph_api_internal.hpp -- the context behind the opaque sph_ctx handle.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "sph.h"
#include "sph_device.hpp"
#include "sph_internal.hpp"
#include "sph_mlp.hpp"

struct sph_closure;

struct sph_ctx {
  std::string err;
  hipStream_t stream = nullptr;          // caller's stream (not owned)
  hipStream_t capture_stream = nullptr;  // owned; graphs are recorded here
  int nscenes = 0;
  std::vector<sph::DScene> hs;
  std::vector<sph_params> params;
  uint32_t N = 0, A = 0, C = 0, AC = 0;  // totals over scenes
  bool diag = false, check_finite = false;
  int64_t steps = 0;

  char* arena = nullptr;  // one device allocation holding every array below
  size_t bytes = 0;
  // fluid: storage (next step's input), cell-ordered copies, per-element scratch
  float *px, *py, *pz, *vx, *vy, *vz;
  float *sx, *sy, *sz, *svx, *svy, *svz;
  uint32_t *sid, *key, *rank, *tsrc, *tid;
  float* rho;
  uint32_t* nbr;
  uint32_t* nmask;
  uint32_t* rowcode;
  uint32_t *cnt, *off;
  // agents: state (id order), cell-ordered copies, scratch
  float *agx, *agy, *agz, *aux, *auy, *auz;
  float *asx, *asy, *asz, *asvx, *asvy, *asvz;
  uint32_t *asid, *aiota, *akey, *arank, *atsrc, *atid;
  uint32_t *acnt, *aoff;
  // diagnostics
  float *d_aint = nullptr, *d_acoup = nullptr, *d_steer = nullptr, *d_force = nullptr;
  uint32_t *d_touch = nullptr, *d_acnt = nullptr;
  // tables
  uint32_t* bsum;
  sph::SortSet* d_sets;
  uint32_t *d_prefix, *d_bprefix, *d_chunk_prefix, *d_fprefix, *d_aprefix;
  sph::DScene* d_scenes;
  unsigned long long* d_pairs;
  uint32_t* d_tprefix;
  uint32_t* d_counters;
  unsigned long long* d_tile_list;
  uint32_t ntiles = 0;
  int* d_flag;
  int nsets = 0;
  uint32_t nchunks = 0;

  sph::SortPlan sort;
  sph::PhysPlan phys;
  // execution form: per-phase launches or one fused launch per step
  bool fused = false;
  int fused_variant = 0;
  uint32_t* d_bar;   // [2] grid-barrier counter, generation
  int* d_abort;      // fused barrier timed out (sticky)
  int* h_abort = nullptr;  // pinned host copy of d_abort, refreshed after every fused launch
  bool fused_ran = false;  // fused steps were enqueued (sph_read then checks d_abort)
  float tuned_ms = 0.0f;

  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int32_t graph_steps = 0;
  std::vector<hipEvent_t> prof_ev;  // sph_step_profiled (created on first use)

  void* staging = nullptr;  // readback staging (allocated on first read)
  size_t staging_bytes = 0;

  // learned coupling closure (not owned) and per-agent feature buffers
  sph_closure* closure = nullptr;
  bool features = false;     // compute features every step (training-data collection)
  sph::ClosurePlan cplan{};  // buffers allocated on first use
  char* cl_arena = nullptr;

  // neighbour-list forms of the fluid passes (mode kSearchTiles: none)
  sph::ListPlan list{};
  char* list_arena = nullptr;

  // voxel density at cube corners (phi == nullptr: off)
  sph::VoxelPlan voxel{};

  // obstacle grid (phys.obst; owned here)
  float4* obst = nullptr;
};

sph_status sph_ctx_build(const std::vector<sph_params>& params, const std::vector<int64_t>& n,
                         const std::vector<int64_t>& na, const std::vector<const float*>& pos,
                         const std::vector<const float*>& vel, const std::vector<const float*>& apos,
                         const std::vector<const float*>& avel, void* stream, sph_ctx** out);
sph_status sph_enqueue_steps(sph_ctx* ctx, int32_t n_steps, hipStream_t st);
sph_status set_tiling(sph_ctx* ctx, int tx, int variant, bool fused);
sph_status sph_ctx_closure_buffers(sph_ctx* ctx);
void sph_ctx_closure_phase(sph_ctx* ctx, hipStream_t st);
void sph_ctx_closure_end(sph_ctx* ctx, hipStream_t st);
