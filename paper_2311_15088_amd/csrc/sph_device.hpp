// sph_device.hpp -- device-side descriptors and helpers shared by the kernels
// of libsph.so (internal; not part of the C ABI).
//
// Layout in HBM: every per-element array is SoA float32 / uint32.  Several
// independent scenes live in one set of arrays: scene s owns fluid elements
// [pbase, pbase + n), agent elements [abase, abase + na), fluid cell counters
// [cbase, cbase + cells), fluid offsets [obase, obase + cells + 1), and the
// same for the agent grid.  Offsets are local to the scene.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sph {

constexpr int kWave = 64;

// Uniform grid (Section "Neighborhood Search"): get_cell(p) = floor((p - m)/d)
// evaluated as fl32(fl32(p - m) * inv_d), and the linear hash
// c_x + dim_x (c_y + dim_y c_z).
struct DGrid {
  float mn[3];
  float inv;   // 1 / cell edge, as used by get_cell
  float cell;  // cell edge
  int dim[3];
  uint32_t ncells;
};

// Per-scene constants, derived on the host from sph_params.
struct DScene {
  uint32_t n, na;
  uint32_t pbase, abase;
  uint32_t cbase, obase;   // fluid cell counters / offsets
  uint32_t acbase, aobase; // agent cell counters / offsets
  DGrid g, ga;
  int ns_c;                // fluid-grid stencil half-width covering r_couple
  // fluid
  float h2, inv_h, c6m, rho0, cpk_h, cvmu, m, inv_m, dt, e;
  float grav[3], bmin[3], bmax[3];
  // coupling (agent = particle of mass m at rest density)
  float rc2, inv_rc, cpk_hc, cvmu_c, m_over_rho0, cf;
  // boids
  float rsep2, rali2, rcoh2, inv_rsep, wsep, wali, wcoh, vmin, vmax;
};

// A set of points to be ordered by cell (the fluid or the agents of a scene).
struct SortSet {
  const float *x, *y, *z, *vx, *vy, *vz;  // storage order (input)
  const uint32_t* id;
  float *sx, *sy, *sz, *svx, *svy, *svz;  // cell order (output)
  uint32_t* sid;
  uint32_t *key, *rank, *tsrc, *tid;      // per-element scratch
  uint32_t *cnt, *off;                    // per-cell counters, offsets (cells + 1)
  DGrid g;
  uint32_t n;
};

// ------------------------------------------------------------------------
// Exact single-precision predicates.  Contraction is off inside these
// functions so that every operation is rounded as written: this is the
// definition the reference evaluates too.  The squared distance is
// fl(dz^2 + fl(dy^2 + fl(dx^2))) with the two outer steps fused
// multiply-adds (v_fma_f32: one rounding of the exact product plus sum),
// three instructions after the differences.
// ------------------------------------------------------------------------
__device__ __forceinline__ float dist2_exact(float dx, float dy, float dz) {
#pragma clang fp contract(off)
  float s = dx * dx;
  s = __builtin_fmaf(dy, dy, s);
  s = __builtin_fmaf(dz, dz, s);
  return s;
}

// A product rounded on its own, never fused into the add that uses it: the
// force passes scale C_p k h (rho - rho0) and C_v mu v once per particle or
// per staged candidate, and every form must round them alike.
__device__ __forceinline__ float mul_rn(float a, float b) {
#pragma clang fp contract(off)
  return a * b;
}

__device__ __forceinline__ int cell_coord(float p, float mn, float inv, int dim) {
#pragma clang fp contract(off)
  float t = p - mn;
  t = t * inv;
  float f = floorf(t);
  int c;
  if (!(f >= 0.0f)) c = 0;
  else if (f >= (float)dim) c = dim - 1;
  else c = (int)f;
  return c;
}

__device__ __forceinline__ void cell_of(const DGrid& g, float x, float y, float z, int& cx, int& cy, int& cz) {
  cx = cell_coord(x, g.mn[0], g.inv, g.dim[0]);
  cy = cell_coord(y, g.mn[1], g.inv, g.dim[1]);
  cz = cell_coord(z, g.mn[2], g.inv, g.dim[2]);
}

__device__ __forceinline__ uint32_t hash3(const DGrid& g, int cx, int cy, int cz) {
  return (uint32_t)cx + (uint32_t)g.dim[0] * ((uint32_t)cy + (uint32_t)g.dim[1] * (uint32_t)cz);
}

// Index of the set holding flat element gi: largest s with prefix[s] <= gi.
__device__ __forceinline__ int find_set(const uint32_t* __restrict__ prefix, int nsets, uint32_t gi) {
  int lo = 0, hi = nsets - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= gi) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Values the compiler cannot prove wave-uniform but that are: kept in scalar registers.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// Row spans of a stencil (up to 64 rows, lane r holding row r) as a flat list:
// pre[r] = first flat index of row r (pre[nrows] = total), dlt[r] = start_r - pre[r].
struct FlatRows {
  uint32_t* pre;
  uint32_t* dlt;
  uint32_t total;
};

__device__ __forceinline__ FlatRows flat_rows(uint32_t* pre, uint32_t* dlt, int lane, int nrows, uint32_t start,
                                              uint32_t len) {
  __builtin_amdgcn_wave_barrier();  // earlier reads of pre / dlt by this wave come first
  uint32_t incl = lane < nrows ? len : 0u;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)incl, d);
    if (lane >= d) incl += o;
  }
  const uint32_t excl = incl - (lane < nrows ? len : 0u);
  if (lane < nrows) {
    pre[lane] = excl;
    dlt[lane] = start - excl;
  }
  const uint32_t total = uniform_u32((uint32_t)__shfl((int)incl, kWave - 1));
  if (lane == 0) pre[nrows] = total;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return FlatRows{pre, dlt, total};
}

// Element index of flat position t (< total), advancing the lane's row cursor r.
__device__ __forceinline__ uint32_t flat_index(const FlatRows& F, uint32_t t, int& r) {
  while (t >= F.pre[r + 1]) ++r;
  return F.dlt[r] + t;
}

// Reflecting walls: a coordinate that left [lo, hi] is mirrored back and its
// velocity component scaled by -e; finally the coordinate is clamped.
__device__ __forceinline__ void wall(float& x, float& v, float lo, float hi, float e) {
  if (x < lo) {
    x = 2.0f * lo - x;
    v = -e * v;
  } else if (x > hi) {
    x = 2.0f * hi - x;
    v = -e * v;
  }
  x = fminf(fmaxf(x, lo), hi);
}

}  // namespace sph
