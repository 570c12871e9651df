// sph_voxel.hip -- voxel density at cube corners ("Voxel Density" section):
// at corner x, phi(x) = |x - xbar| - rbar with xbar the k-weighted mean of the
// particle positions within radius R, k(s) = (1 - s^2)^3, s = |x - x_i| / R,
// and rbar = r (every particle has radius r).  A corner with no particle
// within R gets +inf.
//
// A second neighbour gather on the step's cell table: one thread per corner,
// corners in x-fastest order, so a wavefront holds 64 neighbouring corners of
// one row that read the same few cell rows (their spans are contiguous in the
// sorted arrays) and share them through the caches.  The sums are taken
// relative to the corner, sum k (x_i - x) and sum k, so |x - xbar| =
// |sum k (x_i - x)| / sum k without cancellation.
#include "sph_internal.hpp"

namespace sph {

constexpr int kVoxelBD = 256;

__global__ void __launch_bounds__(kVoxelBD) k_voxel(PhysPlan P, VoxelPlan V) {
  const uint32_t c = blockIdx.x * kVoxelBD + threadIdx.x;
  if (c >= V.n) return;
  const DScene& S = P.scenes[0];
  const uint32_t nx = (uint32_t)V.dims[0], ny = (uint32_t)V.dims[1];
  const uint32_t ix = c % nx, iy = (c / nx) % ny, iz = c / (nx * ny);
  float q[3];
  {
#pragma clang fp contract(off)
    q[0] = V.mn[0] + (float)ix * V.gs;
    q[1] = V.mn[1] + (float)iy * V.gs;
    q[2] = V.mn[2] + (float)iz * V.gs;
  }
  // cells that can hold a particle within R of the corner
  int lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = cell_coord(q[k] - V.reach, S.g.mn[k], S.g.inv, S.g.dim[k]);
    hi[k] = cell_coord(q[k] + V.reach, S.g.mn[k], S.g.inv, S.g.dim[k]);
  }
  const uint32_t* __restrict__ off = P.off + S.obase;
  float sk = 0.0f, sx = 0.0f, sy = 0.0f, sz = 0.0f;
  for (int z = lo[2]; z <= hi[2]; ++z)
    for (int y = lo[1]; y <= hi[1]; ++y) {
      const uint32_t a = S.pbase + off[hash3(S.g, lo[0], y, z)], b = S.pbase + off[hash3(S.g, hi[0], y, z) + 1];
      for (uint32_t j = a; j < b; ++j) {
        const float dx = P.sx[j] - q[0], dy = P.sy[j] - q[1], dz = P.sz[j] - q[2];
        const float d2 = dist2_exact(dx, dy, dz);
        if (d2 < V.R2) {
          // (1 - s^2) = (R^2 - d^2) / R^2 > 0: the subtraction is exact here
          const float t = (V.R2 - d2) * V.inv_R2;
          const float k = t * t * t;
          sk += k;
          sx += k * dx;
          sy += k * dy;
          sz += k * dz;
        }
      }
    }
  V.phi[c] = sk > 0.0f ? sqrtf(sx * sx + sy * sy + sz * sz) / sk - V.r : __builtin_huge_valf();
}

void launch_voxel(const PhysPlan& P, const VoxelPlan& V, hipStream_t st) {
  if (!V.phi || !V.n) return;
  hipLaunchKernelGGL(k_voxel, dim3((V.n + kVoxelBD - 1) / kVoxelBD), dim3(kVoxelBD), 0, st, P, V);
}

}  // namespace sph
