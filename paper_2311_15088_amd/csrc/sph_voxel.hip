// sph_voxel.hip -- voxel density at cube corners ("Voxel Density" section):
// at corner x, phi(x) = |x - xbar| - rbar with xbar the k-weighted mean of the
// particle positions within radius R, k(s) = (1 - s^2)^3, s = |x - x_i| / R,
// and rbar = r (every particle has radius r).  A corner with no particle
// within R gets +inf.
//
// A second neighbour gather on the step's cell table.  k_voxel runs one
// thread per corner, corners in x-fastest order, reading the particles from
// HBM through the caches; k_voxel_rows (below, the form launched when the
// grid fits a 3-D launch) stages them in LDS per segment of a corner row.  The sums are taken
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

// Row-tiled form: a workgroup takes kVoxelBD consecutive corners of one
// corner row (fixed y, z) and stages, cell row by cell row, the particles that
// any of its corners can reach into LDS (in windows of kVoxelCap); each corner
// then tests only its own cells' part of the window.  Empty cell rows cost two
// offset loads.  A corner visits its candidates in the same order as k_voxel
// (cell rows in (z, y) order, each in sorted order), so the two give identical
// fields.
constexpr int kVoxelCap = 1024;
constexpr int kVoxelRows = 64;  // cell rows whose spans are loaded up front (9 when R <= the cell edge)

__global__ void __launch_bounds__(kVoxelBD) k_voxel_rows(PhysPlan P, VoxelPlan V) {
  __shared__ float s_x[kVoxelCap], s_y[kVoxelCap], s_z[kVoxelCap];
  __shared__ uint32_t s_ra[kVoxelRows], s_rb[kVoxelRows];
  const DScene& S = P.scenes[0];
  const int tid = threadIdx.x;
  const uint32_t nx = (uint32_t)V.dims[0];
  const uint32_t ix0 = blockIdx.x * kVoxelBD, iy = blockIdx.y, iz = blockIdx.z;
  const uint32_t ix = ix0 + tid;
  const bool act = ix < nx;
  const uint32_t ixl = min(ix0 + kVoxelBD - 1u, nx - 1u);  // last corner of the segment
  float qx, qy, qz, qx0, qx1;
  {
#pragma clang fp contract(off)
    qx = V.mn[0] + (float)(act ? ix : ixl) * V.gs;
    qy = V.mn[1] + (float)iy * V.gs;
    qz = V.mn[2] + (float)iz * V.gs;
    qx0 = V.mn[0] + (float)ix0 * V.gs;
    qx1 = V.mn[0] + (float)ixl * V.gs;
  }
  const int y0 = cell_coord(qy - V.reach, S.g.mn[1], S.g.inv, S.g.dim[1]);
  const int y1 = cell_coord(qy + V.reach, S.g.mn[1], S.g.inv, S.g.dim[1]);
  const int z0 = cell_coord(qz - V.reach, S.g.mn[2], S.g.inv, S.g.dim[2]);
  const int z1 = cell_coord(qz + V.reach, S.g.mn[2], S.g.inv, S.g.dim[2]);
  const int sx0 = cell_coord(qx0 - V.reach, S.g.mn[0], S.g.inv, S.g.dim[0]);
  const int sx1 = cell_coord(qx1 + V.reach, S.g.mn[0], S.g.inv, S.g.dim[0]);
  const int tx0 = cell_coord(qx - V.reach, S.g.mn[0], S.g.inv, S.g.dim[0]);
  const int tx1 = cell_coord(qx + V.reach, S.g.mn[0], S.g.inv, S.g.dim[0]);
  const uint32_t* __restrict__ off = P.off + S.obase;
  // the segment's span of each cell row, loaded at once (one latency for the
  // whole stencil); a segment with no particle in reach is done here
  const int nyr = y1 - y0 + 1, nrows = nyr * (z1 - z0 + 1);
  const bool staged = nrows <= kVoxelRows;
  if (staged && tid < nrows) {
    const int y = y0 + tid % nyr, z = z0 + tid / nyr;
    s_ra[tid] = off[hash3(S.g, sx0, y, z)];
    s_rb[tid] = off[hash3(S.g, sx1, y, z) + 1];
  }
  __syncthreads();
  if (staged) {
    uint32_t any = 0;
    for (int r = 0; r < nrows; ++r) any |= s_rb[r] - s_ra[r];
    if (uniform_u32(any) == 0) {
      if (act) V.phi[(size_t)ix + (size_t)nx * ((size_t)iy + (size_t)V.dims[1] * iz)] = __builtin_huge_valf();
      return;  // the whole block
    }
  }
  float sk = 0.0f, sx = 0.0f, sy = 0.0f, sz = 0.0f;
  for (int z = z0; z <= z1; ++z)
    for (int y = y0; y <= y1; ++y) {
      // the segment's span of this cell row, and this corner's part of it
      const int r = (z - z0) * nyr + (y - y0);
      const uint32_t ra = uniform_u32(staged ? s_ra[r] : off[hash3(S.g, sx0, y, z)]);
      const uint32_t rb = uniform_u32(staged ? s_rb[r] : off[hash3(S.g, sx1, y, z) + 1]);
      if (ra >= rb) continue;
      // (a thread past the row's last corner only helps to stage)
      const uint32_t ta = act ? off[hash3(S.g, tx0, y, z)] : 0u, tb = act ? off[hash3(S.g, tx1, y, z) + 1] : 0u;
      for (uint32_t c0 = ra; c0 < rb; c0 += kVoxelCap) {
        const uint32_t len = min((uint32_t)kVoxelCap, rb - c0);
        __syncthreads();
        for (uint32_t e = tid; e < len; e += kVoxelBD) {
          const uint32_t j = S.pbase + c0 + e;
          s_x[e] = P.sx[j];
          s_y[e] = P.sy[j];
          s_z[e] = P.sz[j];
        }
        __syncthreads();
        const uint32_t a = max(ta, c0), b = min(tb, c0 + len);
        for (uint32_t jj = a; jj < b; ++jj) {
          const uint32_t e = jj - c0;
          const float dx = s_x[e] - qx, dy = s_y[e] - qy, dz = s_z[e] - qz;
          const float d2 = dist2_exact(dx, dy, dz);
          if (d2 < V.R2) {
            const float t = (V.R2 - d2) * V.inv_R2;
            const float k = t * t * t;
            sk += k;
            sx += k * dx;
            sy += k * dy;
            sz += k * dz;
          }
        }
      }
    }
  if (act) {
    const size_t c = (size_t)ix + (size_t)nx * ((size_t)iy + (size_t)V.dims[1] * iz);
    V.phi[c] = sk > 0.0f ? sqrtf(sx * sx + sy * sy + sz * sz) / sk - V.r : __builtin_huge_valf();
  }
}

void launch_voxel(const PhysPlan& P, const VoxelPlan& V, hipStream_t st) {
  if (!V.phi || !V.n) return;
  if (V.dims[1] <= 65535 && V.dims[2] <= 65535) {
    const dim3 grid((V.dims[0] + kVoxelBD - 1) / kVoxelBD, V.dims[1], V.dims[2]);
    hipLaunchKernelGGL(k_voxel_rows, grid, dim3(kVoxelBD), 0, st, P, V);
  } else {
    hipLaunchKernelGGL(k_voxel, dim3((V.n + kVoxelBD - 1) / kVoxelBD), dim3(kVoxelBD), 0, st, P, V);
  }
}

}  // namespace sph
