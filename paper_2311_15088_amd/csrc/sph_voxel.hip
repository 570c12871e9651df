// sph_voxel.hip -- voxel density at cube corners ("Voxel Density" section):
// at corner x, phi(x) = |x - xbar| - rbar with xbar the k-weighted mean of the
// particle positions within radius R, k(s) = (1 - s^2)^3, s = |x - x_i| / R,
// and rbar = r (every particle has radius r).  A corner with no particle
// within R gets +inf.
//
// A second neighbour gather on the step's cell table, in three forms that
// give the same field: k_voxel_tile (64 x 2 x 2 corner blocks sharing their
// LDS-staged cell rows; launched whenever a block's cell rows fit the table
// of row spans), k_voxel_rows (one corner-row segment per workgroup; grids of
// up to 65,535 corners in y and z) and k_voxel (one thread per corner reading
// the particles through the caches; any grid).  The sums are taken
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

// Block-tiled form: a workgroup takes a 64 x 2 x 2 block of corners, one
// wavefront per corner row segment, and stages each cell row that any of them
// reaches once for all four rows (a cell row is shared by corners in y and z
// as well as in x).  A wavefront skips the cell rows outside its corners' y
// and z ranges, so every corner still visits its candidates in k_voxel's
// order and the field is the same.
constexpr int kTileX = 64, kTileY = 2, kTileZ = 2;
static_assert(kTileX * kTileY * kTileZ == kVoxelBD, "one corner per thread");

__global__ void __launch_bounds__(kVoxelBD) k_voxel_tile(PhysPlan P, VoxelPlan V) {
  __shared__ float s_x[kVoxelCap], s_y[kVoxelCap], s_z[kVoxelCap];
  __shared__ uint32_t s_ra[kVoxelRows], s_rb[kVoxelRows];
  const DScene& S = P.scenes[0];
  const int tid = threadIdx.x;
  const uint32_t nx = (uint32_t)V.dims[0], ny = (uint32_t)V.dims[1], nz = (uint32_t)V.dims[2];
  const uint32_t bx = blockIdx.x * kTileX, by = blockIdx.y * kTileY, bz = blockIdx.z * kTileZ;
  // corners of the block (clamped to the grid for the ranges) and of this thread
  const uint32_t lx = min(bx + kTileX - 1u, nx - 1u), ly = min(by + kTileY - 1u, ny - 1u),
                 lz = min(bz + kTileZ - 1u, nz - 1u);
  const uint32_t ix = bx + (uint32_t)(tid % kTileX), iy = by + (uint32_t)((tid / kTileX) % kTileY),
                 iz = bz + (uint32_t)(tid / (kTileX * kTileY));
  const bool act = ix < nx && iy < ny && iz < nz;
  float q[3], b0[3], b1[3];
  {
#pragma clang fp contract(off)
    q[0] = V.mn[0] + (float)min(ix, lx) * V.gs;
    q[1] = V.mn[1] + (float)min(iy, ly) * V.gs;
    q[2] = V.mn[2] + (float)min(iz, lz) * V.gs;
    b0[0] = V.mn[0] + (float)bx * V.gs;
    b0[1] = V.mn[1] + (float)by * V.gs;
    b0[2] = V.mn[2] + (float)bz * V.gs;
    b1[0] = V.mn[0] + (float)lx * V.gs;
    b1[1] = V.mn[1] + (float)ly * V.gs;
    b1[2] = V.mn[2] + (float)lz * V.gs;
  }
  int blo[3], bhi[3], tlo[3], thi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    blo[k] = cell_coord(b0[k] - V.reach, S.g.mn[k], S.g.inv, S.g.dim[k]);
    bhi[k] = cell_coord(b1[k] + V.reach, S.g.mn[k], S.g.inv, S.g.dim[k]);
    tlo[k] = cell_coord(q[k] - V.reach, S.g.mn[k], S.g.inv, S.g.dim[k]);
    thi[k] = cell_coord(q[k] + V.reach, S.g.mn[k], S.g.inv, S.g.dim[k]);
  }
  const uint32_t* __restrict__ off = P.off + S.obase;
  const int nyr = bhi[1] - blo[1] + 1, nrows = nyr * (bhi[2] - blo[2] + 1);
  // the host picks this form when a block's rows fit kVoxelRows; should
  // rounding give one more, the spans are read from the table directly
  const bool staged = nrows <= kVoxelRows;
  if (staged && tid < nrows) {
    const int y = blo[1] + tid % nyr, z = blo[2] + tid / nyr;
    s_ra[tid] = off[hash3(S.g, blo[0], y, z)];
    s_rb[tid] = off[hash3(S.g, bhi[0], y, z) + 1];
  }
  __syncthreads();
  if (staged) {
    uint32_t any = 0;
    for (int r = 0; r < nrows; ++r) any |= s_rb[r] - s_ra[r];
    if (uniform_u32(any) == 0) {
      if (act) V.phi[(size_t)ix + (size_t)nx * ((size_t)iy + (size_t)ny * iz)] = __builtin_huge_valf();
      return;  // the whole block
    }
  }
  float sk = 0.0f, sx = 0.0f, sy = 0.0f, sz = 0.0f;
  for (int z = blo[2]; z <= bhi[2]; ++z)
    for (int y = blo[1]; y <= bhi[1]; ++y) {
      const int r = (z - blo[2]) * nyr + (y - blo[1]);
      const uint32_t ra = uniform_u32(staged ? s_ra[r] : off[hash3(S.g, blo[0], y, z)]);
      const uint32_t rb = uniform_u32(staged ? s_rb[r] : off[hash3(S.g, bhi[0], y, z) + 1]);
      if (ra >= rb) continue;
      // this corner's part of the row (none if the row is outside its y / z range)
      bool mine = act && y >= tlo[1] && y <= thi[1] && z >= tlo[2] && z <= thi[2];
      // the row's cells that the sphere of radius R around the corner meets:
      // its distance to the row's y / z slab (less a margin of 1e-3 cells for
      // the rounding of the cell bounds) leaves a half-width e along x
      int x0 = tlo[0], x1 = thi[0];
      if (mine) {
        const float tol = 1e-3f * S.g.cell;
        const float ylo = S.g.mn[1] + (float)y * S.g.cell, zlo = S.g.mn[2] + (float)z * S.g.cell;
        const float dy = fmaxf(fmaxf(ylo - q[1], q[1] - (ylo + S.g.cell)) - tol, 0.0f);
        const float dz = fmaxf(fmaxf(zlo - q[2], q[2] - (zlo + S.g.cell)) - tol, 0.0f);
        const float e2 = V.reach * V.reach - (dy * dy + dz * dz);
        if (e2 <= 0.0f) {
          mine = false;
        } else {
          const float e = sqrtf(e2);
          x0 = cell_coord(q[0] - e, S.g.mn[0], S.g.inv, S.g.dim[0]);
          x1 = cell_coord(q[0] + e, S.g.mn[0], S.g.inv, S.g.dim[0]);
        }
      }
      const uint32_t ta = mine ? off[hash3(S.g, x0, y, z)] : 0u;
      const uint32_t tb = mine ? off[hash3(S.g, x1, y, z) + 1] : 0u;
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
          const float dx = s_x[e] - q[0], dy = s_y[e] - q[1], dz = s_z[e] - q[2];
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
    const size_t c = (size_t)ix + (size_t)nx * ((size_t)iy + (size_t)ny * iz);
    V.phi[c] = sk > 0.0f ? sqrtf(sx * sx + sy * sy + sz * sz) / sk - V.r : __builtin_huge_valf();
  }
}

void launch_voxel(const PhysPlan& P, const VoxelPlan& V, hipStream_t st) {
  if (!V.phi || !V.n) return;
  if (V.tile_ok) {
    const dim3 grid((V.dims[0] + kTileX - 1) / kTileX, (V.dims[1] + kTileY - 1) / kTileY,
                    (V.dims[2] + kTileZ - 1) / kTileZ);
    hipLaunchKernelGGL(k_voxel_tile, grid, dim3(kVoxelBD), 0, st, P, V);
  } else if (V.dims[1] <= 65535 && V.dims[2] <= 65535) {
    const dim3 grid((V.dims[0] + kVoxelBD - 1) / kVoxelBD, V.dims[1], V.dims[2]);
    hipLaunchKernelGGL(k_voxel_rows, grid, dim3(kVoxelBD), 0, st, P, V);
  } else {
    hipLaunchKernelGGL(k_voxel, dim3((V.n + kVoxelBD - 1) / kVoxelBD), dim3(kVoxelBD), 0, st, P, V);
  }
}

}  // namespace sph
