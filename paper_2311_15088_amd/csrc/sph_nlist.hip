// sph_nlist.hip -- the paper's materialised neighbour lists as alternative
// forms of the fluid passes, kept beside the tiled cell gather as ablations.
//
//  * Sorted list (the "Neighbor Search with Sorting" section): on the
//    counting-sorted particles, count each particle's neighbours over its 27
//    cells, scan the counts into list offsets, fill the list, then run the
//    density and the force pass over the list.
//  * Bucket list (the "Neighbor Search" section): cell buckets of a fixed
//    capacity, filled through one atomic slot per particle, and a list of
//    27 x capacity entries per particle filled from the 27 buckets around it.
//
// A list holds sorted indices and includes the particle itself (r^2 = 0 < h^2):
// the density sum takes it at its place and the force pass skips it (r^2 > 0).
// The sorted list visits the candidates in the tiled passes' order (halo rows
// in (dz, dy) order, each row's cells in x order, each cell in sorted order),
// so its densities, forces and new state are bit-identical to theirs.  The
// bucket list visits a cell's particles in slot order, which the atomics
// decide, so its sums differ from them by rounding only.
//
// One thread per particle, in cell order; every neighbour is gathered from
// the global arrays (the paper's design), not staged in LDS.
#include <hip/hip_ext.h>

#include "sph_fluid_impl.hpp"

namespace sph {

constexpr int kListBD = 256;
constexpr int kListChunk = 1024;  // counts per scan chunk (4 per thread)

// f(a, b) for each halo row [a, b) of sorted indices around cell (cx, cy, cz),
// rows in (dz, dy) order; a row is the cells cx - 1 .. cx + 1 inside the grid
template <class F>
__device__ __forceinline__ void for_each_row(const PhysPlan& P, const DScene& S, int cx, int cy, int cz, F&& f) {
  const uint32_t* __restrict__ off = P.off + S.obase;
  const int x0 = max(cx - 1, 0), x1 = min(cx + 1, S.g.dim[0] - 1);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = cy + dy, z = cz + dz;
      if (y < 0 || y >= S.g.dim[1] || z < 0 || z >= S.g.dim[2]) continue;
      f(S.pbase + off[hash3(S.g, x0, y, z)], S.pbase + off[hash3(S.g, x1, y, z) + 1]);
    }
}

// ------------------------------------------------------------- sorted list --

// FILL = false: lcnt[i] = number of j in the 27 cells with r_ij^2 < h^2;
// FILL = true: the same j, in order, to list[loff[i] ..] (entries past the
// buffer are dropped; the scan has flagged that case)
template <bool FILL>
__global__ void __launch_bounds__(kListBD) k_list_sorted(PhysPlan P, ListPlan L) {
  const uint32_t i = blockIdx.x * kListBD + threadIdx.x;
  if (i >= P.nf) return;
  const DScene& S = P.scenes[find_set(P.fprefix, P.nscenes, i)];
  const float xi = P.sx[i], yi = P.sy[i], zi = P.sz[i];
  const float h2 = S.h2;
  int cx, cy, cz;
  cell_of(S.g, xi, yi, zi, cx, cy, cz);
  uint32_t k = 0;
  const uint64_t o = FILL ? L.loff[i] : 0;
  for_each_row(P, S, cx, cy, cz, [&](uint32_t a, uint32_t b) {
    for (uint32_t j = a; j < b; ++j) {
      const float r2 = dist2_exact(P.sx[j] - xi, P.sy[j] - yi, P.sz[j] - zi);
      if (r2 < h2) {
        if (FILL && o + k < L.list_cap) L.list[o + k] = j;
        ++k;
      }
    }
  });
  if (!FILL) L.lcnt[i] = k;
}

// block-wide exclusive scan of one value per thread; returns the block total
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t& excl, uint32_t* s_w) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t t = __shfl_up(inc, d);
    if (lane >= d) inc += t;
  }
  if (lane == kWave - 1) s_w[wave] = inc;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kListBD / kWave; ++w) {
    before += w < wave ? s_w[w] : 0u;
    total += s_w[w];
  }
  excl = before + inc - v;
  return total;
}

// lsum[c] = sum of the counts of chunk c
__global__ void __launch_bounds__(kListBD) k_list_scan_reduce(ListPlan L, uint32_t n) {
  __shared__ uint32_t s_w[kListBD / kWave];
  const uint32_t e0 = blockIdx.x * kListChunk + threadIdx.x * 4;
  uint32_t v = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (e0 + q < n) v += L.lcnt[e0 + q];
  uint32_t excl;
  const uint32_t total = block_exscan(v, excl, s_w);
  if (threadIdx.x == 0) L.lsum[blockIdx.x] = total;
}

// loff[e] = sum of the counts before e; each chunk adds up the sums of the
// chunks before it itself.  The last chunk writes loff[n] and flags a total
// larger than the list buffer.
__global__ void __launch_bounds__(kListBD) k_list_scan_apply(ListPlan L, uint32_t n) {
  __shared__ uint32_t s_w[kListBD / kWave];
  __shared__ uint32_t s_base;
  uint32_t part = 0;
  for (uint32_t c = threadIdx.x; c < blockIdx.x; c += kListBD) part += L.lsum[c];
  uint32_t excl;
  const uint32_t base = block_exscan(part, excl, s_w);
  if (threadIdx.x == 0) s_base = base;
  __syncthreads();  // every wave has read s_w before it is reused
  const uint32_t e0 = blockIdx.x * kListChunk + threadIdx.x * 4;
  uint32_t c[4], v = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c[q] = e0 + q < n ? L.lcnt[e0 + q] : 0u;
    v += c[q];
  }
  const uint32_t total = block_exscan(v, excl, s_w);
  uint32_t o = s_base + excl;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (e0 + q < n) L.loff[e0 + q] = o;
    o += c[q];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const uint64_t all = (uint64_t)s_base + total;
    L.loff[n] = (uint32_t)all;
    if (all > L.list_cap) L.status[kListOverflow] = 1u;
  }
}

// ------------------------------------------------------------- bucket list --

__global__ void k_bucket_clear(ListPlan L) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < L.ncells; c += gridDim.x * blockDim.x) L.bcnt[c] = 0u;
}

// the paper's hash-grid insertion: an atomic slot in the particle's cell; a
// particle past the capacity is flagged (and left out)
__global__ void __launch_bounds__(kListBD) k_bucket_fill(PhysPlan P, ListPlan L) {
  const uint32_t i = blockIdx.x * kListBD + threadIdx.x;
  if (i >= P.nf) return;
  const DScene& S = P.scenes[find_set(P.fprefix, P.nscenes, i)];
  int cx, cy, cz;
  cell_of(S.g, P.sx[i], P.sy[i], P.sz[i], cx, cy, cz);
  const uint32_t c = S.cbase + hash3(S.g, cx, cy, cz);
  const uint32_t slot = atomicAdd(&L.bcnt[c], 1u);
  if (slot < L.cap) L.bucket[(size_t)c * L.cap + slot] = i;
  else atomicOr(&L.status[kBucketOverflow], 1u);
}

// list[i][0 .. lcnt[i]) from the 27 buckets around the particle, cells in
// (z, y, x) order, each bucket in slot order
__global__ void __launch_bounds__(kListBD) k_list_bucket(PhysPlan P, ListPlan L) {
  const uint32_t i = blockIdx.x * kListBD + threadIdx.x;
  if (i >= P.nf) return;
  const DScene& S = P.scenes[find_set(P.fprefix, P.nscenes, i)];
  const float xi = P.sx[i], yi = P.sy[i], zi = P.sz[i];
  const float h2 = S.h2;
  int cx, cy, cz;
  cell_of(S.g, xi, yi, zi, cx, cy, cz);
  const size_t o = (size_t)i * 27u * L.cap;
  uint32_t k = 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = cx + dx, y = cy + dy, z = cz + dz;
        if (x < 0 || x >= S.g.dim[0] || y < 0 || y >= S.g.dim[1] || z < 0 || z >= S.g.dim[2]) continue;
        const uint32_t c = S.cbase + hash3(S.g, x, y, z);
        const uint32_t m = min(L.bcnt[c], L.cap);
        const uint32_t* __restrict__ bk = L.bucket + (size_t)c * L.cap;
        for (uint32_t s = 0; s < m; ++s) {
          const uint32_t j = bk[s];
          const float r2 = dist2_exact(P.sx[j] - xi, P.sy[j] - yi, P.sz[j] - zi);
          if (r2 < h2) L.list[o + k++] = j;
        }
      }
  L.lcnt[i] = k;
}

// ------------------------------------------------------- passes over lists --

__device__ __forceinline__ uint64_t list_start(const ListPlan& L, uint32_t i) {
  return L.mode == kSearchSortedList ? (uint64_t)L.loff[i] : (uint64_t)i * 27u * L.cap;
}

// entries of a list that lie in the buffer: a sorted list whose total
// overflowed the buffer (flagged by the scan) is cut at the buffer's end, so
// that reads stay in bounds; a bucket list always fits its 27 x cap entries
__device__ __forceinline__ uint32_t list_len(const ListPlan& L, uint64_t start, uint32_t n) {
  if (start + n <= L.list_cap) return n;
  return start < L.list_cap ? (uint32_t)(L.list_cap - start) : 0u;
}

// density + EOS (the sums of the tiled density pass, over the list)
__global__ void __launch_bounds__(kListBD) k_list_density(PhysPlan P, ListPlan L) {
  const uint32_t i = blockIdx.x * kListBD + threadIdx.x;
  unsigned long long npairs = 0;
  if (i < P.nf) {
    const DScene& S = P.scenes[find_set(P.fprefix, P.nscenes, i)];
    const float xi = P.sx[i], yi = P.sy[i], zi = P.sz[i];
    const float h2 = S.h2;
    const uint32_t n = L.lcnt[i];
    const uint64_t start = list_start(L, i);
    const uint32_t m = list_len(L, start, n);
    const uint32_t* __restrict__ lst = L.list + start;
    float acc = 0.0f;
    for (uint32_t k = 0; k < m; ++k) {
      const uint32_t j = lst[k];
      const float r2 = dist2_exact(P.sx[j] - xi, P.sy[j] - yi, P.sz[j] - zi);
      const float t3 = fmaxf(h2 - r2, 0.0f);
      acc += t3 * t3 * t3;
    }
    // the particle itself is on its list: it adds W(0) but is not its own neighbour
    P.rho[i] = S.c6m * acc;
    P.nbr[i] = n - 1;
    npairs = n - 1;
  }
  if (P.pairs) {
    npairs = wave_sum_u64(npairs);
    if ((threadIdx.x & (kWave - 1)) == 0 && npairs) atomicAdd(P.pairs, npairs);
  }
}

// pressure + viscosity over the list, the agents' reaction, integration
__global__ void __launch_bounds__(kListBD) k_list_force(PhysPlan P, ListPlan L) {
  const uint32_t i = blockIdx.x * kListBD + threadIdx.x;
  if (i >= P.nf) return;
  const DScene& S = P.scenes[find_set(P.fprefix, P.nscenes, i)];
  const float xi = P.sx[i], yi = P.sy[i], zi = P.sz[i];
  const float vxi = P.svx[i], vyi = P.svy[i], vzi = P.svz[i];
  const float di = P.rho[i] - S.rho0;
  const float inv_h = S.inv_h, cpk_h = S.cpk_h, cvmu = S.cvmu;
  // scaled as in the tiled force pass, so that both forms give the same sums
  const float ci = mul_rn(cpk_h, di), cvx = mul_rn(cvmu, vxi), cvy = mul_rn(cvmu, vyi), cvz = mul_rn(cvmu, vzi);
  const uint64_t start = list_start(L, i);
  const uint32_t m = list_len(L, start, L.lcnt[i]);
  const uint32_t* __restrict__ lst = L.list + start;
  float acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  for (uint32_t k = 0; k < m; ++k) {
    const uint32_t j = lst[k];
    const float dx = P.sx[j] - xi, dy = P.sy[j] - yi, dz = P.sz[j] - zi;
    const float r2 = dist2_exact(dx, dy, dz);
    if (r2 > 0.0f) {
      // (m/rho_j) w [(Cp k h d_i + Cp k h d_j) w / r * r_ij - (Cv mu v_i - Cv mu v_j)],
      // r_ij = -(dx, dy, dz)
      const float rhoj = P.rho[j];
      const float mr = S.m * __builtin_amdgcn_rcpf(rhoj), pj = mul_rn(cpk_h, rhoj - S.rho0);
      const float ir = rsqrt_normal(r2);
      const float w = 1.0f - r2 * ir * inv_h;
      const float sc = mr * w;
      const float fp = (ci + pj) * w * ir;
      acc0 += sc * (-fp * dx - (cvx - mul_rn(cvmu, P.svx[j])));
      acc1 += sc * (-fp * dy - (cvy - mul_rn(cvmu, P.svy[j])));
      acc2 += sc * (-fp * dz - (cvz - mul_rn(cvmu, P.svz[j])));
    }
  }
  const float irho = __builtin_amdgcn_rcpf(di + S.rho0);
  const float ax = acc0 * irho, ay = acc1 * irho, az = acc2 * irho;
  const FluidPoint F{xi, yi, zi, vxi, vyi, vzi, di, S.m * irho};
  AgentReaction R;
  if (S.na) agents_from_grid(P, S, F, R);
  integrate_store(P, S, i, F, ax, ay, az, R);
}

// ---------------------------------------------------------------- launches --

static dim3 per_particle(uint32_t n) { return dim3((n + kListBD - 1) / kListBD); }

uint32_t list_scan_chunks(uint32_t n) { return (n + kListChunk - 1) / kListChunk; }

void launch_list_build(const PhysPlan& P, const ListPlan& L, hipStream_t st) {
  if (!P.nf) return;
  if (L.mode == kSearchSortedList) {
    const uint32_t chunks = list_scan_chunks(P.nf);
    hipLaunchKernelGGL(k_list_sorted<false>, per_particle(P.nf), dim3(kListBD), 0, st, P, L);
    hipLaunchKernelGGL(k_list_scan_reduce, dim3(chunks), dim3(kListBD), 0, st, L, P.nf);
    hipLaunchKernelGGL(k_list_scan_apply, dim3(chunks), dim3(kListBD), 0, st, L, P.nf);
    hipLaunchKernelGGL(k_list_sorted<true>, per_particle(P.nf), dim3(kListBD), 0, st, P, L);
  } else {
    hipLaunchKernelGGL(k_bucket_clear, dim3(std::min<uint32_t>((L.ncells + 255) / 256, 4096u)), dim3(256), 0, st, L);
    hipLaunchKernelGGL(k_bucket_fill, per_particle(P.nf), dim3(kListBD), 0, st, P, L);
    hipLaunchKernelGGL(k_list_bucket, per_particle(P.nf), dim3(kListBD), 0, st, P, L);
  }
}

static void launch_timed(const void* fn, uint32_t n, void** args, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  if (start || stop) (void)hipExtLaunchKernel(fn, per_particle(n), dim3(kListBD), args, 0, st, start, stop, 0);
  else (void)hipLaunchKernel(fn, per_particle(n), dim3(kListBD), args, 0, st);
}

void launch_list_density(const PhysPlan& P, const ListPlan& L, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  if (!P.nf) return;
  void* args[] = {(void*)&P, (void*)&L};
  launch_timed((const void*)k_list_density, P.nf, args, st, start, stop);
}

void launch_list_force(const PhysPlan& P, const ListPlan& L, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  if (!P.nf) return;
  void* args[] = {(void*)&P, (void*)&L};
  launch_timed((const void*)k_list_force, P.nf, args, st, start, stop);
}

}  // namespace sph
