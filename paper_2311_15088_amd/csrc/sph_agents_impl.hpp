// sph_agents_impl.hpp -- the agents' step as a device function shared by the
// per-phase agents kernel and the fused step kernel:
//   one wavefront per agent: separation / alignment / cohesion over the agents
//   in range and the coupling force summed over the fluid within r_couple
//   (Section "Boid Motion and Agent Fluid Interaction"), then u += dt a, speed
//   clamp, y += dt u, walls.
#pragma once
#include "sph_fluid_impl.hpp"  // wave reductions, rsqrt_normal

namespace sph {

// ----------------------------------------------------------------------------
// Agents: one wavefront per agent, agents taken in cell order.
//
// Both gathers (boid rules over the 27 agent cells, coupling over the fluid
// cells within r_couple) read stencil rows, each a contiguous span of the
// cell-sorted arrays.  The wave concatenates the rows of a stencil (lane r
// holds row r; an exclusive scan of the lengths goes to LDS) and lane l takes
// elements l, l + 64, ... of the concatenation, kGatherBatch at a time with
// all their loads in flight together (the coupling gather loads a fluid
// element's density and velocity with its position; the boid gather loads an
// agent's velocity only when it is within range).  Each lane sums its elements in that
// order and the wave reductions run in a fixed order, so the results are
// deterministic.
// ----------------------------------------------------------------------------
constexpr int kGatherBatch = 3;

template <int BD>
__device__ __forceinline__ void agents_block(const PhysPlan& P, uint32_t blk) {
  __shared__ uint32_t s_pre[BD / kWave][kWave + 1], s_dlt[BD / kWave][kWave];
  const uint32_t ga_ = (blk * BD + threadIdx.x) / kWave;  // agent handled by this wave
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = (int)(threadIdx.x / kWave);
  if (ga_ >= P.na) return;
  const uint32_t gi = uniform_u32(ga_);
  const int s = (int)uniform_u32((uint32_t)find_set(P.aprefix, P.nscenes, gi));
  const DScene& S = P.scenes[s];
  // waves take the agents in cell order, so that neighbouring waves read
  // neighbouring fluid and agent cells; the agent's own id names its slot
  // (its state is read from the cell-ordered copy at the wave's own index,
  // alongside the id rather than after it)
  const uint32_t w = S.abase + (gi - P.aprefix[s]);
  const uint32_t la = uniform_u32(P.asid[w]);
  const uint32_t a = S.abase + la;
  const float ya[3] = {P.asx[w], P.asy[w], P.asz[w]};
  const float ua[3] = {P.asvx[w], P.asvy[w], P.asvz[w]};

  // bounds of the coupling stencil's first 64 fluid rows (lane q holds row q):
  // loaded now, together with the boid rows below, and used after them
  const uint32_t* __restrict__ off = P.off + S.obase;
  int fx, fy, fz;
  cell_of(S.g, ya[0], ya[1], ya[2], fx, fy, fz);
  const int ns = S.ns_c, side = 2 * ns + 1, nrows = side * side;
  const int fx0 = max(fx - ns, 0), fx1 = min(fx + ns, S.g.dim[0] - 1);
  // each row is cut to the cells that can hold a point within r_couple: a
  // row whose y/z slab lies farther is empty, and in the others only the
  // cells meeting [x - e, x + e], e = sqrt(r_couple^2 - d_yz^2), are read
  // (a margin of 10^-3 cells absorbs float32 rounding, so the coupling set is
  // exactly that of the full stencil)
  const float gd = S.g.cell, gslack = 1e-3f * gd;
  const float rcut = sqrtf(S.rc2) * (1.0f + 1e-5f);
  auto fluid_row = [&](int q, uint32_t& r0, uint32_t& r1) {
    r0 = r1 = 0;
    if (q < nrows) {
      const int y = fy + q % side - ns, z = fz + q / side - ns;
      if (y >= 0 && y < S.g.dim[1] && z >= 0 && z < S.g.dim[2]) {
        const float ylo = S.g.mn[1] + (float)y * gd, zlo = S.g.mn[2] + (float)z * gd;
        const float gy = fmaxf(fmaxf(ylo - ya[1], ya[1] - (ylo + gd)) - gslack, 0.0f);
        const float gz = fmaxf(fmaxf(zlo - ya[2], ya[2] - (zlo + gd)) - gslack, 0.0f);
        const float q2 = gy * gy + gz * gz;
        if (q2 < rcut * rcut) {
          const float e = __builtin_amdgcn_sqrtf(rcut * rcut - q2) + gslack;
          const int lo = max(fx0, (int)floorf((ya[0] - e - S.g.mn[0]) * S.g.inv));
          const int hi = min(fx1, (int)floorf((ya[0] + e - S.g.mn[0]) * S.g.inv));
          if (lo <= hi) {
            r0 = off[hash3(S.g, lo, y, z)];
            r1 = off[hash3(S.g, hi, y, z) + 1];
          }
        }
      }
    }
  };
  uint32_t rj0_first, rj1_first;
  fluid_row(lane, rj0_first, rj1_first);

  // --- boid rules over the agents in the 27 agent cells ---
  const uint32_t* __restrict__ aoff = P.aoff + S.aobase;
  int cx, cy, cz;
  cell_of(S.ga, ya[0], ya[1], ya[2], cx, cy, cz);
  float sep[3] = {0, 0, 0}, dv[3] = {0, 0, 0}, dp[3] = {0, 0, 0};
  uint32_t nsep = 0, nali = 0, ncoh = 0;
  {
    const float rsep2 = uniform_f(S.rsep2), rali2 = uniform_f(S.rali2), rcoh2 = uniform_f(S.rcoh2);
    const float inv_rsep = uniform_f(S.inv_rsep);
    const float rmax2 = fmaxf(rsep2, fmaxf(rali2, rcoh2));
    const int x0 = max(cx - 1, 0), x1 = min(cx + 1, S.ga.dim[0] - 1);
    uint32_t rb0 = 0, rb1 = 0;
    if (lane < 9) {
      // rows cut to the cells within the widest boid radius, as the fluid rows
      const int y = cy + (lane % 3) - 1, z = cz + (lane / 3) - 1;
      if (y >= 0 && y < S.ga.dim[1] && z >= 0 && z < S.ga.dim[2]) {
        const float ad = S.ga.cell, aslack = 1e-3f * ad;
        const float rmax = sqrtf(rmax2) * (1.0f + 1e-5f);
        const float ylo = S.ga.mn[1] + (float)y * ad, zlo = S.ga.mn[2] + (float)z * ad;
        const float gy = fmaxf(fmaxf(ylo - ya[1], ya[1] - (ylo + ad)) - aslack, 0.0f);
        const float gz = fmaxf(fmaxf(zlo - ya[2], ya[2] - (zlo + ad)) - aslack, 0.0f);
        const float q2 = gy * gy + gz * gz;
        if (q2 < rmax * rmax) {
          const float e = __builtin_amdgcn_sqrtf(rmax * rmax - q2) + aslack;
          const int lo = max(x0, (int)floorf((ya[0] - e - S.ga.mn[0]) * S.ga.inv));
          const int hi = min(x1, (int)floorf((ya[0] + e - S.ga.mn[0]) * S.ga.inv));
          if (lo <= hi) {
            rb0 = aoff[hash3(S.ga, lo, y, z)];
            rb1 = aoff[hash3(S.ga, hi, y, z) + 1];
          }
        }
      }
    }
    const FlatRows F = flat_rows(s_pre[wave], s_dlt[wave], lane, 9, S.abase + rb0, rb1 - rb0);
    int cur = 0;
    for (uint32_t t0 = 0; t0 < F.total; t0 += kGatherBatch * kWave) {
      uint32_t b[kGatherBatch], sid[kGatherBatch];
      bool ok[kGatherBatch], in[kGatherBatch];
      float dx[kGatherBatch], dy[kGatherBatch], dz[kGatherBatch], r2[kGatherBatch];
      float bvx[kGatherBatch], bvy[kGatherBatch], bvz[kGatherBatch];
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        const uint32_t t = t0 + (uint32_t)(u * kWave + lane);
        ok[u] = t < F.total;
        b[u] = ok[u] ? flat_index(F, t, cur) : 0u;
      }
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        if (ok[u]) {
          sid[u] = P.asid[b[u]];
          dx[u] = P.asx[b[u]];
          dy[u] = P.asy[b[u]];
          dz[u] = P.asz[b[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        in[u] = false;
        if (ok[u]) {
          dx[u] -= ya[0];
          dy[u] -= ya[1];
          dz[u] -= ya[2];
          r2[u] = dist2_exact(dx[u], dy[u], dz[u]);
          in[u] = sid[u] != la && r2[u] < rmax2;
        }
      }
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        if (in[u]) {
          bvx[u] = P.asvx[b[u]];
          bvy[u] = P.asvy[b[u]];
          bvz[u] = P.asvz[b[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < kGatherBatch; ++u) {
        if (!in[u]) continue;
        if (r2[u] < rsep2) {
          ++nsep;
          const float w = fmaxf(0.0f, 1.0f - sqrtf(r2[u]) * inv_rsep);
          sep[0] -= w * dx[u];
          sep[1] -= w * dy[u];
          sep[2] -= w * dz[u];
        }
        if (r2[u] < rali2) {
          ++nali;
          dv[0] += bvx[u] - ua[0];
          dv[1] += bvy[u] - ua[1];
          dv[2] += bvz[u] - ua[2];
        }
        if (r2[u] < rcoh2) {
          ++ncoh;
          dp[0] += dx[u];
          dp[1] += dy[u];
          dp[2] += dz[u];
        }
      }
    }
  }

  // --- coupling force: fluid particles within r_couple (fluid-grid stencil) ---
  // A learned closure, when its controller says so, replaces this gather.
  const bool surrogate = P.cl_state && P.cl_state[kClUse];
  const bool check = P.cl_state && P.cl_state[kClCheck];
  float F[3] = {0, 0, 0};
  uint32_t ncpl = 0;
  if (!surrogate) {
    const float rc2 = uniform_f(S.rc2), inv_rc = uniform_f(S.inv_rc), mr0 = uniform_f(S.m_over_rho0);
    const float m = uniform_f(S.m), rho0 = uniform_f(S.rho0), cpk_hc = uniform_f(S.cpk_hc);
    const float cvmu_c = uniform_f(S.cvmu_c);
    for (int g0 = 0; g0 < nrows; g0 += kWave) {
      uint32_t rj0 = rj0_first, rj1 = rj1_first;
      if (g0) fluid_row(g0 + lane, rj0, rj1);
      const FlatRows R = flat_rows(s_pre[wave], s_dlt[wave], lane, min(kWave, nrows - g0), S.pbase + rj0, rj1 - rj0);
      int cur = 0;
      for (uint32_t t0 = 0; t0 < R.total; t0 += kGatherBatch * kWave) {
        uint32_t j[kGatherBatch];
        bool ok[kGatherBatch], in[kGatherBatch];
        float dx[kGatherBatch], dy[kGatherBatch], dz[kGatherBatch], r2[kGatherBatch];
        float rh[kGatherBatch], vx[kGatherBatch], vy[kGatherBatch], vz[kGatherBatch];
#pragma unroll
        for (int u = 0; u < kGatherBatch; ++u) {
          const uint32_t t = t0 + (uint32_t)(u * kWave + lane);
          ok[u] = t < R.total;
          j[u] = ok[u] ? flat_index(R, t, cur) : 0u;
        }
        // density and velocity are loaded with the position, before the
        // distance test: after the row pruning about half the candidates
        // are within r_couple, and one round of dependent loads is saved
#pragma unroll
        for (int u = 0; u < kGatherBatch; ++u) {
          if (ok[u]) {
            dx[u] = P.sx[j[u]];
            dy[u] = P.sy[j[u]];
            dz[u] = P.sz[j[u]];
            rh[u] = P.rho[j[u]];
            vx[u] = P.svx[j[u]];
            vy[u] = P.svy[j[u]];
            vz[u] = P.svz[j[u]];
          }
        }
#pragma unroll
        for (int u = 0; u < kGatherBatch; ++u) {
          in[u] = false;
          if (ok[u]) {
            dx[u] -= ya[0];
            dy[u] -= ya[1];
            dz[u] -= ya[2];
            r2[u] = dist2_exact(dx[u], dy[u], dz[u]);
            in[u] = r2[u] < rc2;
          }
        }
#pragma unroll
        for (int u = 0; u < kGatherBatch; ++u) {
          if (!in[u]) continue;
          ++ncpl;
          if (r2[u] > 0.0f) {
            const float ir = rsqrt_normal(r2[u]);
            const float w = 1.0f - r2[u] * ir * inv_rc;
            // G_aj = (m/rho0)(m/rho_j) w [Cp k rc (0 + d_j) w / r (y_a - x_j) - Cv mu (u_a - v_j)]
            const float sc = mr0 * (m * __builtin_amdgcn_rcpf(rh[u])) * w;
            const float fp = cpk_hc * (rh[u] - rho0) * w * ir;
            F[0] += sc * (-fp * dx[u] - cvmu_c * (ua[0] - vx[u]));
            F[1] += sc * (-fp * dy[u] - cvmu_c * (ua[1] - vy[u]));
            F[2] += sc * (-fp * dz[u] - cvmu_c * (ua[2] - vz[u]));
          }
        }
      }
      // the LDS rows are rewritten by the next group of rows
      __builtin_amdgcn_wave_barrier();
    }
  }

  // --- obstacle avoidance: lane q < 27 takes obstacle cell q of the 27 around
  // the agent's cell; a cell counts twice if its centre is within r_sep, once
  // if within r_ali ("Boid Motion" section, obstacle avoidance) ---
  float ob[3] = {0.0f, 0.0f, 0.0f};
  if (P.obst) {
    if (lane < 27) {
      const int x = cx + lane % 3 - 1, y = cy + (lane / 3) % 3 - 1, z = cz + lane / 9 - 1;
      if (x >= 0 && x < S.ga.dim[0] && y >= 0 && y < S.ga.dim[1] && z >= 0 && z < S.ga.dim[2]) {
        const float4 o = P.obst[S.acbase + hash3(S.ga, x, y, z)];
        if (o.w > 0.0f) {
          float c[3];
          {
#pragma clang fp contract(off)
            c[0] = S.ga.mn[0] + ((float)x + 0.5f) * S.ga.cell;
            c[1] = S.ga.mn[1] + ((float)y + 0.5f) * S.ga.cell;
            c[2] = S.ga.mn[2] + ((float)z + 0.5f) * S.ga.cell;
          }
          const float d2 = dist2_exact(c[0] - ya[0], c[1] - ya[1], c[2] - ya[2]);
          const float om = d2 < S.rsep2 ? 2.0f : (d2 < S.rali2 ? 1.0f : 0.0f);
          ob[0] = om * o.x;
          ob[1] = om * o.y;
          ob[2] = om * o.z;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) ob[k] = wave_sum_f(ob[k]);
  }

  // --- wave reductions (fixed order: deterministic) ---
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    sep[k] = wave_sum_f(sep[k]);
    dv[k] = wave_sum_f(dv[k]);
    dp[k] = wave_sum_f(dp[k]);
    F[k] = wave_sum_f(F[k]);
  }
  nsep = wave_sum_u(nsep);
  nali = wave_sum_u(nali);
  ncoh = wave_sum_u(ncoh);
  ncpl = wave_sum_u(ncpl);
  if (lane != 0) return;

  if (surrogate) {
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] = P.cl_fhat[3 * a + k];
  } else if (check) {
    float e = 0.0f, f = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float d = P.cl_fhat[3 * a + k] - F[k];
      e += d * d;
      f += F[k] * F[k];
    }
    P.cl_err[2 * a] = e;
    P.cl_err[2 * a + 1] = f;
  }

  const float ia = nali ? 1.0f / (float)nali : 0.0f;
  const float ic = ncoh ? 1.0f / (float)ncoh : 0.0f;
  float steer[3], un[3], yn[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    steer[k] = S.wsep * sep[k] + S.wali * dv[k] * ia + S.wcoh * dp[k] * ic;
    if (P.obst) steer[k] += P.obst_w * ob[k];
    un[k] = ua[k] + S.dt * (steer[k] + S.cf * F[k] * S.inv_m);
  }
  const float sp = sqrtf(un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
  float scale = 1.0f;
  if (sp > S.vmax) scale = S.vmax / sp;
  else if (sp > 0.0f && sp < S.vmin) scale = S.vmin / sp;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    un[k] *= scale;
    yn[k] = ya[k] + S.dt * un[k];
    wall(yn[k], un[k], S.bmin[k], S.bmax[k], S.e);
  }
  P.agx[a] = yn[0];
  P.agy[a] = yn[1];
  P.agz[a] = yn[2];
  P.aux[a] = un[0];
  P.auy[a] = un[1];
  P.auz[a] = un[2];
  if (P.d_steer) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      P.d_steer[3 * a + k] = steer[k];
      P.d_force[3 * a + k] = F[k];
    }
    P.d_acnt[4 * a + 0] = nsep;
    P.d_acnt[4 * a + 1] = nali;
    P.d_acnt[4 * a + 2] = ncoh;
    P.d_acnt[4 * a + 3] = ncpl;
  }
}

}  // namespace sph
