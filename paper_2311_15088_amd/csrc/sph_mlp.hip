// sph_mlp.hip -- the learned coupling closure on the GPU: per-agent features,
// a bfloat16 MFMA GEMM with fused epilogues, the MLP forward / backward passes,
// Adam, the network of a step in one MFMA kernel, and the per-step closure
// controller kernels.
//
// GEMM: a 256-thread workgroup computes a 64 x 64 tile of C as 2 x 2
// wavefronts of 32 x 32, each a 2 x 2 grid of v_mfma_f32_16x16x32_bf16.  Every
// K step of 32 stages the A tile (64 rows x 32 k) and the B tile (64 columns x
// 32 k, stored k-contiguous) in LDS; rows are padded to 40 elements so that
// the 16 lanes of a fragment read land on distinct banks.  A lane's fragment
// is 8 consecutive k of one row (A) or one column (B); the same k order is
// used for both operands, so the product does not depend on how the
// instruction distributes k over lanes.  The result fragment of a 16 x 16
// tile holds rows 4 (lane / 16) + i, column lane % 16.
#include <math.h>

#include "sph_device.hpp"
#include "sph_mlp.hpp"

namespace sph {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// float32 -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// erf by Abramowitz and Stegun, Handbook of Mathematical Functions, formula
// 7.1.26: 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p x), for x >= 0,
// odd in x; absolute error at most 1.5e-7 (about a float32 ulp near 1), in a
// dozen instructions
__device__ __forceinline__ float erf_as(float x) {
  const float z = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * z);
  const float q = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  return copysignf(1.0f - q * __expf(-z * z), x);
}

// GELU (x Phi(x), erf form) and its derivative Phi(x) + x phi(x)
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  const float cdf = 0.5f * (1.0f + erf_as(x * 0.70710678118654752f));
  const float pdf = expf(-0.5f * x * x) * 0.39894228040143268f;
  return cdf + x * pdf;
}

constexpr int kGT = 64;   // block tile
constexpr int kGK = 32;   // k step
constexpr int kGPad = 40; // LDS row length (elements)

// AVEC: A has contiguous k and 16-byte aligned rows, staged 8 elements at a time
template <int EPI, bool AVEC>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kGT][kGPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kGT][kGPad];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  const int sr = tid >> 2, sk = (tid & 3) * 8;  // staging: row / column sr, k offset sk
  for (int k0 = 0; k0 < g.K; k0 += kGK) {
    uint16_t av[8], bv[8];
    const int m = m0 + sr, n = n0 + sr;
    if constexpr (AVEC) {
      uint4 a4 = make_uint4(0, 0, 0, 0);
      if (m < g.M && k0 + sk + 8 <= g.K) {
        a4 = *reinterpret_cast<const uint4*>(g.A + (long long)m * g.sam + k0 + sk);
      } else if (m < g.M) {  // the ragged end of k
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (k0 + sk + q < g.K) w[q >> 1] |= (uint32_t)g.A[(long long)m * g.sam + k0 + sk + q] << (16 * (q & 1));
        a4 = make_uint4(w[0], w[1], w[2], w[3]);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + sk + q;
        bv[q] = (n < g.N && k < g.K) ? g.B[(long long)k * g.sbk + (long long)n * g.sbn] : (uint16_t)0;
      }
      __syncthreads();
      *reinterpret_cast<uint4*>(&As[sr][sk]) = a4;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + sk + q;
        av[q] = (m < g.M && k < g.K) ? g.A[(long long)m * g.sam + (long long)k * g.sak] : (uint16_t)0;
        bv[q] = (n < g.N && k < g.K) ? g.B[(long long)k * g.sbk + (long long)n * g.sbn] : (uint16_t)0;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 8; ++q) As[sr][sk + q] = av[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) Bs[sr][sk + q] = bv[q];
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&As[wm * 32 + i * 16 + fr][fk]));
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bs[wn * 32 + j * 16 + fr][fk]));
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
      }
    }
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + q;
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        const long long o = (long long)m * g.N + n;
        float c = acc[i][j][q];
        if constexpr (EPI == kEpiStore) {
          g.C[o] = c;
        } else if constexpr (EPI == kEpiBias) {
          g.C[o] = c + g.bias[n];
        } else if constexpr (EPI == kEpiBiasGelu) {
          c += g.bias[n];
          if (g.Z) g.Z[o] = c;
          g.Cb[o] = f2bf(gelu(c));
        } else {
          const float d = c * gelu_grad(g.aux[o]);
          g.C[o] = d;
          g.Cb[o] = f2bf(d);
        }
      }
}

template <bool AVEC>
static void gemm_v(const GemmArgs& g, int epi, hipStream_t st) {
  const dim3 grid((g.N + kGT - 1) / kGT, (g.M + kGT - 1) / kGT);
  switch (epi) {
    case kEpiStore: hipLaunchKernelGGL((k_gemm<kEpiStore, AVEC>), grid, dim3(256), 0, st, g); break;
    case kEpiBias: hipLaunchKernelGGL((k_gemm<kEpiBias, AVEC>), grid, dim3(256), 0, st, g); break;
    case kEpiBiasGelu: hipLaunchKernelGGL((k_gemm<kEpiBiasGelu, AVEC>), grid, dim3(256), 0, st, g); break;
    default: hipLaunchKernelGGL((k_gemm<kEpiGeluBwd, AVEC>), grid, dim3(256), 0, st, g); break;
  }
}

static void gemm(const GemmArgs& g, int epi, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  const bool avec = g.sak == 1 && (g.sam & 7) == 0 && (reinterpret_cast<uintptr_t>(g.A) & 15) == 0;
  if (avec) gemm_v<true>(g, epi, st);
  else gemm_v<false>(g, epi, st);
}

void launch_gemm(const GemmArgs& g, int epilogue, hipStream_t st) { gemm(g, epilogue, st); }

static GemmArgs gargs(int M, int N, int K, const uint16_t* A, long long sam, long long sak, const uint16_t* B,
                      long long sbk, long long sbn) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.sam = sam;
  g.sak = sak;
  g.B = B;
  g.sbk = sbk;
  g.sbn = sbn;
  return g;
}

// ---------------------------------------------------------------- forward --

static void forward(const MlpWeights& W, const uint16_t* x, int rows, MlpWork& wk, hipStream_t st) {
  // Z1 = X W1 + b1, H1 = bf16(gelu(Z1))
  GemmArgs g = gargs(rows, kHid, kFeat, x, kFeat, 1, W.wb + kOffW1, kHid, 1);
  g.Z = wk.z1;
  g.Cb = wk.h1;
  g.bias = W.w + kOffB1;
  gemm(g, kEpiBiasGelu, st);
  g = gargs(rows, kHid, kHid, wk.h1, kHid, 1, W.wb + kOffW2, kHid, 1);
  g.Z = wk.z2;
  g.Cb = wk.h2;
  g.bias = W.w + kOffB2;
  gemm(g, kEpiBiasGelu, st);
  g = gargs(rows, kOut, kHid, wk.h2, kHid, 1, W.wb + kOffW3, kOut, 1);
  g.C = wk.y;
  g.bias = W.w + kOffB3;
  gemm(g, kEpiBias, st);
}

void mlp_forward(const MlpWeights& W, const uint16_t* x, int rows, MlpWork& wk, hipStream_t st) {
  forward(W, x, rows, wk, st);
}

// --------------------------------------------------------------- backward --

// dY = 2 (y - t) / (3 rows); per-block partial sums of (y - t)^2
__global__ void __launch_bounds__(256) k_loss_grad(const float* y, const float* t, float tscale, int rows, float* dy,
                                                   uint16_t* dyb, float* partial) {
  __shared__ float red[256];
  const int r = blockIdx.x * 256 + threadIdx.x;
  float ss = 0.0f;
  if (r < rows) {
    const float inv = 2.0f / (3.0f * (float)rows);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float e = y[3 * r + k] - t[3 * r + k] * tscale;
      ss += e * e;
      const float d = e * inv;
      dy[3 * r + k] = d;
      dyb[3 * r + k] = f2bf(d);
    }
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_loss_final(const float* partial, int nblocks, int rows, float* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b];
  *loss = (float)(s / (3.0 * rows));
}

// Column sums of a row-major [rows][n] float matrix, in two deterministic
// passes: 256-row chunks, then the chunks.
__global__ void k_colsum_partial(const float* a, int rows, int n, float* part) {
  const int c = threadIdx.x;
  if (c >= n) return;
  const int r0 = blockIdx.x * 256, r1 = min(rows, r0 + 256);
  float s = 0.0f;
  for (int r = r0; r < r1; ++r) s += a[(long long)r * n + c];
  part[(long long)blockIdx.x * n + c] = s;
}

__global__ void k_colsum_final(const float* part, int chunks, int n, float* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float s = 0.0f;
  for (int q = 0; q < chunks; ++q) s += part[(long long)q * n + c];
  out[c] = s;
}

static void colsum(const float* a, int rows, int n, float* scratch, float* out, hipStream_t st) {
  const int chunks = (rows + 255) / 256;
  hipLaunchKernelGGL(k_colsum_partial, dim3(chunks), dim3(n <= 64 ? 64 : 128), 0, st, a, rows, n, scratch);
  hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(128), 0, st, scratch, chunks, n, out);
}

void mlp_backward(const MlpWeights& W, const uint16_t* x, const float* t, int rows, MlpWork& wk, float* loss_out,
                  hipStream_t st) {
  mlp_backward_scaled(W, x, t, 1.0f, rows, wk, loss_out, st);
}

void mlp_backward_scaled(const MlpWeights& W, const uint16_t* x, const float* t, float tscale, int rows, MlpWork& wk,
                         float* loss_out, hipStream_t st) {
  const int nb = (rows + 255) / 256;
  hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, st, wk.y, t, tscale, rows, wk.dy, wk.dyb, wk.partial);
  if (loss_out) hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, wk.partial, nb, rows, loss_out);
  float* col = wk.partial + nb;  // column-sum scratch after the loss partials
  // layer 3: dW3 = H2^T dY, db3 = sum dY, dZ2 = (dY W3^T) * gelu'(Z2)
  GemmArgs g = gargs(kHid, kOut, rows, wk.h2, 1, kHid, wk.dyb, kOut, 1);
  g.C = W.grad + kOffW3;
  gemm(g, kEpiStore, st);
  colsum(wk.dy, rows, kOut, col, W.grad + kOffB3, st);
  g = gargs(rows, kHid, kOut, wk.dyb, kOut, 1, W.wb + kOffW3, 1, kOut);
  g.C = wk.dz2;
  g.Cb = wk.dz2b;
  g.aux = wk.z2;
  gemm(g, kEpiGeluBwd, st);
  // layer 2
  g = gargs(kHid, kHid, rows, wk.h1, 1, kHid, wk.dz2b, kHid, 1);
  g.C = W.grad + kOffW2;
  gemm(g, kEpiStore, st);
  colsum(wk.dz2, rows, kHid, col, W.grad + kOffB2, st);
  g = gargs(rows, kHid, kHid, wk.dz2b, kHid, 1, W.wb + kOffW2, 1, kHid);
  g.C = wk.dz1;
  g.Cb = wk.dz1b;
  g.aux = wk.z1;
  gemm(g, kEpiGeluBwd, st);
  // layer 1
  g = gargs(kFeat, kHid, rows, x, 1, kFeat, wk.dz1b, kHid, 1);
  g.C = W.grad + kOffW1;
  gemm(g, kEpiStore, st);
  colsum(wk.dz1, rows, kHid, col, W.grad + kOffB1, st);
}

// ------------------------------------------------------------------- Adam --

__global__ void k_adam(float* w, uint16_t* wb, float* m, float* v, const float* g, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wb[i] = f2bf(wi);
}

// wt = the transposed bfloat16 weights (from wb, so the values are identical)
__global__ void k_refresh_t(const uint16_t* __restrict__ wb, uint16_t* __restrict__ wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kWT) return;
  uint16_t v;
  if (i < kOffT2) {
    const int n = i / kFeat, k = i % kFeat;
    v = wb[kOffW1 + k * kHid + n];
  } else if (i < kOffT3) {
    const int n = (i - kOffT2) / kHid, k = (i - kOffT2) % kHid;
    v = wb[kOffW2 + k * kHid + n];
  } else {
    const int n = (i - kOffT3) / kHid, k = (i - kOffT3) % kHid;
    v = n < kOut ? wb[kOffW3 + k * kOut + n] : (uint16_t)0;
  }
  wt[i] = v;
}

static void refresh_t(const MlpWeights& W, hipStream_t st) {
  hipLaunchKernelGGL(k_refresh_t, dim3((kWT + 255) / 256), dim3(256), 0, st, W.wb, W.wt);
}

void mlp_adam(const MlpWeights& W, int step, float lr, float b1, float b2, float eps, hipStream_t st) {
  const float c1 = (float)(1.0 - pow((double)b1, step)), c2 = (float)(1.0 - pow((double)b2, step));
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, W.w, W.wb, W.m, W.v, W.grad, kParams, lr,
                     b1, b2, eps, c1, c2);
  refresh_t(W, st);
}

__global__ void k_refresh(const float* w, uint16_t* wb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = f2bf(w[i]);
}

void mlp_refresh_bf16(const MlpWeights& W, hipStream_t st) {
  hipLaunchKernelGGL(k_refresh, dim3((kParams + 255) / 256), dim3(256), 0, st, W.w, W.wb, kParams);
  refresh_t(W, st);
}

// ---------------------------------------------------------------- features --

// Velocity sum of every fluid cell, summed in cell order (one thread per
// cell-offset entry; a scene's last entry bounds its last cell).
__global__ void __launch_bounds__(256) k_cell_vsum(PhysPlan P, ClosurePlan C, int always) {
  if (!always && !C.state[kClNeed]) return;
  const uint32_t g = blockIdx.x * 256 + threadIdx.x;
  if (g >= C.noff) return;
  const int s = find_set(C.oprefix, P.nscenes, g);
  const DScene& S = P.scenes[s];
  if (g - S.obase >= S.g.ncells) return;
  const uint32_t j0 = P.off[g], j1 = P.off[g + 1];
  float vs[3] = {0.0f, 0.0f, 0.0f};
  uint32_t t = j0;
  for (; t + 4 <= j1; t += 4) {  // four particles' loads in flight; the sums stay in cell order
    const uint32_t j = S.pbase + t;
    float w[3][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      w[0][u] = P.svx[j + u];
      w[1][u] = P.svy[j + u];
      w[2][u] = P.svz[j + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      vs[0] += w[0][u];
      vs[1] += w[1][u];
      vs[2] += w[2][u];
    }
  }
  for (; t < j1; ++t) {
    const uint32_t j = S.pbase + t;
    vs[0] += P.svx[j];
    vs[1] += P.svy[j];
    vs[2] += P.svz[j];
  }
  C.cvs[g] = vs[0];
  C.cvs[C.noff + g] = vs[1];
  C.cvs[2 * (size_t)C.noff + g] = vs[2];
}

// One wavefront per agent, agents taken in cell order; lane q is cell q of
// the agent's 4 x 4 x 4 block (x fastest): count / 8 and (mean fluid velocity
// - agent velocity) / 0.5, from the cell offsets and the cell velocity sums.
template <int BD>
__global__ void __launch_bounds__(BD) k_features(PhysPlan P, ClosurePlan C, int always) {
  if (!always && !C.state[kClNeed]) return;
  const uint32_t gi = (blockIdx.x * BD + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (gi >= P.na) return;
  const int s = (int)uniform_u32((uint32_t)find_set(P.aprefix, P.nscenes, gi));
  const DScene& S = P.scenes[s];
  // row a of the features is agent a
  const uint32_t a = S.abase + uniform_u32(P.asid[S.abase + (gi - P.aprefix[s])]);
  const float ya[3] = {P.agx[a], P.agy[a], P.agz[a]};
  const float ua[3] = {P.aux[a], P.auy[a], P.auz[a]};
  const int l[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
  int c[3];
  bool inside = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma clang fp contract(off)
    float t = ya[k] - S.g.mn[k];
    t = t * S.g.inv;
    c[k] = (int)rintf(t) - 2 + l[k];
    inside = inside && c[k] >= 0 && c[k] < S.g.dim[k];
  }
  uint32_t n = 0;
  float vs[3] = {0.0f, 0.0f, 0.0f};
  if (inside) {
    const uint32_t g = S.obase + hash3(S.g, c[0], c[1], c[2]);
    n = P.off[g + 1] - P.off[g];
    vs[0] = C.cvs[g];
    vs[1] = C.cvs[C.noff + g];
    vs[2] = C.cvs[2 * (size_t)C.noff + g];
  }
  uint16_t f[4];
  f[0] = f2bf((float)n / 8.0f);
#pragma unroll
  for (int k = 0; k < 3; ++k) f[k + 1] = n ? f2bf((vs[k] / (float)n - ua[k]) / 0.5f) : (uint16_t)0;
  uint2 packed;
  packed.x = (uint32_t)f[0] | ((uint32_t)f[1] << 16);
  packed.y = (uint32_t)f[2] | ((uint32_t)f[3] << 16);
  *reinterpret_cast<uint2*>(C.feat + (size_t)a * kFeat + 4 * lane) = packed;
  const uint64_t any = __ballot(n > 0);
  if (lane == 0) C.occ[a] = any ? 1u : 0u;
}

void launch_features(const PhysPlan& P, const ClosurePlan& C, bool always, hipStream_t st) {
  if (!P.na) return;
  if (C.noff) hipLaunchKernelGGL(k_cell_vsum, dim3((C.noff + 255) / 256), dim3(256), 0, st, P, C, always ? 1 : 0);
  hipLaunchKernelGGL(k_features<256>, dim3((P.na + 3) / 4), dim3(256), 0, st, P, C, always ? 1 : 0);
}

// ------------------------------------------------------- fused inference --

// One wave per kInferTiles 16-row tiles of agents: the three layers in
// registers and a per-wave LDS tile, on the same v_mfma_f32_16x16x32_bf16
// sequence as k_gemm (operand k order, k steps of 32 in ascending order, the
// same epilogues), so fhat is bit-identical to mlp_forward followed by the
// scaling.  Each weight fragment loaded is used for every row tile of the
// wave.  (Four tiles per wave took 336 registers, one wave per SIMD, and ran
// slower: 79 us against 61 us at 65,536 agents, where the exact GELU
// epilogues are most of the vector work.)  A lane's A fragment is row (lane % 16) of a tile, k
// 8 (lane / 16) .. + 7 of the step; its B fragment the same k of column
// (lane % 16), read from the transposed weights as 16 contiguous bytes; the
// result holds rows 4 (lane / 16) + q, column lane % 16.
constexpr int kInferWaves = 4;
constexpr int kInferTiles = 1;                   // 16-row tiles per wave
constexpr int kInferRows = 16 * kInferTiles;     // agents per wave
constexpr int kHPad = kHid + 8;  // LDS row of a hidden tile (16-byte aligned rows)

// LDS written by some lanes of a wave and read by others: order them
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bf16x8 ld_frag(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

__global__ void __launch_bounds__(kInferWaves * kWave) k_closure_infer(const uint16_t* __restrict__ X, uint32_t rows,
                                                                     const uint16_t* __restrict__ wt,
                                                                     const float* __restrict__ w, ClosurePlan C,
                                                                     float scale) {
  constexpr int T = kInferTiles, NJ = kHid / 16;
  __shared__ __attribute__((aligned(16))) uint16_t sH[kInferWaves][kInferRows][kHPad];
  if (!C.state[kClNeed]) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint32_t r0 = (blockIdx.x * kInferWaves + wave) * (uint32_t)kInferRows;
  if (r0 >= rows) return;  // whole wave; no block-wide barriers below
  const int fr = lane & 15, fk = (lane >> 4) * 8, qr = (lane >> 4) * 4;
  uint16_t(*H)[kHPad] = sH[wave];
  const bf16x8 zero = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));

  // layer 1: H1 = bf16(gelu(X W1 + b1))
  f32x4 acc[NJ][T];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int t = 0; t < T; ++t) acc[j][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < kFeat; k0 += 32) {
    bf16x8 a[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const uint32_t ra = r0 + (uint32_t)(16 * t + fr);
      a[t] = ra < rows ? ld_frag(X + (size_t)ra * kFeat + k0 + fk) : zero;
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const bf16x8 bj = ld_frag(wt + kOffT1 + (j * 16 + fr) * kFeat + k0 + fk);
#pragma unroll
      for (int t = 0; t < T; ++t) acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], bj, acc[j][t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const float bias = w[kOffB1 + j * 16 + fr];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) H[16 * t + qr + q][j * 16 + fr] = f2bf(gelu(acc[j][t][q] + bias));
  }
  wave_lds_sync();

  // layer 2: H2 = bf16(gelu(H1 W2 + b2)), written over H1 once it has been read
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int t = 0; t < T; ++t) acc[j][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < kHid; k0 += 32) {
    bf16x8 a[T];
#pragma unroll
    for (int t = 0; t < T; ++t) a[t] = ld_frag(&H[16 * t + fr][k0 + fk]);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const bf16x8 bj = ld_frag(wt + kOffT2 + (j * 16 + fr) * kHid + k0 + fk);
#pragma unroll
      for (int t = 0; t < T; ++t) acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], bj, acc[j][t], 0, 0, 0);
    }
  }
  wave_lds_sync();  // every lane has read H1
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const float bias = w[kOffB2 + j * 16 + fr];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) H[16 * t + qr + q][j * 16 + fr] = f2bf(gelu(acc[j][t][q] + bias));
  }
  wave_lds_sync();

  // layer 3: y = H2 W3 + b3 (columns 3..15 of the tile are zero weights)
  f32x4 y[T];
#pragma unroll
  for (int t = 0; t < T; ++t) y[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k0 = 0; k0 < kHid; k0 += 32) {
    const bf16x8 b3 = ld_frag(wt + kOffT3 + fr * kHid + k0 + fk);
#pragma unroll
    for (int t = 0; t < T; ++t)
      y[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld_frag(&H[16 * t + fr][k0 + fk]), b3, y[t], 0, 0, 0);
  }
  if (fr >= kOut) return;
  const float bias = w[kOffB3 + fr];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t a = r0 + (uint32_t)(16 * t + qr + q);
      if (a < rows) C.fhat[3 * (size_t)a + fr] = C.occ[a] ? (y[t][q] + bias) * scale : 0.0f;
    }
}

void launch_closure_infer(const MlpWeights& W, const ClosurePlan& C, uint32_t na, hipStream_t st) {
  if (!na) return;
  const uint32_t per_block = kInferWaves * (uint32_t)kInferRows;
  hipLaunchKernelGGL(k_closure_infer, dim3((na + per_block - 1) / per_block), dim3(kInferWaves * kWave), 0, st,
                     C.feat, na, W.wt, W.w, C, W.scale);
}

// -------------------------------------------------------------- controller --

// Decides, from the step counter and the current mode, whether this step uses
// the surrogate and whether it is a check step (every check_every steps, both
// forces are computed and compared).
__global__ void k_closure_begin(ClosurePlan C) {
  if (threadIdx.x || blockIdx.x) return;
  const uint32_t step = C.state[kClStep];
  const uint32_t check = (C.check_every > 0 && step % (uint32_t)C.check_every == 0) ? 1u : 0u;
  const uint32_t use = (C.state[kClMode] && !check) ? 1u : 0u;
  C.state[kClCheck] = check;
  C.state[kClUse] = use;
  C.state[kClNeed] = (use || check) ? 1u : 0u;
}

void launch_closure_begin(const ClosurePlan& C, hipStream_t st) {
  hipLaunchKernelGGL(k_closure_begin, dim3(1), dim3(64), 0, st, C);
}

// At a check step: rel_rms = sqrt(sum |fhat - F|^2 / sum |F|^2) over all
// agents (fixed-order reduction), and the surrogate is used for the following
// steps only if rel_rms <= max_rel_rms.  Counts steps by the force used.
__global__ void __launch_bounds__(256) k_closure_end(ClosurePlan C, uint32_t na) {
  __shared__ double se[256], sf[256];
  const uint32_t check = C.state[kClCheck];
  double e = 0.0, f = 0.0;
  if (check)
    for (uint32_t a = threadIdx.x; a < na; a += 256) {
      e += C.err[2 * a];
      f += C.err[2 * a + 1];
    }
  se[threadIdx.x] = e;
  sf[threadIdx.x] = f;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      se[threadIdx.x] += se[threadIdx.x + s];
      sf[threadIdx.x] += sf[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x) return;
  if (check) {
    const double rel = sf[0] > 0.0 ? sqrt(se[0] / sf[0]) : 0.0;
    C.relrms[0] = (float)rel;
    const uint32_t ok = (float)rel <= C.max_rel_rms ? 1u : 0u;
    C.state[kClMode] = ok;
    C.state[kClChecks] += 1;
    if (!ok) C.state[kClFallbacks] += 1;
  }
  if (C.state[kClUse]) C.state[kClSurrogateSteps] += 1;
  else C.state[kClExactSteps] += 1;
  C.state[kClStep] += 1;
}

void launch_closure_end(const ClosurePlan& C, uint32_t na, hipStream_t st) {
  hipLaunchKernelGGL(k_closure_end, dim3(1), dim3(256), 0, st, C, na);
}


}  // namespace sph
