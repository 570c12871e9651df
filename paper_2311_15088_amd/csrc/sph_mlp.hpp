// sph_mlp.hpp -- the learned coupling closure: per-agent features and a small
// MLP (256 -> 128 -> 128 -> 3, GELU) on bfloat16 MFMA with float32
// accumulation, its backward pass and Adam (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sph_internal.hpp"

namespace sph {

constexpr int kFeat = 256, kHid = 128, kOut = 3;
constexpr int kW1 = kFeat * kHid, kW2 = kHid * kHid, kW3 = kHid * kOut;
// flat parameter order: W1 [256][128], b1, W2 [128][128], b2, W3 [128][3], b3
constexpr int kOffW1 = 0, kOffB1 = kW1, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kW2, kOffW3 = kOffB2 + kHid,
              kOffB3 = kOffW3 + kW3, kParams = kOffB3 + kOut;  // 49,795

enum GemmEpilogue { kEpiStore = 0, kEpiBias = 1, kEpiBiasGelu = 2, kEpiGeluBwd = 3 };

// C[M][N] = A(M x K) B(K x N), bfloat16 operands with element strides
// (A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn]), float32
// accumulation.  Outputs are row-major [M][N].  Epilogues:
//   kEpiStore     c = acc                              -> C
//   kEpiBias      c = acc + bias[n]                    -> C
//   kEpiBiasGelu  z = acc + bias[n] -> Z (optional); Cb = bf16(gelu(z))
//   kEpiGeluBwd   d = acc * gelu'(aux[m][n]) -> C (float), Cb = bf16(d)
struct GemmArgs {
  int M, N, K;
  const uint16_t* A;
  long long sam, sak;
  const uint16_t* B;
  long long sbk, sbn;
  float* C;
  uint16_t* Cb;
  float* Z;
  const float* bias;
  const float* aux;
};

void launch_gemm(const GemmArgs& g, int epilogue, hipStream_t st);

// Closure weights and optimiser state on the device.
// Transposed bfloat16 weights for the fused inference kernel: W1^T [128][256],
// W2^T [128][128], W3^T padded to [16][128] (rows 3..15 zero).
constexpr int kOffT1 = 0, kOffT2 = kOffT1 + kHid * kFeat, kOffT3 = kOffT2 + kHid * kHid, kWT = kOffT3 + 16 * kHid;

struct MlpWeights {
  float* w;       // [kParams] float32 master weights
  uint16_t* wb;   // [kParams] bfloat16 copy used by the products
  uint16_t* wt;   // [kWT] transposed bfloat16 copy (fused inference), refreshed with wb
  float* m;       // Adam moments
  float* v;
  float* grad;    // [kParams]
  float scale;    // force scale: the network predicts F / scale
};

// Work buffers for a forward (and backward) pass over up to rows rows.
struct MlpWork {
  int rows;
  float *z1, *z2, *y;          // [rows][128], [rows][128], [rows][3]
  uint16_t *h1, *h2;           // bf16 activations
  float *dy, *dz2, *dz1;       // float32 gradients
  uint16_t *dyb, *dz2b, *dz1b; // bf16 gradients
  float* partial;              // [blocks] loss partial sums
};

void mlp_forward(const MlpWeights& W, const uint16_t* x, int rows, MlpWork& wk, hipStream_t st);
// Gradient of the mean squared error of (y - t) over rows x 3 into W.grad;
// loss_out (device, may be null) receives the loss.
void mlp_backward(const MlpWeights& W, const uint16_t* x, const float* t, int rows, MlpWork& wk, float* loss_out,
                  hipStream_t st);
void mlp_backward_scaled(const MlpWeights& W, const uint16_t* x, const float* t, float tscale, int rows, MlpWork& wk,
                         float* loss_out, hipStream_t st);
void mlp_adam(const MlpWeights& W, int step, float lr, float b1, float b2, float eps, hipStream_t st);
void mlp_refresh_bf16(const MlpWeights& W, hipStream_t st);

// Per-step closure kernels of a context (see sph_api.hip).
struct ClosurePlan {
  uint16_t* feat;     // [na][256]
  float* fhat;        // [na][3] surrogate forces
  uint32_t* occ;      // [na] any fluid in the agent's block
  float* err;         // [na][2] |fhat - F|^2, |F|^2 at check steps
  uint32_t* state;    // kCl* words (sph_internal.hpp)
  float* relrms;      // [1] last check
  float* cvs;         // [3][noff] velocity sum of every fluid cell, indexed like the cell offsets
  uint32_t* oprefix;  // [nscenes + 1] first cell-offset entry of every scene (last = noff)
  uint32_t noff;      // cell-offset entries of all scenes (cells + one per scene)
  int check_every;
  float max_rel_rms;
};

void launch_features(const PhysPlan& P, const ClosurePlan& C, bool always, hipStream_t st);
void launch_closure_begin(const ClosurePlan& C, hipStream_t st);
// The closure's per-step inference in one kernel (gated on the controller):
// fhat = occ ? MLP(features) * scale : 0, bit-identical to mlp_forward.
void launch_closure_infer(const MlpWeights& W, const ClosurePlan& C, uint32_t na, hipStream_t st);
void launch_closure_end(const ClosurePlan& C, uint32_t na, hipStream_t st);

}  // namespace sph
