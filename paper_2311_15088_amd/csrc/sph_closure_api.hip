// sph_closure_api.hip -- C ABI of the learned coupling closure: create, train
// on (features, exact force) pairs with the project's own forward / backward /
// Adam kernels, predict, attach to a context, statistics.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "sph.h"
#include "sph_api_internal.hpp"
#include "sph_mlp.hpp"

using namespace sph;

static std::string g_closure_error;

struct sph_closure {
  std::string err;
  hipStream_t stream = nullptr;
  MlpWeights W{};
  char* arena = nullptr;
  // training / prediction work buffers, grown on demand
  MlpWork wk{};
  char* work = nullptr;
  int work_rows = 0;
  int32_t adam_t = 0;  // Adam steps taken on the current moments
};

static sph_status cfail(sph_closure* cl, sph_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (cl) cl->err = buf;
  else g_closure_error = buf;
  return st;
}

#define CLCHK(call)                                                                   \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return cfail(cl, SPH_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static size_t al(size_t b) { return (b + 255) / 256 * 256; }

// Work buffers for `rows` rows of a forward and backward pass.
static sph_status ensure_work(sph_closure* cl, int rows) {
  if (rows <= cl->work_rows) return SPH_OK;
  if (cl->work) CLCHK(hipFree(cl->work));
  cl->work = nullptr;
  const size_t r = (size_t)rows;
  const size_t nb = (r + 255) / 256;
  size_t sizes[] = {4 * r * kHid, 4 * r * kHid, 4 * r * 4,      2 * r * kHid, 2 * r * kHid, 4 * r * 4,
                    4 * r * kHid, 4 * r * kHid, 2 * r * 4,       2 * r * kHid, 2 * r * kHid, 4 * (nb + nb * kHid + 64)};
  size_t tot = 0;
  for (size_t s : sizes) tot += al(s);
  CLCHK(hipMalloc((void**)&cl->work, tot));
  char* p = cl->work;
  void** dst[] = {(void**)&cl->wk.z1, (void**)&cl->wk.z2, (void**)&cl->wk.y, (void**)&cl->wk.h1, (void**)&cl->wk.h2,
                  (void**)&cl->wk.dy, (void**)&cl->wk.dz2, (void**)&cl->wk.dz1, (void**)&cl->wk.dyb,
                  (void**)&cl->wk.dz2b, (void**)&cl->wk.dz1b, (void**)&cl->wk.partial};
  for (int k = 0; k < 12; ++k) {
    *dst[k] = p;
    p += al(sizes[k]);
  }
  cl->wk.rows = rows;
  cl->work_rows = rows;
  return SPH_OK;
}

// ---------------------------------------------------------------- helpers --

__global__ void k_gather_rows(const uint16_t* __restrict__ x, const float* __restrict__ f, const uint32_t* idx,
                              int rows, uint16_t* __restrict__ xb, float* __restrict__ fb) {
  const int r = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (r >= rows) return;
  const size_t src = idx[r];
  // 256 bf16 = 64 lanes x 4 values
  reinterpret_cast<uint2*>(xb + (size_t)r * kFeat)[lane] = reinterpret_cast<const uint2*>(x + src * kFeat)[lane];
  if (lane < 3) fb[3 * r + lane] = f[3 * src + lane];
}

// sum over rows of |y scale - f|^2 and |f|^2 (per block, fixed order)
__global__ void k_val_err(const float* y, const float* f, float scale, int rows, double* out) {
  __shared__ double se[256], sf[256];
  double e = 0.0, g = 0.0;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < rows; r += gridDim.x * 256)
    for (int k = 0; k < 3; ++k) {
      const double d = (double)y[3 * r + k] * scale - (double)f[3 * r + k];
      e += d * d;
      g += (double)f[3 * r + k] * f[3 * r + k];
    }
  se[threadIdx.x] = e;
  sf[threadIdx.x] = g;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      se[threadIdx.x] += se[threadIdx.x + s];
      sf[threadIdx.x] += sf[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = se[0];
    out[2 * blockIdx.x + 1] = sf[0];
  }
}

__global__ void k_scale_out(const float* y, float scale, int n, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * n) out[i] = y[i] * scale;
}

// SplitMix64 (Steele, Lea & Flood 2014) for the seeded shuffles.
static uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static void shuffle(std::vector<uint32_t>& v, uint64_t seed) {
  uint64_t s = seed;
  for (size_t i = v.size(); i > 1; --i) {
    const size_t j = (size_t)(splitmix(s) % i);
    std::swap(v[i - 1], v[j]);
  }
}

// -------------------------------------------------------------------- ABI --

extern "C" {

sph_status sph_closure_create(const float* weights, float force_scale, void* hip_stream, sph_closure** out) {
  if (!out) return cfail(nullptr, SPH_EINVAL, "NULL out");
  *out = nullptr;
  if (!(force_scale > 0.0f)) return cfail(nullptr, SPH_EINVAL, "force_scale must be positive");
  sph_closure* cl = new sph_closure();
  cl->stream = (hipStream_t)hip_stream;
  const size_t tot = al(4 * kParams) * 5 + al(2 * kParams) + al(2 * (size_t)kWT);
  hipError_t e = hipMalloc((void**)&cl->arena, tot);
  if (e != hipSuccess) {
    delete cl;
    return cfail(nullptr, SPH_ENOMEM, "hipMalloc: %s", hipGetErrorString(e));
  }
  char* p = cl->arena;
  cl->W.w = (float*)p;
  p += al(4 * kParams);
  cl->W.m = (float*)p;
  p += al(4 * kParams);
  cl->W.v = (float*)p;
  p += al(4 * kParams);
  cl->W.grad = (float*)p;
  p += al(4 * kParams);
  p += al(4 * kParams);  // spare
  cl->W.wb = (uint16_t*)p;
  p += al(2 * kParams);
  cl->W.wt = (uint16_t*)p;
  cl->W.scale = force_scale;
  hipStream_t st = cl->stream;
  e = hipMemsetAsync(cl->arena, 0, tot, st);
  if (e == hipSuccess && weights) e = hipMemcpyAsync(cl->W.w, weights, 4 * (size_t)kParams, hipMemcpyDefault, st);
  if (e == hipSuccess) {
    mlp_refresh_bf16(cl->W, st);
    e = hipStreamSynchronize(st);
  }
  if (e != hipSuccess) {
    (void)hipFree(cl->arena);
    delete cl;
    return cfail(nullptr, SPH_EHIP, "closure upload: %s", hipGetErrorString(e));
  }
  *out = cl;
  return SPH_OK;
}

void sph_closure_destroy(sph_closure* cl) {
  if (!cl) return;
  (void)hipStreamSynchronize(cl->stream);
  if (cl->work) (void)hipFree(cl->work);
  if (cl->arena) (void)hipFree(cl->arena);
  delete cl;
}

const char* sph_closure_last_error(const sph_closure* cl) { return cl ? cl->err.c_str() : g_closure_error.c_str(); }

sph_status sph_closure_weights(sph_closure* cl, int32_t write, float* weights, float* force_scale) {
  if (!cl) return cfail(nullptr, SPH_EINVAL, "NULL closure");
  if (write) {
    if (force_scale) {
      if (!(*force_scale > 0.0f)) return cfail(cl, SPH_EINVAL, "force_scale must be positive");
      cl->W.scale = *force_scale;
    }
    if (weights) {
      CLCHK(hipMemcpyAsync(cl->W.w, weights, 4 * (size_t)kParams, hipMemcpyDefault, cl->stream));
      mlp_refresh_bf16(cl->W, cl->stream);
    }
  } else {
    if (force_scale) *force_scale = cl->W.scale;
    if (weights) CLCHK(hipMemcpyAsync(weights, cl->W.w, 4 * (size_t)kParams, hipMemcpyDefault, cl->stream));
  }
  CLCHK(hipStreamSynchronize(cl->stream));
  return SPH_OK;
}

sph_status sph_closure_predict(sph_closure* cl, const uint16_t* features, int64_t n, float* forces) {
  if (!cl || (n > 0 && (!features || !forces)) || n < 0 || n >= (1ll << 31))
    return cfail(cl, SPH_EINVAL, "invalid arguments");
  if (n == 0) return SPH_OK;
  sph_status s = ensure_work(cl, (int)n);
  if (s != SPH_OK) return s;
  mlp_forward(cl->W, features, (int)n, cl->wk, cl->stream);
  hipLaunchKernelGGL(k_scale_out, dim3((3 * n + 255) / 256), dim3(256), 0, cl->stream, cl->wk.y, cl->W.scale, (int)n,
                     forces);
  CLCHK(hipGetLastError());
  return SPH_OK;
}

// ------------------------------------------------- allocation-free predict --
// sph_closure_predict_static runs the same forward pass as sph_closure_predict
// with its activations in a fixed device array instead of the closure's work
// buffers (which grow with hipMalloc): the two hidden layers' bfloat16
// activations and the unscaled outputs of up to kStaticRows rows.
constexpr int kStaticRows = 65536;  // one config-4 agent set per call
constexpr size_t kStaticH = (size_t)kStaticRows * kHid * 2;  // one bf16 hidden layer
constexpr size_t kStaticBytes = 2 * kStaticH + (size_t)kStaticRows * kOut * 4;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
static char* g_scratch_ptr[kMaxDevices];
static std::once_flag g_scratch_once[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current (the array's name is a host-side stand-in
// and must never be passed to a kernel).
static char* scratch_ptr(int dev, hipError_t* err) {
  std::call_once(g_scratch_once[dev], [dev]() {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? (char*)p : nullptr;
  });
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}

sph_status sph_closure_predict_static(sph_closure* cl, const uint16_t* features, int64_t n, float* forces) {
  if (!cl || (n > 0 && (!features || !forces)) || n < 0) return cfail(cl, SPH_EINVAL, "invalid arguments");
  if (n > kStaticRows)
    return cfail(cl, SPH_ECAPACITY, "%lld rows exceed the static scratch of %d rows; split the call",
                 (long long)n, kStaticRows);
  if (n == 0) return SPH_OK;
  int dev = 0;
  CLCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return cfail(cl, SPH_EINVAL, "device %d out of range", dev);
  hipError_t e = hipSuccess;
  char* base = scratch_ptr(dev, &e);
  if (!base) return cfail(cl, SPH_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  MlpWork wk{};
  wk.rows = (int)n;
  wk.h1 = (uint16_t*)base;
  wk.h2 = (uint16_t*)(base + kStaticH);
  wk.y = (float*)(base + 2 * kStaticH);
  // z1, z2 (kept for a backward pass) are not written: the GEMM epilogue skips a null Z
  mlp_forward(cl->W, features, (int)n, wk, cl->stream);
  hipLaunchKernelGGL(k_scale_out, dim3((3 * n + 255) / 256), dim3(256), 0, cl->stream, wk.y, cl->W.scale, (int)n,
                     forces);
  CLCHK(hipGetLastError());
  return SPH_OK;
}

sph_status sph_closure_gradient(sph_closure* cl, const uint16_t* features, const float* forces, int64_t n,
                                float* grad, float* loss) {
  if (!cl || !features || !forces || !grad || n <= 0 || n >= (1ll << 31))
    return cfail(cl, SPH_EINVAL, "invalid arguments");
  sph_status s = ensure_work(cl, (int)n);
  if (s != SPH_OK) return s;
  mlp_forward(cl->W, features, (int)n, cl->wk, cl->stream);
  float* dloss = cl->wk.partial + ((n + 255) / 256) * (1 + kHid) + 8;  // a float of the scratch tail
  mlp_backward_scaled(cl->W, features, forces, 1.0f / cl->W.scale, (int)n, cl->wk, dloss, cl->stream);
  CLCHK(hipMemcpyAsync(grad, cl->W.grad, 4 * (size_t)kParams, hipMemcpyDefault, cl->stream));
  if (loss) CLCHK(hipMemcpyAsync(loss, dloss, 4, hipMemcpyDefault, cl->stream));
  CLCHK(hipStreamSynchronize(cl->stream));
  return SPH_OK;
}

sph_status sph_closure_adam_step(sph_closure* cl, const float* grad, int32_t t, float lr, float beta1, float beta2,
                                 float eps) {
  if (!cl || !grad || t < 1) return cfail(cl, SPH_EINVAL, "invalid arguments");
  CLCHK(hipMemcpyAsync(cl->W.grad, grad, 4 * (size_t)kParams, hipMemcpyDefault, cl->stream));
  mlp_adam(cl->W, t, lr, beta1, beta2, eps, cl->stream);
  CLCHK(hipStreamSynchronize(cl->stream));
  cl->adam_t = t;
  return SPH_OK;
}

// Checkpoint of the whole closure state: weights, Adam moments, force scale
// and the Adam step count, one float32 buffer (layout in sph.h).
sph_status sph_closure_io(sph_closure* cl, int32_t dir, float* buf, int64_t bytes) {
  if (!cl || !buf || (dir != 0 && dir != 1)) return cfail(cl, SPH_EINVAL, "invalid arguments");
  const size_t P = (size_t)kParams;
  if (bytes < (int64_t)(4 * SPH_CLOSURE_STATE_FLOATS))
    return cfail(cl, SPH_EINVAL, "buffer holds %lld bytes, the state needs %lld", (long long)bytes,
                 (long long)(4 * SPH_CLOSURE_STATE_FLOATS));
  float* dev[3] = {cl->W.w, cl->W.m, cl->W.v};
  if (dir == 0) {
    for (int k = 0; k < 3; ++k) CLCHK(hipMemcpyAsync(buf + k * P, dev[k], 4 * P, hipMemcpyDefault, cl->stream));
    CLCHK(hipStreamSynchronize(cl->stream));
    float tail[2] = {cl->W.scale, (float)cl->adam_t};
    CLCHK(hipMemcpy(buf + 3 * P, tail, sizeof tail, hipMemcpyDefault));
  } else {
    float tail[2];
    CLCHK(hipMemcpy(tail, buf + 3 * P, sizeof tail, hipMemcpyDefault));
    if (!(tail[0] > 0.0f) || !(tail[1] >= 0.0f) || tail[1] > 16777216.0f || tail[1] != floorf(tail[1]))
      return cfail(cl, SPH_EINVAL, "invalid force scale or step count in the state");
    for (int k = 0; k < 3; ++k) CLCHK(hipMemcpyAsync(dev[k], buf + k * P, 4 * P, hipMemcpyDefault, cl->stream));
    mlp_refresh_bf16(cl->W, cl->stream);
    CLCHK(hipStreamSynchronize(cl->stream));
    cl->W.scale = tail[0];
    cl->adam_t = (int32_t)tail[1];
  }
  return SPH_OK;
}

sph_status sph_closure_train(sph_closure* cl, const uint16_t* features, const float* forces, int64_t n,
                             const sph_train_params* tp, sph_train_report* rep) {
  if (!cl || !features || !forces || !tp || n < 2 || n >= (1ll << 31))
    return cfail(cl, SPH_EINVAL, "invalid arguments");
  if (tp->epochs < 0 || tp->batch <= 0 || !(tp->lr > 0.0f) || !(tp->val_fraction >= 0.0f && tp->val_fraction < 1.0f))
    return cfail(cl, SPH_EINVAL, "invalid training parameters");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = cl->stream;
  const int B = tp->batch;
  sph_status s = ensure_work(cl, B);
  if (s != SPH_OK) return s;
  // split: a seeded permutation; the last val_fraction of it is held out
  std::vector<uint32_t> perm((size_t)n);
  std::iota(perm.begin(), perm.end(), 0u);
  shuffle(perm, (uint64_t)tp->seed * 0x100000001ull + 17);
  const int64_t n_val = (int64_t)floor((double)n * tp->val_fraction);
  const int64_t n_tr = n - n_val;
  // force scale: root mean square of the training force components
  std::vector<float> hf((size_t)n * 3);
  CLCHK(hipMemcpy(hf.data(), forces, 12 * (size_t)n, hipMemcpyDefault));
  double ss = 0.0;
  for (int64_t i = 0; i < n_tr; ++i)
    for (int k = 0; k < 3; ++k) ss += (double)hf[3 * (size_t)perm[i] + k] * hf[3 * (size_t)perm[i] + k];
  const float scale = ss > 0.0 ? (float)sqrt(ss / (3.0 * (double)n_tr)) : 1.0f;
  cl->W.scale = scale;
  uint32_t* didx = nullptr;
  uint16_t* xb = nullptr;
  float* fb = nullptr;
  float* losses = nullptr;
  double* verr = nullptr;
  const int64_t nbatch = (n_tr + B - 1) / B;
  const int vblocks = 64;
  CLCHK(hipMalloc((void**)&didx, 4 * (size_t)n));
  CLCHK(hipMalloc((void**)&xb, 2 * (size_t)B * kFeat));
  CLCHK(hipMalloc((void**)&fb, 12 * (size_t)B));
  CLCHK(hipMalloc((void**)&losses, 4 * (size_t)std::max<int64_t>(nbatch, 1)));
  CLCHK(hipMalloc((void**)&verr, 16 * vblocks));
  CLCHK(hipMemsetAsync(cl->W.m, 0, 4 * (size_t)kParams, st));
  CLCHK(hipMemsetAsync(cl->W.v, 0, 4 * (size_t)kParams, st));
  mlp_refresh_bf16(cl->W, st);
  std::vector<uint32_t> tr(perm.begin(), perm.begin() + n_tr);
  int step = 0;
  double last_loss = 0.0;
  for (int ep = 0; ep < tp->epochs; ++ep) {
    shuffle(tr, (uint64_t)tp->seed * 0x9E3779B9ull + 101 + ep);
    CLCHK(hipMemcpyAsync(didx, tr.data(), 4 * (size_t)n_tr, hipMemcpyHostToDevice, st));
    for (int64_t b = 0; b < nbatch; ++b) {
      const int rows = (int)std::min<int64_t>(B, n_tr - b * B);
      hipLaunchKernelGGL(k_gather_rows, dim3((rows + 3) / 4), dim3(256), 0, st, features, forces, didx + b * B, rows,
                         xb, fb);
      mlp_forward(cl->W, xb, rows, cl->wk, st);
      mlp_backward_scaled(cl->W, xb, fb, 1.0f / scale, rows, cl->wk, losses + b, st);
      mlp_adam(cl->W, ++step, tp->lr, tp->beta1, tp->beta2, tp->eps, st);
    }
    std::vector<float> hl((size_t)nbatch);
    CLCHK(hipMemcpyAsync(hl.data(), losses, 4 * (size_t)nbatch, hipMemcpyDeviceToHost, st));
    CLCHK(hipStreamSynchronize(st));
    double sl = 0.0;
    for (float l : hl) sl += l;
    last_loss = nbatch ? sl / (double)nbatch : 0.0;
  }
  CLCHK(hipGetLastError());
  // validation: relative RMS error of the predicted forces on the held-out part
  double se = 0.0, sf = 0.0;
  if (n_val > 0) {
    std::vector<uint32_t> vi(perm.begin() + n_tr, perm.end());
    CLCHK(hipMemcpyAsync(didx, vi.data(), 4 * (size_t)n_val, hipMemcpyHostToDevice, st));
    std::vector<double> h(2 * vblocks);
    for (int64_t b = 0; b < n_val; b += B) {
      const int rows = (int)std::min<int64_t>(B, n_val - b);
      hipLaunchKernelGGL(k_gather_rows, dim3((rows + 3) / 4), dim3(256), 0, st, features, forces, didx + b, rows, xb,
                         fb);
      mlp_forward(cl->W, xb, rows, cl->wk, st);
      hipLaunchKernelGGL(k_val_err, dim3(vblocks), dim3(256), 0, st, cl->wk.y, fb, scale, rows, verr);
      CLCHK(hipMemcpyAsync(h.data(), verr, 16 * vblocks, hipMemcpyDeviceToHost, st));
      CLCHK(hipStreamSynchronize(st));
      for (int q = 0; q < vblocks; ++q) {
        se += h[2 * q];
        sf += h[2 * q + 1];
      }
    }
  }
  CLCHK(hipStreamSynchronize(st));
  (void)hipFree(didx);
  (void)hipFree(xb);
  (void)hipFree(fb);
  (void)hipFree(losses);
  (void)hipFree(verr);
  cl->adam_t = step;
  if (rep) {
    rep->train_loss = (float)last_loss;
    rep->val_rel_rms = sf > 0.0 ? (float)sqrt(se / sf) : 0.0f;
    rep->force_scale = scale;
    rep->steps = step;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return SPH_OK;
}

// ----------------------------------------------------- context integration --

sph_status sph_closure_attach(sph_ctx* ctx, sph_closure* cl, int32_t check_every, float max_rel_rms) {
  if (!ctx) return cfail(nullptr, SPH_EINVAL, "NULL context");
  if (cl && (check_every < 1 || !(max_rel_rms >= 0.0f))) return cfail(cl, SPH_EINVAL, "invalid controller settings");
  if (ctx->graph_exec) {
    (void)hipGraphExecDestroy(ctx->graph_exec);
    (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_steps = 0;
  }
  ctx->closure = cl;
  if (!cl) {
    ctx->phys.cl_fhat = nullptr;
    ctx->phys.cl_state = nullptr;
    ctx->phys.cl_err = nullptr;
    return SPH_OK;
  }
  sph_status s = sph_ctx_closure_buffers(ctx);
  if (s != SPH_OK) return s;
  s = ensure_work(cl, std::max<int>(1, (int)ctx->A));
  if (s != SPH_OK) return s;
  ctx->cplan.check_every = check_every;
  ctx->cplan.max_rel_rms = max_rel_rms;
  hipError_t e = hipMemsetAsync(ctx->cplan.state, 0, 4 * kClWords, ctx->stream);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->cplan.relrms, 0, 4, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return cfail(cl, SPH_EHIP, "attach: %s", hipGetErrorString(e));
  ctx->phys.cl_fhat = ctx->cplan.fhat;
  ctx->phys.cl_state = ctx->cplan.state;
  ctx->phys.cl_err = ctx->cplan.err;
  if (ctx->fused) {
    // the closure runs between phases of a step: back to per-phase launches
    // of the context's kernel variant, with that variant's tiles
    const sph_status t = set_tiling(ctx, ctx->phys.tx, ctx->phys.variant, false);
    if (t != SPH_OK) return t;
    ctx->fused = false;
    ctx->phys.item_max = (uint32_t)fluid_item_max(0, ctx->phys.variant);
  }
  return SPH_OK;
}

sph_status sph_closure_stats_get(sph_ctx* ctx, sph_closure_stats* out) {
  if (!ctx || !out) return cfail(nullptr, SPH_EINVAL, "NULL argument");
  memset(out, 0, sizeof *out);
  if (!ctx->closure) return SPH_OK;
  uint32_t st[kClWords];
  float rel = 0.0f;
  hipError_t e = hipMemcpyAsync(st, ctx->cplan.state, sizeof st, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&rel, ctx->cplan.relrms, 4, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return cfail(nullptr, SPH_EHIP, "stats: %s", hipGetErrorString(e));
  out->mode = (int32_t)st[kClMode];
  out->last_rel_rms = rel;
  out->checks = st[kClChecks];
  out->fallbacks = st[kClFallbacks];
  out->surrogate_steps = st[kClSurrogateSteps];
  out->exact_steps = st[kClExactSteps];
  return SPH_OK;
}

}  // extern "C"

// Closure kernels of one step, between the density and the agent phases.
void sph_ctx_closure_phase(sph_ctx* ctx, hipStream_t st) {
  if (ctx->closure) {
    sph_closure* cl = ctx->closure;
    launch_closure_begin(ctx->cplan, st);
    launch_features(ctx->phys, ctx->cplan, false, st);
    launch_closure_infer(cl->W, ctx->cplan, ctx->A, st);
  } else if (ctx->features) {
    launch_features(ctx->phys, ctx->cplan, true, st);
  }
}

void sph_ctx_closure_end(sph_ctx* ctx, hipStream_t st) {
  if (ctx->closure) launch_closure_end(ctx->cplan, ctx->A, st);
}
