// The learned stopping index and regularisation parameter: a 16-64-64-2 GELU
// network on the first Golub-Kahan steps (Algorithm 4) and the LSQR residuals
// (Algorithm 6), with its inference, gradient and Adam kernels.
//
// Parameters: one flat FP32 master vector [W1 (64x16), b1, W2 (64x64), b2,
// W3 (2x64), b3] (weights row-major (output, input)), and the bfloat16 copy
// (round to nearest even) that every forward and backward pass reads; all
// arithmetic accumulates in FP32.  Per-sample work is one thread per sample
// with the 5378 parameters staged in LDS; weight gradients are summed over
// chunks of 32 samples per workgroup, then over the chunks in a fixed order
// (deterministic).
#include <cmath>
#include <new>
#include <vector>

#include "internal.h"

namespace dctk {

constexpr int kNIn = 16, kNH = 64, kNOut = 2;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kNH * kNIn, kOffW2 = kOffB1 + kNH, kOffB2 = kOffW2 + kNH * kNH,
              kOffW3 = kOffB2 + kNH, kOffB3 = kOffW3 + kNOut * kNH, kNParams = kOffB3 + kNOut;
static_assert(kNParams == DCTK_MLP_PARAMS, "parameter count");
constexpr int kCache = 2 * kNH;      // per sample: h1, h2 (pre-activations)
constexpr int kChunk = 32;           // samples per weight-gradient workgroup
constexpr int kFeatSteps = 8;

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__device__ inline void stage_params(const bf16_t* Pb, float* sW) {
  for (int i = threadIdx.x; i < kNParams; i += blockDim.x) sW[i] = bf16_to_float(Pb[i]);
  __syncthreads();
}

// one sample: hidden pre-activations (optionally stored) and the two outputs
__device__ inline void mlp_sample(const float* sW, const float* x, float* h1o, float* h2o, float* out) {
  float a1[kNH];
#pragma unroll 8
  for (int o = 0; o < kNH; ++o) {
    float acc = sW[kOffB1 + o];
#pragma unroll
    for (int i = 0; i < kNIn; ++i) acc += sW[kOffW1 + o * kNIn + i] * x[i];
    if (h1o) h1o[o] = acc;
    a1[o] = gelu_f(acc);
  }
  float o0 = sW[kOffB3], o1 = sW[kOffB3 + 1];
  for (int o = 0; o < kNH; ++o) {
    float acc = sW[kOffB2 + o];
#pragma unroll
    for (int i = 0; i < kNH; ++i) acc += sW[kOffW2 + o * kNH + i] * a1[i];
    if (h2o) h2o[o] = acc;
    const float a2 = gelu_f(acc);
    o0 += sW[kOffW3 + o] * a2;
    o1 += sW[kOffW3 + kNH + o] * a2;
  }
  out[0] = o0;
  out[1] = o1;
}

__global__ __launch_bounds__(256) void k_mlp_forward(int B, const float* X, const bf16_t* Pb, float* out,
                                                     float* cache) {
  __shared__ float sW[kNParams];
  stage_params(Pb, sW);
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float x[kNIn];
#pragma unroll
  for (int i = 0; i < kNIn; ++i) x[i] = X[(int64_t)b * kNIn + i];
  float y[2];
  float* c = cache ? cache + (int64_t)b * kCache : nullptr;
  mlp_sample(sW, x, c, c ? c + kNH : nullptr, y);
  out[(int64_t)b * 2] = y[0];
  out[(int64_t)b * 2 + 1] = y[1];
}

// dout = w (out - T) / B and per-block partials of (1/2B) sum w (out - T)^2
__global__ __launch_bounds__(256) void k_mlp_loss(int B, const float* out, const float* T, float w0, float w1,
                                                  float* dout, double* loss_part) {
  __shared__ double sh[kShCtl];
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (b < B) {
    const float r0 = out[(int64_t)b * 2] - T[(int64_t)b * 2];
    const float r1 = out[(int64_t)b * 2 + 1] - T[(int64_t)b * 2 + 1];
    dout[(int64_t)b * 2] = w0 * r0 / (float)B;
    dout[(int64_t)b * 2 + 1] = w1 * r1 / (float)B;
    l = 0.5 * ((double)w0 * r0 * r0 + (double)w1 * r1 * r1) / (double)B;
  }
  const double t = block_sum_all(l, sh);
  if (threadIdx.x == 0) loss_part[blockIdx.x] = t;
}

// per-sample back-propagated errors of the two hidden layers: delta = [d1, d2]
__global__ __launch_bounds__(256) void k_mlp_delta(int B, const bf16_t* Pb, const float* cache, const float* dout,
                                                   float* delta) {
  __shared__ float sW[kNParams];
  stage_params(Pb, sW);
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float* h = cache + (int64_t)b * kCache;
  const float d30 = dout[(int64_t)b * 2], d31 = dout[(int64_t)b * 2 + 1];
  float d2[kNH];
#pragma unroll 8
  for (int i = 0; i < kNH; ++i) {
    const float da2 = sW[kOffW3 + i] * d30 + sW[kOffW3 + kNH + i] * d31;
    d2[i] = da2 * gelu_grad_f(h[kNH + i]);
  }
  float* dl = delta + (int64_t)b * kCache;
  for (int i = 0; i < kNH; ++i) {
    float da1 = 0.0f;
#pragma unroll
    for (int o = 0; o < kNH; ++o) da1 += sW[kOffW2 + o * kNH + i] * d2[o];
    dl[i] = da1 * gelu_grad_f(h[i]);
  }
#pragma unroll 8
  for (int i = 0; i < kNH; ++i) dl[kNH + i] = d2[i];
}

// partial weight gradients of one chunk of samples: gpart[chunk][param]
__global__ __launch_bounds__(256) void k_mlp_wgrad(int B, const float* X, const float* cache, const float* delta,
                                                   const float* dout, float* gpart) {
  __shared__ float sx[kChunk][kNIn];
  __shared__ float sa1[kChunk][kNH], sa2[kChunk][kNH], sd1[kChunk][kNH], sd2[kChunk][kNH];
  __shared__ float sd3[kChunk][kNOut];
  const int b0 = blockIdx.x * kChunk;
  for (int i = threadIdx.x; i < kChunk * kNH; i += blockDim.x) {
    const int s = i / kNH, j = i % kNH, b = b0 + s;
    const bool ok = b < B;
    sa1[s][j] = ok ? gelu_f(cache[(int64_t)b * kCache + j]) : 0.0f;
    sa2[s][j] = ok ? gelu_f(cache[(int64_t)b * kCache + kNH + j]) : 0.0f;
    sd1[s][j] = ok ? delta[(int64_t)b * kCache + j] : 0.0f;
    sd2[s][j] = ok ? delta[(int64_t)b * kCache + kNH + j] : 0.0f;
  }
  for (int i = threadIdx.x; i < kChunk * kNIn; i += blockDim.x) {
    const int s = i / kNIn, j = i % kNIn, b = b0 + s;
    sx[s][j] = b < B ? X[(int64_t)b * kNIn + j] : 0.0f;
  }
  for (int i = threadIdx.x; i < kChunk * kNOut; i += blockDim.x) {
    const int s = i / kNOut, j = i % kNOut, b = b0 + s;
    sd3[s][j] = b < B ? dout[(int64_t)b * kNOut + j] : 0.0f;
  }
  __syncthreads();
  float* g = gpart + (int64_t)blockIdx.x * kNParams;
  for (int q = threadIdx.x; q < kNParams; q += blockDim.x) {
    float acc = 0.0f;
    if (q < kOffB1) {
      const int o = q / kNIn, i = q % kNIn;
      for (int s = 0; s < kChunk; ++s) acc += sd1[s][o] * sx[s][i];
    } else if (q < kOffW2) {
      const int o = q - kOffB1;
      for (int s = 0; s < kChunk; ++s) acc += sd1[s][o];
    } else if (q < kOffB2) {
      const int o = (q - kOffW2) / kNH, i = (q - kOffW2) % kNH;
      for (int s = 0; s < kChunk; ++s) acc += sd2[s][o] * sa1[s][i];
    } else if (q < kOffW3) {
      const int o = q - kOffB2;
      for (int s = 0; s < kChunk; ++s) acc += sd2[s][o];
    } else if (q < kOffB3) {
      const int o = (q - kOffW3) / kNH, i = (q - kOffW3) % kNH;
      for (int s = 0; s < kChunk; ++s) acc += sd3[s][o] * sa2[s][i];
    } else {
      const int o = q - kOffB3;
      for (int s = 0; s < kChunk; ++s) acc += sd3[s][o];
    }
    g[q] = acc;
  }
}

// grad[q] = sum over chunks in order
__global__ __launch_bounds__(256) void k_mlp_reduce(int nchunk, const float* gpart, float* grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kNParams) return;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += (double)gpart[(int64_t)c * kNParams + q];
  grad[q] = (float)acc;
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* P, const float* g, float* m, float* v, float bc1, float bc2,
                                                  float lr, bf16_t* Pb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kNParams) return;
  const float gq = g[q];
  const float mq = 0.9f * m[q] + 0.1f * gq;
  const float vq = 0.999f * v[q] + 0.001f * gq * gq;
  m[q] = mq;
  v[q] = vq;
  const float p = P[q] - lr * (mq / bc1) / (sqrtf(vq / bc2) + 1e-8f);
  P[q] = p;
  Pb[q] = float_to_bf16(p);
}

__global__ void k_mlp_round(const float* P, bf16_t* Pb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < kNParams) Pb[q] = float_to_bf16(P[q]);
}

// the 16 features of a GKB workspace state (after >= 8 steps)
__device__ inline bool state_features(const KState* st, float* f) {
  if (ld_state(&st->steps) < kFeatSteps) return false;
  const double b1 = st->beta[0];
  for (int j = 0; j < kFeatSteps; ++j) {
    f[j] = (float)log(st->alpha[j] / st->beta[j]);
    f[kFeatSteps + j] = (float)log(fabs(st->phibar[j + 1]) / b1);
  }
  for (int j = 0; j < kNIn; ++j)
    if (!isfinite(f[j])) return false;
  return true;
}

__global__ void k_mlp_features(const KState* st, float* out) {
  if (threadIdx.x != 0) return;
  float f[kNIn];
  const bool ok = state_features(st, f);
  for (int j = 0; j < kNIn; ++j) out[j] = ok ? f[j] : __builtin_nanf("");
}

// features -> network -> pred = {t_lambda, t_k, lambda, k (as float), valid}
__global__ __launch_bounds__(64) void k_mlp_predict(const KState* st, const bf16_t* Pb, float mu, float sigma,
                                                    float kscale, float koffset, int kmin, int kmax, float* pred) {
  __shared__ float sW[kNParams];
  __shared__ float f[kNIn];
  __shared__ int ok;
  stage_params(Pb, sW);
  if (threadIdx.x == 0) ok = state_features(st, f) ? 1 : 0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  float y[2] = {0.0f, 0.0f};
  if (ok) mlp_sample(sW, f, nullptr, nullptr, y);
  const float lam = expf(y[0] * sigma + mu);
  float kf = rintf(y[1] * kscale + koffset);
  kf = fminf(fmaxf(kf, (float)kmin), (float)kmax);
  pred[0] = y[0];
  pred[1] = y[1];
  pred[2] = lam;
  pred[3] = kf;
  pred[4] = (ok && isfinite(lam) && lam > 0.0f && isfinite(y[1])) ? 1.0f : 0.0f;
}

// Device-side learned stop for a workspace (plain or grouped launch, one
// 64-thread workgroup per instance): after step 8, sets the step limit and
// the proposed lambda in the state; no limit when the features are unusable.
struct StopArgs {
  int gx, gy, gz;
  int kmin, kmax;
  KState* st;
  const bf16_t* Pb;
  float mu, sigma, kscale, koffset;
};

__device__ __forceinline__ void k_mlp_stop_body(const StopArgs& a, const VBlock vb, const bool grouped) {
  __shared__ float sW[kNParams];
  __shared__ float f[kNIn];
  __shared__ int ok;
  stage_params(a.Pb, sW);
  KState* st = a.st;
  if (threadIdx.x == 0) ok = (ld_state(&st->stop_step) < 0 && state_features(st, f)) ? 1 : 0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (!ok) {
    st->k_limit = 0;
    st->pred_lambda = 0.0;
    return;
  }
  float y[2];
  mlp_sample(sW, f, nullptr, nullptr, y);
  const float lam = expf(y[0] * a.sigma + a.mu);
  float kf = rintf(y[1] * a.kscale + a.koffset);
  kf = fminf(fmaxf(kf, (float)a.kmin), (float)a.kmax);
  const bool valid = isfinite(lam) && lam > 0.0f && isfinite(kf);
  st->k_limit = valid ? (int)kf : 0;
  st->pred_lambda = valid ? (double)lam : 0.0;
}

template <bool GROUPED>
__global__ __launch_bounds__(64) void k_mlp_stop(StopArgs a_, const StopArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_mlp_stop_body(a_, hw_block(), false);
  } else {
    VBlock vb;
    const StopArgs g = group_args(grp, bmap, vb);
    k_mlp_stop_body(g, vb, true);
  }
}

}  // namespace dctk

using namespace dctk;

struct dctk_mlp_s {
  dctk_ctx ctx;
  float* P;        // FP32 master parameters
  bf16_t* Pb;      // bfloat16 parameters used by every pass
  float* m;        // Adam moments
  float* v;
  float* grad;
  float* pred;     // 8 floats: last prediction
  int t;           // Adam step count
  double mu, sigma, kscale, koffset;
  // scratch for a batch of up to cap samples
  int cap;
  float* out;
  float* dout;
  float* cache;
  float* delta;
  float* gpart;
  double* loss_part;
};

static void mlp_free_scratch(dctk_mlp m) {
  (void)hipFree(m->out);
  (void)hipFree(m->dout);
  (void)hipFree(m->cache);
  (void)hipFree(m->delta);
  (void)hipFree(m->gpart);
  (void)hipFree(m->loss_part);
  m->out = m->dout = m->cache = m->delta = m->gpart = nullptr;
  m->loss_part = nullptr;
  m->cap = 0;
}

static hipError_t mlp_reserve(dctk_mlp m, int B) {
  if (B <= m->cap) return hipSuccess;
  mlp_free_scratch(m);
  const int nchunk = (B + kChunk - 1) / kChunk, nblk = (B + 255) / 256;
  hipError_t e = hipMalloc((void**)&m->out, sizeof(float) * 2 * B);
  if (e == hipSuccess) e = hipMalloc((void**)&m->dout, sizeof(float) * 2 * B);
  if (e == hipSuccess) e = hipMalloc((void**)&m->cache, sizeof(float) * kCache * (size_t)B);
  if (e == hipSuccess) e = hipMalloc((void**)&m->delta, sizeof(float) * kCache * (size_t)B);
  if (e == hipSuccess) e = hipMalloc((void**)&m->gpart, sizeof(float) * kNParams * (size_t)nchunk);
  if (e == hipSuccess) e = hipMalloc((void**)&m->loss_part, sizeof(double) * nblk);
  if (e != hipSuccess) {
    mlp_free_scratch(m);
    return e;
  }
  m->cap = B;
  return hipSuccess;
}

// splitmix64 (Steele, Lea and Flood 2014): the deterministic initial weights
static uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// gradient of sum_b <dout_b, out_b> into m->grad (forward with cache first)
static hipError_t mlp_grad(dctk_ctx ctx, dctk_mlp m, int B, const float* X, const float* dout) {
  const int nblk = (B + 255) / 256, nchunk = (B + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_mlp_forward, dim3(nblk), dim3(256), 0, ctx->stream, B, X, m->Pb, m->out, m->cache);
  hipLaunchKernelGGL(k_mlp_delta, dim3(nblk), dim3(256), 0, ctx->stream, B, m->Pb, m->cache, dout, m->delta);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(nchunk), dim3(256), 0, ctx->stream, B, X, m->cache, m->delta, dout, m->gpart);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParams + 255) / 256), dim3(256), 0, ctx->stream, nchunk, m->gpart,
                     m->grad);
  return hipGetLastError();
}

namespace dctk {
hipError_t launch_mlp_stop(dctk_ctx ctx, dctk_mlp m, KState* st, int kmin, int kmax) {
  StopArgs a{};
  a.kmin = kmin;
  a.kmax = kmax;
  a.st = st;
  a.Pb = m->Pb;
  a.mu = (float)m->mu;
  a.sigma = (float)m->sigma;
  a.kscale = (float)m->kscale;
  a.koffset = (float)m->koffset;
  return launch_kernel(ctx, ctx->stream, k_mlp_stop<false>, k_mlp_stop<true>, dim3(1), 64, 0, a);
}

hipError_t mlp_predict(dctk_ctx ctx, dctk_mlp m, const KState* st, int kmin, int kmax, float* host_pred) {
  hipLaunchKernelGGL(k_mlp_predict, dim3(1), dim3(64), 0, ctx->stream, st, m->Pb, (float)m->mu, (float)m->sigma,
                     (float)m->kscale, (float)m->koffset, kmin, kmax, m->pred);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(host_pred, m->pred, sizeof(float) * 5, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e;
}
}  // namespace dctk

extern "C" {

int dctk_mlp_create(dctk_ctx ctx, uint64_t seed, dctk_mlp* out) {
  if (!ctx || !out) return DCTK_EINVAL;
  *out = nullptr;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  dctk_mlp m = new (std::nothrow) dctk_mlp_s();
  if (!m) return DCTK_ENOMEM;
  m->ctx = ctx;
  m->mu = 0.0;
  m->sigma = 1.0;
  m->kscale = 40.0;
  m->koffset = 0.0;
  hipError_t e = hipMalloc((void**)&m->P, sizeof(float) * kNParams);
  if (e == hipSuccess) e = hipMalloc((void**)&m->Pb, sizeof(bf16_t) * kNParams);
  if (e == hipSuccess) e = hipMalloc((void**)&m->m, sizeof(float) * kNParams);
  if (e == hipSuccess) e = hipMalloc((void**)&m->v, sizeof(float) * kNParams);
  if (e == hipSuccess) e = hipMalloc((void**)&m->grad, sizeof(float) * kNParams);
  if (e == hipSuccess) e = hipMalloc((void**)&m->pred, sizeof(float) * 8);
  // Xavier-uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)); zero biases
  std::vector<float> h(kNParams, 0.0f);
  uint64_t s = seed;
  auto fill = [&](int off, int fo, int fi) {
    const double a = std::sqrt(6.0 / (double)(fo + fi));
    for (int i = 0; i < fo * fi; ++i) {
      const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
      h[off + i] = (float)((2.0 * u - 1.0) * a);
    }
  };
  fill(kOffW1, kNH, kNIn);
  fill(kOffW2, kNH, kNH);
  fill(kOffW3, kNOut, kNH);
  if (e != hipSuccess) {
    dctk_mlp_destroy(m);
    return hip_fail(ctx, e);
  }
  const int r = dctk_mlp_set_params(ctx, m, h.data());
  if (r != DCTK_OK) {
    dctk_mlp_destroy(m);
    return r;
  }
  *out = m;
  return DCTK_OK;
}

int dctk_mlp_destroy(dctk_mlp m) {
  if (!m) return DCTK_EINVAL;
  (void)hipSetDevice(m->ctx->device);
  (void)hipStreamSynchronize(m->ctx->stream);
  mlp_free_scratch(m);
  (void)hipFree(m->P);
  (void)hipFree(m->Pb);
  (void)hipFree(m->m);
  (void)hipFree(m->v);
  (void)hipFree(m->grad);
  (void)hipFree(m->pred);
  delete m;
  return DCTK_OK;
}

int dctk_mlp_set_params(dctk_ctx ctx, dctk_mlp m, const float* host) {
  if (!ctx || !m || !host || m->ctx != ctx) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  DCTK_HIP(ctx, hipMemcpyAsync(m->P, host, sizeof(float) * kNParams, hipMemcpyHostToDevice, ctx->stream));
  DCTK_HIP(ctx, hipMemsetAsync(m->m, 0, sizeof(float) * kNParams, ctx->stream));
  DCTK_HIP(ctx, hipMemsetAsync(m->v, 0, sizeof(float) * kNParams, ctx->stream));
  hipLaunchKernelGGL(k_mlp_round, dim3((kNParams + 255) / 256), dim3(256), 0, ctx->stream, m->P, m->Pb);
  DCTK_HIP(ctx, hipGetLastError());
  DCTK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  m->t = 0;
  return DCTK_OK;
}

int dctk_mlp_get_params(dctk_ctx ctx, dctk_mlp m, float* host, uint16_t* host_bf16) {
  if (!ctx || !m || m->ctx != ctx) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  if (host) DCTK_HIP(ctx, hipMemcpyAsync(host, m->P, sizeof(float) * kNParams, hipMemcpyDeviceToHost, ctx->stream));
  if (host_bf16)
    DCTK_HIP(ctx, hipMemcpyAsync(host_bf16, m->Pb, sizeof(bf16_t) * kNParams, hipMemcpyDeviceToHost, ctx->stream));
  DCTK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return DCTK_OK;
}

int dctk_mlp_set_scaling(dctk_mlp m, double mu, double sigma, double k_scale, double k_offset) {
  if (!m || !std::isfinite(mu) || !(sigma > 0.0) || !std::isfinite(sigma) || !(k_scale > 0.0) ||
      !std::isfinite(k_scale) || !std::isfinite(k_offset))
    return DCTK_EINVAL;
  m->mu = mu;
  m->sigma = sigma;
  m->kscale = k_scale;
  m->koffset = k_offset;
  return DCTK_OK;
}

int dctk_mlp_forward(dctk_ctx ctx, dctk_mlp m, int B, const float* X, float* out) {
  if (!ctx || !m || m->ctx != ctx || !X || !out || B < 1 || B > DCTK_MLP_MAX_BATCH) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_mlp_forward, dim3((B + 255) / 256), dim3(256), 0, ctx->stream, B, X, m->Pb, out,
                     (float*)nullptr);
  DCTK_HIP(ctx, hipGetLastError());
  return DCTK_OK;
}

int dctk_mlp_gradient(dctk_ctx ctx, dctk_mlp m, int B, const float* X, const float* dout, float* grad) {
  if (!ctx || !m || m->ctx != ctx || !X || !dout || !grad || B < 1 || B > DCTK_MLP_MAX_BATCH) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  DCTK_HIP(ctx, mlp_reserve(m, B));
  DCTK_HIP(ctx, mlp_grad(ctx, m, B, X, dout));
  DCTK_HIP(ctx, hipMemcpyAsync(grad, m->grad, sizeof(float) * kNParams, hipMemcpyDeviceToDevice, ctx->stream));
  return DCTK_OK;
}

int dctk_mlp_train_step(dctk_ctx ctx, dctk_mlp m, int B, const float* X, const float* T, double w_lambda,
                        double w_k, double lr, double* loss) {
  if (!ctx || !m || m->ctx != ctx || !X || !T || B < 1 || B > DCTK_MLP_MAX_BATCH) return DCTK_EINVAL;
  if (!(w_lambda >= 0.0) || !(w_k >= 0.0) || !(lr > 0.0) || !std::isfinite(lr)) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  DCTK_HIP(ctx, mlp_reserve(m, B));
  const int nblk = (B + 255) / 256;
  hipLaunchKernelGGL(k_mlp_forward, dim3(nblk), dim3(256), 0, ctx->stream, B, X, m->Pb, m->out, m->cache);
  hipLaunchKernelGGL(k_mlp_loss, dim3(nblk), dim3(256), 0, ctx->stream, B, m->out, T, (float)w_lambda, (float)w_k,
                     m->dout, m->loss_part);
  DCTK_HIP(ctx, hipGetLastError());
  DCTK_HIP(ctx, mlp_grad(ctx, m, B, X, m->dout));
  m->t += 1;
  const float bc1 = (float)(1.0 - std::pow(0.9, m->t)), bc2 = (float)(1.0 - std::pow(0.999, m->t));
  hipLaunchKernelGGL(k_mlp_adam, dim3((kNParams + 255) / 256), dim3(256), 0, ctx->stream, m->P, m->grad, m->m, m->v,
                     bc1, bc2, (float)lr, m->Pb);
  DCTK_HIP(ctx, hipGetLastError());
  if (loss) {
    std::vector<double> lp(nblk);
    DCTK_HIP(ctx, hipMemcpyAsync(lp.data(), m->loss_part, sizeof(double) * nblk, hipMemcpyDeviceToHost, ctx->stream));
    DCTK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (double x : lp) s += x;
    *loss = s;
  }
  return DCTK_OK;
}

int dctk_mlp_features(dctk_ctx ctx, dctk_krylov ws, float* out16) {
  if (!ctx || !ws || !out16 || ws->kind != DCTK_KRYLOV_GKB) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_mlp_features, dim3(1), dim3(64), 0, ctx->stream, (const KState*)ws->st, out16);
  DCTK_HIP(ctx, hipGetLastError());
  return DCTK_OK;
}

}  // extern "C"
