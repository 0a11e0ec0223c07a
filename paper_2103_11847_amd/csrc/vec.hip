// Global inner products, Frobenius norms, axpys and basis combinations of the
// Krylov methods (Sec. 2.2 inner product; Algorithms 2, 4 and 6; the
// combination V (*) y of eq. ev1), as streaming kernels.
//
// Reductions are deterministic: every block reduces its share in FP64 with
// wavefront shuffles and writes one partial per value; the last block to
// arrive (ticket counter) sums the partials in block order and applies the
// Krylov "action" (store beta_{j+1}, test for breakdown, advance the LSQR
// scalars, ...) so the scalars never leave the device.  The ticket is
// returned to zero by that block, so no memset is needed between uses.
#include <cfloat>
#include <cmath>

#include "internal.h"

namespace dctk {

static constexpr double kEps = DBL_EPSILON;
static constexpr double kBreak = 64.0;

template <typename T> struct V4;
template <> struct V4<float> {
  __device__ static void ld(const float* p, double* v) {
    float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  __device__ static void st(float* p, const double* v) {
    *reinterpret_cast<float4*>(p) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  }
};
template <> struct V4<double> {
  __device__ static void ld(const double* p, double* v) {
    double2 a = *reinterpret_cast<const double2*>(p);
    double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
  __device__ static void st(double* p, const double* v) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
  }
};

// load/store 4 consecutive elements starting at e (vectorised when all 4 exist and vec)
template <typename T>
__device__ inline void ld4(const T* base, int64_t e, int64_t n, bool vec, double* v) {
  if (vec && e + 4 <= n) {
    V4<T>::ld(base + e, v);
  } else {
    for (int i = 0; i < 4; ++i) v[i] = (e + i < n) ? (double)base[e + i] : 0.0;
  }
}
template <typename T>
__device__ inline void st4(T* base, int64_t e, int64_t n, bool vec, const double* v) {
  if (vec && e + 4 <= n) {
    V4<T>::st(base + e, v);
  } else {
    for (int i = 0; i < 4; ++i)
      if (e + i < n) base[e + i] = (T)v[i];
  }
}

// ---- Krylov actions applied by the last block --------------------------------
__device__ void apply_action(int act, double sum, double* dst, KState* st, int j) {
  const double ss = sqrt(sum);
  const bool finite = isfinite(sum);
  switch (act) {
    case ACT_STORE:
      if (dst) dst[0] = ss;
      break;
    case ACT_GKB_BETA1:
      st->beta[0] = ss;
      st->beta0 = ss;
      st->scale = ss;
      st->phibar = ss;
      st->steps = 0;
      if (!finite) { st->status = DCTK_ENONFINITE; st->stop_step = 0; st->stop_kind = STOP_BETA; }
      else if (ss == 0.0) { st->status = DCTK_BREAKDOWN; st->stop_step = 0; st->stop_kind = STOP_BETA; }
      break;
    case ACT_GKB_ALPHA1:
      st->alpha[0] = ss;
      st->rhobar = ss;
      st->scale = fmax(st->scale, ss);
      if (!finite) { st->status = DCTK_ENONFINITE; st->stop_step = 0; st->stop_kind = STOP_ALPHA; }
      else if (ss <= kBreak * kEps * st->scale) { st->status = DCTK_BREAKDOWN; st->stop_step = 0; st->stop_kind = STOP_ALPHA; }
      break;
    case ACT_GKB_BETA:
      st->beta[j] = ss;
      st->scale = fmax(st->scale, ss);
      st->steps = j;
      if (!finite) { st->status = DCTK_ENONFINITE; st->stop_step = j; st->stop_kind = STOP_BETA; }
      else if (ss <= kBreak * kEps * st->scale) { st->status = DCTK_BREAKDOWN; st->stop_step = j; st->stop_kind = STOP_BETA; }
      break;
    case ACT_GKB_ALPHA:
      st->alpha[j] = ss;
      st->scale = fmax(st->scale, ss);
      st->steps = j;
      if (!finite) { st->status = DCTK_ENONFINITE; st->stop_step = j; st->stop_kind = STOP_ALPHA; }
      else if (ss <= kBreak * kEps * st->scale) { st->status = DCTK_BREAKDOWN; st->stop_step = j; st->stop_kind = STOP_ALPHA; }
      break;
    case ACT_ARN_BETA:
      st->beta0 = ss;
      st->steps = 0;
      if (!finite) { st->status = DCTK_ENONFINITE; st->halt = 1; }
      else if (ss == 0.0) { st->halt = 1; }
      break;
    case ACT_ARN_H: {
      st->H[j * kMaxK + (j - 1)] = ss;
      double sc = st->scale;
      for (int i = 0; i <= j; ++i) sc = fmax(sc, fabs(st->H[i * kMaxK + (j - 1)]));
      st->scale = sc;
      st->steps = j;
      if (!finite) { st->status = DCTK_ENONFINITE; st->stop_step = j; st->stop_kind = STOP_BETA; st->halt = 1; }
      else if (ss <= kBreak * kEps * sc) { st->status = DCTK_BREAKDOWN; st->stop_step = j; st->stop_kind = STOP_BETA; }
      break;
    }
    case ACT_GMRES_RES:
      st->resnorm = ss;
      st->cycles += 1;
      st->total_steps += st->steps;
      if (!finite) { st->status = DCTK_ENONFINITE; st->halt = 1; }
      else if (ss < st->tol) { st->converged = 1; st->halt = 1; }
      break;
    case ACT_DOT_STORE:
      if (dst) dst[0] = sum;
      break;
    default:
      break;
  }
}

// Last-block protocol: returns true in the block that must finish the reduction.
__device__ inline bool arrive_last(unsigned* ticket) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = atomicAdd(ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

__device__ inline void reset_ticket(unsigned* ticket) {
  if (threadIdx.x == 0) atomicExch(ticket, 0u);
}

// out = x + c*y, optional reduction of out . z (z == nullptr: out . out).
// `out` may be nullptr (reduce only).  act < 0: no reduction.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_axpy_red(int64_t n, T* out, const T* x,
                                                       const T* y, const double* cptr, double csign,
                                                       double cconst, const T* z, int act, double* dst,
                                                       KState* st, int j, double* partials, unsigned* ticket,
                                                       bool vec, Gate g) {
  if (!gate_open(g)) return;
  __shared__ double sh[kThreads / 64];
  const double c = cptr ? csign * cptr[0] : cconst;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < n; e += stride) {
    double xv[4], yv[4], o[4];
    ld4(x, e, n, vec, xv);
    if (y) {
      ld4(y, e, n, vec, yv);
      for (int i = 0; i < 4; ++i) o[i] = xv[i] + c * yv[i];
    } else {
      for (int i = 0; i < 4; ++i) o[i] = xv[i];
    }
    if (out) {
      st4(out, e, n, vec, o);
      // use the stored (rounded) values so the norm describes the vector in memory
      for (int i = 0; i < 4; ++i) o[i] = (double)(T)o[i];
    }
    if (act >= 0) {
      if (z) {
        double zv[4];
        ld4(z, e, n, vec, zv);
        for (int i = 0; i < 4; ++i) acc += o[i] * zv[i];
      } else {
        for (int i = 0; i < 4; ++i) acc += o[i] * o[i];
      }
    }
  }
  if (act < 0) return;
  double bs = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = bs;
  if (!arrive_last(ticket)) return;
  double v = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) v += ((volatile double*)partials)[b];
  double total = block_sum(v, sh);
  if (threadIdx.x == 0) apply_action(act, total, dst, st, j);
  reset_ticket(ticket);
}

// out = in / den[0]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale(int64_t n, T* out, const T* in, const double* den,
                                                    bool vec, Gate g) {
  if (!gate_open(g)) return;
  const double s = 1.0 / den[0];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < n; e += stride) {
    double v[4];
    ld4(in, e, n, vec, v);
    for (int i = 0; i < 4; ++i) v[i] *= s;
    st4(out, e, n, vec, v);
  }
}

// coef_i = <basis_i, w>, i < nb.  Partials laid out [value][block].
template <typename T>
__global__ __launch_bounds__(kThreads) void k_multidot(int64_t n, const T* basis, int64_t bstride, int nb,
                                                       const T* w, double* dst, int dst_stride,
                                                       int accumulate, double* coef_copy, double* partials,
                                                       unsigned* ticket, bool vec, Gate g) {
  if (!gate_open(g)) return;
  __shared__ double sh[kThreads / 64];
  __shared__ double blk[kRedVals];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int i0 = 0; i0 < nb; i0 += 8) {
    double acc[8];
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < n; e += stride) {
      double wv[4];
      ld4(w, e, n, vec, wv);
      for (int u = 0; u < 8 && i0 + u < nb; ++u) {
        double bv[4];
        ld4(basis + (int64_t)(i0 + u) * bstride, e, n, vec, bv);
        acc[u] += bv[0] * wv[0] + bv[1] * wv[1] + bv[2] * wv[2] + bv[3] * wv[3];
      }
    }
    for (int u = 0; u < 8 && i0 + u < nb; ++u) {
      double bs = block_sum(acc[u], sh);
      if (threadIdx.x == 0) blk[i0 + u] = bs;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) partials[(int64_t)i * gridDim.x + blockIdx.x] = blk[i];
  if (!arrive_last(ticket)) return;
  // one wave per value: fixed order over blocks
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = wid; i < nb; i += (int)(blockDim.x >> 6)) {
    double v = 0.0;
    for (int b = lane; b < (int)gridDim.x; b += 64) v += ((volatile double*)partials)[(int64_t)i * gridDim.x + b];
    v = wave_sum(v);
    if (lane == 0) {
      if (accumulate) dst[i * dst_stride] += v;
      else dst[i * dst_stride] = v;
      if (coef_copy) coef_copy[i] = v;
    }
  }
  reset_ticket(ticket);
}

// w -= sum_i coef[i*cstride] basis_i
template <typename T>
__global__ __launch_bounds__(kThreads) void k_subtract(int64_t n, T* w, const T* basis, int64_t bstride,
                                                       int nb, const double* coef, int cstride, bool vec, Gate g) {
  if (!gate_open(g)) return;
  __shared__ double sc[kRedVals];
  for (int i = threadIdx.x; i < nb; i += blockDim.x) sc[i] = coef[i * cstride];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < n; e += stride) {
    double wv[4];
    ld4(w, e, n, vec, wv);
    for (int i = 0; i < nb; ++i) {
      double bv[4];
      ld4(basis + (int64_t)i * bstride, e, n, vec, bv);
      for (int u = 0; u < 4; ++u) wv[u] -= sc[i] * bv[u];
    }
    st4(w, e, n, vec, wv);
  }
}

// out = x0 + sum_{i < nb} y[i] basis_i   (nb from *nptr when given)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_combine(int64_t n, T* out, const T* x0, const T* basis,
                                                      int64_t bstride, int nb, const int* nptr, const double* y,
                                                      bool vec, Gate g) {
  if (!gate_open(g)) return;
  __shared__ double sy[kRedVals];
  int cnt = nptr ? nptr[0] : nb;
  if (cnt > nb) cnt = nb;
  if (cnt < 0) cnt = 0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) sy[i] = y[i];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < n; e += stride) {
    double o[4] = {0.0, 0.0, 0.0, 0.0};
    if (x0) ld4(x0, e, n, vec, o);
    for (int i = 0; i < cnt; ++i) {
      double bv[4];
      ld4(basis + (int64_t)i * bstride, e, n, vec, bv);
      for (int u = 0; u < 4; ++u) o[u] += sy[i] * bv[u];
    }
    st4(out, e, n, vec, o);
  }
}

// Algorithm 6 steps (c)-(e) and (g) for step j: one thread.
__global__ void k_lsqr_scalars(KState* st, int j) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int ss = st->stop_step;
  if (ss >= 0 && ss < j) return;
  const bool beta_break = (ss == j && st->stop_kind == STOP_BETA);
  const double bnext = st->beta[j];
  const double anext = beta_break ? 0.0 : st->alpha[j];
  const double rhobar = st->rhobar, phibar = st->phibar;
  const double rho = sqrt(rhobar * rhobar + bnext * bnext);
  const double c = rhobar / rho, s = bnext / rho;
  const double theta = s * anext;
  st->rhobar = c * anext;
  const double phi = c * phibar;
  st->phibar = -s * phibar;
  st->cx = phi / rho;
  st->cw = theta / rho;
  if (ss < 0 && fabs(st->phibar) < st->tol) {
    st->stop_step = j;
    st->stop_kind = STOP_CONV;
    st->converged = 1;
  }
}

// Algorithm 6 step (f) for step j, with V_{j+1} = V~ / alpha_{j+1} done in place.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lsqr_update(int64_t n, T* X, T* W, T* Vn, KState* st, int j, bool vec) {
  const int ss = st->stop_step;
  if (ss >= 0 && ss < j) return;
  const int kind = (ss == j) ? st->stop_kind : STOP_NONE;
  const bool have_v = (kind == STOP_NONE || kind == STOP_CONV);
  const double cx = st->cx, cw = st->cw;
  const double ia = have_v ? 1.0 / st->alpha[j] : 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < n; e += stride) {
    double xv[4], wv[4];
    ld4(X, e, n, vec, xv);
    ld4(W, e, n, vec, wv);
    for (int u = 0; u < 4; ++u) xv[u] += cx * wv[u];
    st4(X, e, n, vec, xv);
    if (have_v) {
      double vv[4];
      ld4(Vn, e, n, vec, vv);
      for (int u = 0; u < 4; ++u) {
        vv[u] *= ia;
        vv[u] = (double)(T)vv[u];
        wv[u] = vv[u] - cw * wv[u];
      }
      st4(Vn, e, n, vec, vv);
      st4(W, e, n, vec, wv);
    }
  }
}

// LSQR start (Algorithm 6 step 2): V_1 = V~/alpha_1 in place, W_1 = V_1, X_0 = 0.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lsqr_start(int64_t n, T* X, T* W, T* V1, KState* st, bool vec) {
  const bool ok = st->stop_step < 0;
  const double ia = ok ? 1.0 / st->alpha[0] : 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < n; e += stride) {
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    st4(X, e, n, vec, z);
    if (ok) {
      double v[4];
      ld4(V1, e, n, vec, v);
      for (int u = 0; u < 4; ++u) v[u] = (double)(T)(v[u] * ia);
      st4(V1, e, n, vec, v);
      st4(W, e, n, vec, v);
    } else {
      st4(W, e, n, vec, z);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_zero(int64_t n, T* x) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) x[e] = (T)0;
}

// full = 1: clear everything (new solve); full = 0: start a new GMRES cycle (unless halted)
__global__ void k_state_reset(KState* st, int full, double tol) {
  if (full == 0 && st->halt) return;
  double* d = reinterpret_cast<double*>(st);
  const int nd = (int)(sizeof(KState) / sizeof(double));
  if (full) {
    for (int i = threadIdx.x; i < nd; i += blockDim.x) d[i] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      st->stop_step = -1;
      st->stop_kind = STOP_NONE;
      st->status = DCTK_OK;
      st->tol = tol;
      st->gcv = __builtin_nan("");
    }
  } else {
    for (int i = threadIdx.x; i < (kMaxK + 1) * kMaxK; i += blockDim.x) st->H[i] = 0.0;
    if (threadIdx.x == 0) {
      st->steps = 0;
      st->stop_step = -1;
      st->stop_kind = STOP_NONE;
      st->scale = 0.0;
    }
  }
}

template <typename TO>
__global__ __launch_bounds__(kThreads) void k_cast(int64_t n, const double* in, TO* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) out[e] = cvt<TO, double>(in[e]);
}

// ---- launchers ---------------------------------------------------------------
static inline unsigned grid_for(int64_t n) {
  int64_t b = ((n + 3) / 4 + kThreads - 1) / kThreads;
  if (b > kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (unsigned)b;
}
static inline bool aligned32(const void* p) { return p == nullptr || ((uintptr_t)p % 32) == 0; }

hipError_t launch_axpy_red(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* x, const void* y,
                           const double* cptr, double csign, double cconst, const void* z, int act,
                           double* dst, KState* st, int j, Gate g) {
  unsigned grid = grid_for(n);
  bool vec = (n % 4 == 0) && aligned32(out) && aligned32(x) && aligned32(y) && aligned32(z);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_axpy_red<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)out,
                       (const double*)x, (const double*)y, cptr, csign, cconst, (const double*)z, act, dst, st, j,
                       ctx->red_partials, ctx->red_tickets, vec, g);
  else
    hipLaunchKernelGGL(k_axpy_red<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)out,
                       (const float*)x, (const float*)y, cptr, csign, cconst, (const float*)z, act, dst, st, j,
                       ctx->red_partials, ctx->red_tickets, vec, g);
  return hipGetLastError();
}

hipError_t launch_scale(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* in, const double* den, Gate g) {
  unsigned grid = grid_for(n);
  bool vec = (n % 4 == 0) && aligned32(out) && aligned32(in);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_scale<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)out,
                       (const double*)in, den, vec, g);
  else
    hipLaunchKernelGGL(k_scale<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)out,
                       (const float*)in, den, vec, g);
  return hipGetLastError();
}

hipError_t launch_multidot(dctk_ctx ctx, int dtype, int64_t n, const void* basis, int64_t stride, int nb,
                           const void* w, double* dst, int dst_stride, int accumulate, double* coef_copy, Gate g) {
  if (nb <= 0) return hipSuccess;
  unsigned grid = grid_for(n);
  bool vec = (n % 4 == 0) && (stride % 4 == 0) && aligned32(basis) && aligned32(w);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_multidot<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (const double*)basis,
                       stride, nb, (const double*)w, dst, dst_stride, accumulate, coef_copy, ctx->red_partials,
                       ctx->red_tickets, vec, g);
  else
    hipLaunchKernelGGL(k_multidot<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (const float*)basis,
                       stride, nb, (const float*)w, dst, dst_stride, accumulate, coef_copy, ctx->red_partials,
                       ctx->red_tickets, vec, g);
  return hipGetLastError();
}

hipError_t launch_subtract(dctk_ctx ctx, int dtype, int64_t n, void* w, const void* basis, int64_t stride, int nb,
                           const double* coef, int cstride, Gate g) {
  if (nb <= 0) return hipSuccess;
  unsigned grid = grid_for(n);
  bool vec = (n % 4 == 0) && (stride % 4 == 0) && aligned32(basis) && aligned32(w);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_subtract<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)w,
                       (const double*)basis, stride, nb, coef, cstride, vec, g);
  else
    hipLaunchKernelGGL(k_subtract<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)w,
                       (const float*)basis, stride, nb, coef, cstride, vec, g);
  return hipGetLastError();
}

hipError_t launch_combine(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* x0, const void* basis,
                          int64_t stride, int nb, const int* nptr, const double* y, Gate g) {
  unsigned grid = grid_for(n);
  bool vec = (n % 4 == 0) && (stride % 4 == 0) && aligned32(out) && aligned32(x0) && aligned32(basis);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_combine<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)out,
                       (const double*)x0, (const double*)basis, stride, nb, nptr, y, vec, g);
  else
    hipLaunchKernelGGL(k_combine<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)out,
                       (const float*)x0, (const float*)basis, stride, nb, nptr, y, vec, g);
  return hipGetLastError();
}

hipError_t launch_lsqr_update(dctk_ctx ctx, int dtype, int64_t n, void* X, void* W, void* Vn, KState* st, int j) {
  unsigned grid = grid_for(n);
  bool vec = (n % 4 == 0) && aligned32(X) && aligned32(W) && aligned32(Vn);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_lsqr_update<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)X, (double*)W,
                       (double*)Vn, st, j, vec);
  else
    hipLaunchKernelGGL(k_lsqr_update<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)X, (float*)W,
                       (float*)Vn, st, j, vec);
  return hipGetLastError();
}

hipError_t launch_lsqr_start(dctk_ctx ctx, int dtype, int64_t n, void* X, void* W, void* V1, KState* st) {
  unsigned grid = grid_for(n);
  bool vec = (n % 4 == 0) && aligned32(X) && aligned32(W) && aligned32(V1);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_lsqr_start<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)X, (double*)W,
                       (double*)V1, st, vec);
  else
    hipLaunchKernelGGL(k_lsqr_start<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)X, (float*)W,
                       (float*)V1, st, vec);
  return hipGetLastError();
}

hipError_t launch_lsqr_scalars(dctk_ctx ctx, KState* st, int j) {
  hipLaunchKernelGGL(k_lsqr_scalars, dim3(1), dim3(64), 0, ctx->stream, st, j);
  return hipGetLastError();
}

hipError_t launch_fill_zero(dctk_ctx ctx, int dtype, int64_t n, void* x) {
  unsigned grid = grid_for(n * 4 > n ? n : n);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_fill_zero<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)x);
  else
    hipLaunchKernelGGL(k_fill_zero<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)x);
  return hipGetLastError();
}

hipError_t launch_cast(dctk_ctx ctx, int64_t n, const double* in, int out_dtype, void* out) {
  unsigned grid = grid_for(n * 4);
  switch (out_dtype) {
    case DCTK_F64: hipLaunchKernelGGL(k_cast<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, in, (double*)out); break;
    case DCTK_F32: hipLaunchKernelGGL(k_cast<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, in, (float*)out); break;
    case DCTK_BF16: hipLaunchKernelGGL(k_cast<bf16_t>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, in, (bf16_t*)out); break;
    case DCTK_F16: hipLaunchKernelGGL(k_cast<f16_t>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, in, (f16_t*)out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_state_reset(dctk_ctx ctx, KState* st, int full, double tol) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(256), 0, ctx->stream, st, full, tol);
  return hipGetLastError();
}

}  // namespace dctk
