// Internal declarations of libdctkrylov (not installed).  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "../../include/dctkrylov.h"

namespace dctk {

constexpr int kMaxK = 64;              // largest Krylov dimension (projected problem <= 65 x 64)
constexpr int kRedBlocks = 1024;       // max blocks of a reducing kernel
constexpr int kRedVals = kMaxK + 2;    // max values reduced by one kernel
constexpr int kTickets = 8;            // reduction ticket counters per context
constexpr int kThreads = 256;          // threads per block of streaming kernels
constexpr int kMaxTube = 64;           // largest n3 (the p x p transform matrix sits in LDS)

typedef unsigned short bf16_t;         // storage of bfloat16 (bit pattern)
typedef _Float16 f16_t;

// ---- device-resident state of one Krylov workspace ------------------------
// Gate phases: which part of a Golub-Kahan / Arnoldi step a kernel belongs to.
enum Phase : int {
  PH_ALWAYS = 0,   // runs unless the process stopped at an earlier step
  PH_AFTER_U = 1,  // GKB: needs U_{j+1} (skipped after a beta breakdown in this step)
  PH_VNORM = 2,    // GKB: needs V_{j+1} (skipped after any breakdown in this step)
  PH_WUPD = 3,     // LSQR: search-direction update (skipped after any breakdown)
};
enum StopKind : int { STOP_NONE = 0, STOP_BETA = 1, STOP_ALPHA = 2, STOP_CONV = 3 };

struct KState {
  int steps;        // steps completed in the current process
  int stop_step;    // -1 while running; else the 1-based step at which it stopped
  int stop_kind;    // StopKind
  int status;       // DCTK_OK / DCTK_BREAKDOWN
  int converged;
  int cycles;       // GMRES cycles finished
  int halt;         // GMRES: set on convergence / zero residual; every gated kernel skips
  int total_steps;  // GMRES: Arnoldi steps over all cycles
  double scale;     // running max of alpha, beta (or |h|) for the breakdown test
  double rhobar, phibar;
  double cx, cw;    // LSQR step (f): X += cx W;  W = V_{j+1} - cw W
  double tol;
  double beta0;     // ||R_0|| (Arnoldi) or beta_1 (GKB)
  double lambda;    // projected solve: lambda used
  double gcv;       // GCV value at lambda
  double resnorm;   // GMRES: ||C - M(X)||
  double alpha[kMaxK + 2];
  double beta[kMaxK + 2];
  double H[(kMaxK + 1) * kMaxK];   // Arnoldi Hessenberg, row-major, ld = kMaxK
  double coef[kRedVals];           // Gram coefficients of the current reorthogonalisation pass
  double y[kMaxK + 1];             // projected solution
};

struct Gate {
  const KState* st;  // nullptr: always open
  int j;             // 1-based step the kernel belongs to
  int phase;
};

__device__ inline bool gate_open(const Gate& g) {
  if (g.st == nullptr) return true;
  const volatile KState* st = g.st;
  if (st->halt) return false;
  int ss = st->stop_step;
  if (ss < 0 || ss > g.j) return true;
  if (ss < g.j) return false;
  int kind = st->stop_kind;
  switch (g.phase) {
    case PH_AFTER_U: return kind != STOP_BETA;
    case PH_VNORM: return kind == STOP_CONV;
    case PH_WUPD: return kind == STOP_CONV;
    default: return true;
  }
}

// ---- type helpers ----------------------------------------------------------
template <typename T> struct AccOf { typedef float type; };
template <> struct AccOf<double> { typedef double type; };

__device__ __host__ inline float bf16_to_float(bf16_t v) {
  union { uint32_t u; float f; } c;
  c.u = ((uint32_t)v) << 16;
  return c.f;
}
__device__ __host__ inline bf16_t float_to_bf16(float f) {  // round to nearest even
  union { uint32_t u; float f; } c;
  c.f = f;
  uint32_t u = c.u;
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (bf16_t)(u >> 16);
}

template <typename TO, typename TI> __device__ inline TO cvt(TI v) { return (TO)v; }
template <> __device__ inline bf16_t cvt<bf16_t, float>(float v) { return float_to_bf16(v); }
template <> __device__ inline bf16_t cvt<bf16_t, double>(double v) { return float_to_bf16((float)v); }
template <> __device__ inline float cvt<float, bf16_t>(bf16_t v) { return bf16_to_float(v); }
template <> __device__ inline f16_t cvt<f16_t, double>(double v) { return (f16_t)(float)v; }

// ---- wave / block reductions (64-wide waves) -----------------------------
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over a block of kThreads threads; result valid in thread 0.  `sh` holds
// kThreads/64 doubles.  Fixed order: deterministic.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  }
  __syncthreads();
  return r;
}

}  // namespace dctk

// ---- opaque handle definitions ---------------------------------------------
struct dctk_ctx_s {
  int device;
  hipStream_t stream;
  int last_hip_error;
  int num_cus;
  double* red_partials;   // kRedBlocks * kRedVals doubles
  unsigned* red_tickets;  // kTickets counters, zero between uses
  double* red_out;        // kRedVals doubles: results of standalone reductions
  void* prof;             // dctk::Profiler while profiling, else null
};

struct dctk_op_s {
  dctk_ctx ctx;
  int tube, gemm_dtype, vec_dtype;
  int64_t p, n1, n2, s;
  int two_sided;
  void* Ah;       // p*n1*n2, gemm dtype
  void* Bh;       // p*s*s, gemm dtype (two-sided)
  double* Gd;     // 4 matrices p*p (L, L^-1, L^-T, L^T), FP64
  float* Gf;      // same in FP32
  void* xh;       // transformed operand, gemm dtype, p*max(n1,n2)*s
  void* th;       // two-sided intermediate, gemm dtype, p*max(n1,n2)*s
  void* ch;       // slice products, accumulator dtype, p*max(n1,n2)*s
};

struct dctk_krylov_s {
  dctk_op op;
  int kind, k_max, ortho;
  int reorth;
  int initialised;
  int host_steps;          // steps enqueued since init
  int64_t nvec;            // elements of one basis vector: p*max(n1,n2)*s
  size_t vbytes;           // bytes of one basis vector (vector dtype)
  void* U;                 // (k_max+1) vectors (GKB U / Arnoldi V)
  void* V;                 // (k_max+1) vectors (GKB V)
  void* X;                 // LSQR iterate
  void* W;                 // LSQR search direction
  void* T;                 // scratch vector (product result)
  void* R;                 // GMRES residual
  dctk::KState* st;        // device state
};

namespace dctk {

// ---- profiling: HIP events around transform / GEMM launches -----------------
enum ProfKind : int { PROF_TUBE_FWD = 0, PROF_GEMM = 1, PROF_TUBE_INV = 2, PROF_KINDS = 3 };
void prof_begin(dctk_ctx ctx, int kind);  // no-ops unless profiling
void prof_end(dctk_ctx ctx, int kind);

// error plumbing
int hip_fail(dctk_ctx ctx, hipError_t e);
#define DCTK_HIP(ctx, call)                                   \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return ::dctk::hip_fail((ctx), e_); \
  } while (0)

// transform matrices (host, FP64): which = DCTK_MAT_*
int build_tube_matrix(int tube, int which, int64_t p, double* out);

// ---- launchers (all enqueue on `stream`) -----------------------------------
// out[k][e] = a * sum_t G[k][t] in[t][e] + b * src[k][e]   (src may be null when b == 0)
hipError_t launch_tube(hipStream_t s, int vec_dtype, int out_dtype, int64_t p, int64_t count,
                       const void* in, void* out, const double* Gd, const float* Gf,
                       double a, double b, const void* src, Gate g);

// C_k = op(A_k) op(B_k), batched over `batch`; A: M x K (or K x M if ta), B: K x N (or N x K if tb)
hipError_t launch_gemm(hipStream_t s, int in_dtype, int out_acc, int M, int N, int K,
                       const void* A, int64_t lda, int64_t sA, int ta,
                       const void* B, int64_t ldb, int64_t sB, int tb,
                       void* C, int64_t ldc, int64_t sC, int batch, Gate g);

// Full c-product / adjoint on the op's workspaces:  Y = a*M(X) + b*src
hipError_t apply_op(dctk_op op, hipStream_t s, int adjoint, double a, const void* X, double b,
                    const void* src, void* Y, Gate g);

// ---- streaming vector kernels (vec.hip) ------------------------------------
enum Act : int {
  ACT_STORE = 0,       // out_slot[0] = sqrt(sum)
  ACT_GKB_BETA1 = 1,   // GKB init: beta_1
  ACT_GKB_ALPHA1 = 2,  // GKB init: alpha_1 (+ LSQR start)
  ACT_GKB_BETA = 3,    // beta_{j+1} + breakdown test
  ACT_GKB_ALPHA = 4,   // alpha_{j+1} + breakdown test
  ACT_ARN_BETA = 5,    // Arnoldi init: beta = ||R_0||
  ACT_ARN_H = 6,       // h_{j+1,j} + breakdown test
  ACT_GMRES_RES = 7,   // GMRES: ||C - M(X)|| + convergence test
  ACT_DOT_STORE = 8,   // dst[0] = sum (no square root)
};

// out = x + c*y (c = csign * (*cptr) if cptr else cconst); when act >= 0 also
// reduce sum(out . z) (z null: out . out) into the action.  y may be null
// (out = x); out may be null (reduce only).
hipError_t launch_axpy_red(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* x,
                           const void* y, const double* cptr, double csign, double cconst,
                           const void* z, int act, double* dst, KState* st, int j, Gate g);
// out = in / (*den)
hipError_t launch_scale(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* in,
                        const double* den, Gate g);
// coef[i] (+)= <basis_i, w> for i < nb (basis vectors `stride` elements apart); accumulate
// into dst (dst[i*dst_stride]) when accumulate, else overwrite.
hipError_t launch_multidot(dctk_ctx ctx, int dtype, int64_t n, const void* basis, int64_t stride,
                           int nb, const void* w, double* dst, int dst_stride, int accumulate,
                           double* coef_copy, Gate g);
// w -= sum_i coef[i*cstride] basis_i
hipError_t launch_subtract(dctk_ctx ctx, int dtype, int64_t n, void* w, const void* basis,
                           int64_t stride, int nb, const double* coef, int cstride, Gate g);
// out = (x0 ? x0 : 0) + sum_{i < *nptr (or nb)} y[i] basis_i
hipError_t launch_combine(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* x0,
                          const void* basis, int64_t stride, int nb, const int* nptr,
                          const double* y, Gate g);
// LSQR step (f) with V normalisation
hipError_t launch_lsqr_update(dctk_ctx ctx, int dtype, int64_t n, void* X, void* W, void* Vnext,
                              KState* st, int j);
hipError_t launch_lsqr_start(dctk_ctx ctx, int dtype, int64_t n, void* X, void* W, void* V1, KState* st);
hipError_t launch_lsqr_scalars(dctk_ctx ctx, KState* st, int j);
hipError_t launch_fill_zero(dctk_ctx ctx, int dtype, int64_t n, void* x);
hipError_t launch_state_reset(dctk_ctx ctx, KState* st, int full, double tol);
hipError_t launch_cast(dctk_ctx ctx, int64_t n, const double* in, int out_dtype, void* out);
void set_num_cus(int n);
size_t elem_size(int dt);

// projected FP64 problem (projected.hip): bidiag = 1 reads alpha/beta, else H.
// Writes st->y[0..k), st->lambda, st->gcv.
hipError_t launch_projected(dctk_ctx ctx, KState* st, int bidiag, int gcv_mode, double lambda);

}  // namespace dctk
