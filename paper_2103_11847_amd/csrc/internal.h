// Internal declarations of libdctkrylov (not installed).  gfx950 only.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <cstddef>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "../../include/dctkrylov.h"

namespace dctk {

constexpr int kMaxK = 64;              // largest Krylov dimension (projected problem <= 65 x 64)
constexpr int kRedBlocks = 4096;       // max blocks of a reducing kernel (partials per reduction)
constexpr int kNormParts = 4 * kRedBlocks;  // capacity of the norm partial buffers (fused products write one per wave)
constexpr int kRedVals = kMaxK + 2;    // max values reduced by one multi-dot kernel
constexpr int kThreads = 256;          // threads per block of streaming kernels
constexpr int kShCtl = 2 * (kThreads / 64 + 1);  // LDS doubles of the prologue reductions (blocks <= kThreads)
constexpr int kMaxTube = 64;           // largest n3 (the p x p transform matrix sits in LDS)
constexpr int kMaxTubeModes = 6;       // tube modes of an order-N operator (N <= 8)
constexpr int kFusedMaxP = 8;          // n3 up to which a c-product is one fused kernel
constexpr int kFastOpMaxP = 2048;      // longest tube of an operator (the fast transform's FP64 limit)
constexpr double kBreakFactor = 64.0;  // breakdown: new norm <= 64 eps * running max

typedef unsigned short bf16_t;         // storage of bfloat16 (bit pattern)
typedef _Float16 f16_t;

// ---- device-resident state of one Krylov workspace ------------------------
// Every scalar a step produces is stored at its step index, so a kernel only
// reads entries written by earlier kernels: no intra-kernel races between the
// block that records a scalar and the blocks that use it.
enum StopKind : int { STOP_NONE = 0, STOP_BETA = 1, STOP_ALPHA = 2, STOP_CONV = 3 };

struct KState {
  int steps;        // steps completed in the current process
  int stop_step;    // -1 while running; else the 1-based step at which it stopped
  int stop_kind;    // StopKind (GKB: which norm broke down; Arnoldi: STOP_BETA)
  int status;       // DCTK_OK / DCTK_BREAKDOWN / DCTK_ENONFINITE
  int converged;
  int cycles;       // GMRES cycles finished
  int halt;         // GMRES: set on convergence / zero residual; every gated kernel skips
  int total_steps;  // GMRES: Arnoldi steps over all cycles
  double tol;
  double beta0;     // ||R_0|| (Arnoldi)
  double lambda;    // projected solve: lambda used
  double gcv;       // GCV value at lambda
  double resnorm;   // GMRES: ||C - M(X)||
  double sweeps;    // one-sided Jacobi sweeps of the last projected solve
  double gate_ok;   // 1 when a proposed lambda passed the GCV gate of the last projected solve
  double pad;
  double alpha[kMaxK + 2];          // GKB alpha_1.. at [0..]
  double beta[kMaxK + 2];           // GKB beta_1.. at [0..]
  double rhobar[kMaxK + 2];         // LSQR rhobar_{j+1} at [j]
  double phibar[kMaxK + 2];         // LSQR phibar_{j+1} at [j]
  double H[(kMaxK + 1) * kMaxK];    // Arnoldi Hessenberg, row-major, ld = kMaxK
  double coef[kRedVals];            // Gram coefficients of the current reorthogonalisation pass
  double y[kMaxK + 1];              // projected solution
  int k_limit;                      // > 0: GKB steps beyond it are skipped (learned stop)
  int pad_i;
  double pred_lambda;               // learned stop: predicted lambda (0: none)
};


// Loads of state fields that a workgroup of the same kernel may be writing:
// relaxed device-scope atomic loads.  (A volatile access would do, but on this
// target each one waits for every outstanding load of the thread, so a
// prologue of several of them pays the memory latency several times.)
__device__ inline int ld_state(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline double ld_state(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- control of a product kernel inside a Krylov step -----------------------
// A c-product inside a Krylov step reads its scalars from the device: either
// by summing the per-block partials of the previous kernel (fixed order, in
// every block, so all blocks agree bit for bit) or from the state arrays.
enum CtlKind : int {
  CTL_PLAIN = 0,     // out = a*y + b*src with constant a, b; input scale s
  CTL_GKB_INIT = 1,  // Alg. 4 step 2: beta_1 = sqrt(sum part_in); input x 1/beta_1 (-> U_1); out = M*(U_1)
  CTL_GKB_FWD = 2,   // Alg. 4 (a): out = M(V_j) - alpha_j U_j
  CTL_GKB_ADJ = 3,   // Alg. 4 (b)-(d): beta_{j+1} = sqrt(sum part_in); input x 1/beta (-> U_{j+1});
                     //   out = M*(U_{j+1}) - beta_{j+1} V_j
  CTL_ARN_FWD = 4,   // Alg. 2 (a): h_{j,j-1} = sqrt(sum part_in) (j > 1); input x 1/h (-> V_j); out = M(V_j)
  CTL_GKB_FWDU = 5,  // the LSQR update of step j-1 (Alg. 4 (e)-(f), Alg. 6 (c)-(e) without X, W):
                     //   alpha_j = sqrt(sum part_in), the rotation; input V~ x 1/alpha_j (-> V_j);
                     //   then Alg. 4 (a) of step j: out = M(V_j) - alpha_j U_j
};

struct Ctl {
  int kind;
  int j;                  // 1-based step (0: initialisation)
  int from_state;         // 1: scalars already recorded in st (later kernels of an unfused product)
  int npart_in;
  // GKB products: src holds its basis vector unnormalised (beta_j U_j for the
  // forward product, alpha_j V_j for the adjoint), so the epilogue's b is
  // divided by that recorded normaliser
  int src_div;
  int pad_;
  KState* st;
  const double* part_in;  // partials consumed (sums of squares)
  double* part_out;       // per-block sum of squares of the output (nullptr: none)
  double a, b, s;         // CTL_PLAIN constants
};

// ---- type helpers ----------------------------------------------------------
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
template <> __device__ inline f16_t cvt<f16_t, double>(double v) { return (f16_t)(float)v; }

// ---- wave / block reductions (64-wide waves) -----------------------------
// DPP moves of a 64-bit value (two 32-bit halves) within 16-lane rows
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  const long long r = ((long long)(unsigned)lo) | ((long long)hi << 32);
  return __builtin_bit_cast(double, r);
}

// Sum over the 16 lanes of a row, returned to every lane of the row (identical
// bits: each step adds a commuted copy of the same partial sums).  All lanes
// of the wave must be active.
__device__ inline double row16_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}

__device__ inline double readlane_d(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Sum over the wave in a fixed order, the same in every lane (all lanes active).
__device__ inline double wave_sum(double v) {
  v = row16_sum(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Sum over the block; the result is returned to every thread.  `sh` holds
// blockDim/64 + 1 doubles.  Fixed order: deterministic.
__device__ inline double block_sum_all(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
    sh[blockDim.x >> 6] = r;
  }
  __syncthreads();
  return sh[blockDim.x >> 6];
}

__device__ inline double block_max_all(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, sh[w]);
    sh[blockDim.x >> 6] = r;
  }
  __syncthreads();
  return sh[blockDim.x >> 6];
}

// Sum of part[0..n) in a fixed order, returned to every thread of the block.
__device__ inline double block_sum_partials(const double* part, int n, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
  return block_sum_all(v, sh);
}

// This thread's share of sum(part[0..n)): block_sum_all of it is
// block_sum_partials.  The values are added in the order of the plain strided
// loop.  part_first takes the first 4 * blockDim entries with four loads that
// need neither a loop nor a branch (clamped addresses, then selects; part[0]
// must exist), so they stay in flight with the caller's other loads -- on this
// target a load inside a conditional block or a loop is waited for before the
// block ends.  part_rest adds the entries beyond (a loop, rarely entered).
__device__ inline double part_first(const double* part, int n) {
  const int bd = (int)blockDim.x, i = (int)threadIdx.x;
  const int i1 = i + bd, i2 = i + 2 * bd, i3 = i + 3 * bd;
  const double a0 = part[i < n ? i : 0], a1 = part[i1 < n ? i1 : 0];
  const double a2 = part[i2 < n ? i2 : 0], a3 = part[i3 < n ? i3 : 0];
  double v = 0.0;
  v = i < n ? v + a0 : v;
  v = i1 < n ? v + a1 : v;
  v = i2 < n ? v + a2 : v;
  v = i3 < n ? v + a3 : v;
  return v;
}
__device__ inline double part_rest(double v, const double* part, int n) {
  for (int i = (int)threadIdx.x + 4 * (int)blockDim.x; i < n; i += (int)blockDim.x) v += part[i];
  return v;
}
__device__ inline double part_local(const double* part, int n) {
  if (n <= 0) return 0.0;
  return part_rest(part_first(part, n), part, n);
}

// (1 <= na, nb <= kMaxK + 2 < kThreads: one value of each per thread, from an
// index clamped into the range -- a repeated value does not change the max --
// so the loads need no branch)
__device__ inline double gkb_scale_local(const KState* st, int na, int nb) {
  static_assert(kMaxK + 2 <= kThreads, "one history value per thread");
  const int i = (int)threadIdx.x;
  const double av = st->alpha[i < na ? i : na - 1], bv = st->beta[i < nb ? i : nb - 1];
  return fmax(fabs(av), fabs(bv));
}

// Running max of |alpha_1..alpha_na|, |beta_1..beta_nb| over the block.
__device__ inline double gkb_scale(const KState* st, int na, int nb, double* sh) {
  return block_max_all(gkb_scale_local(st, na, nb), sh);
}

// Sum of s (in block_sum_all's order, so the same bits) and max of m over the
// block in one exchange; both returned to every thread.  `sh` holds kShCtl doubles.
__device__ inline void block_sum_max_all(double& s, double& m, double* sh) {
  s = wave_sum(s);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  __syncthreads();
  if (lane == 0) {
    sh[2 * wid] = s;
    sh[2 * wid + 1] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0, x = sh[1];
    for (int w = 0; w < nw; ++w) {
      r += sh[2 * w];
      x = fmax(x, sh[2 * w + 1]);
    }
    sh[2 * nw] = r;
    sh[2 * nw + 1] = x;
  }
  __syncthreads();
  s = sh[2 * nw];
  m = sh[2 * nw + 1];
}

// ---- plain and grouped launches -------------------------------------------------
// A kernel that can run for several problem instances in one launch takes its
// arguments as one struct `a` (which records the instance's own grid in gx, gy,
// gz) plus two pointers: for a grouped launch, `grp` holds the argument
// structs of the instances and `bmap` gives, for every workgroup of the 1-D
// launch grid, {instance, x, y, z} within that instance's grid.  A plain launch
// passes null for both and the hardware indices are used.
struct VBlock {
  int x, y, z;
};

__device__ inline VBlock hw_block() { return VBlock{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z}; }

// Grouped launches: the instance's argument struct and its workgroup index,
// copied word by word through readfirstlane so they stay in scalar registers.
// (Each batchable kernel has a body taking the struct by reference and two
// call sites -- the kernel argument itself, or this copy -- so the plain path
// reads its pointers straight from the kernel arguments, where the compiler
// knows them to be global.)
template <typename A>
__device__ inline A group_args(const A* grp, const int4* bmap, VBlock& vb) {
  static_assert(sizeof(A) % 4 == 0, "argument struct of whole words");
  const int4 m = bmap[blockIdx.x];
  vb = VBlock{__builtin_amdgcn_readfirstlane(m.y), __builtin_amdgcn_readfirstlane(m.z),
              __builtin_amdgcn_readfirstlane(m.w)};
  const int* src = reinterpret_cast<const int*>(grp + __builtin_amdgcn_readfirstlane(m.x));
  A r;
  int* dst = reinterpret_cast<int*>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(A) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return r;
}

// Algorithm 4 (e)-(f) with Algorithm 6 (c)-(e) for step j, after the adjoint
// product: unless beta_{j+1} broke down, alpha_{j+1} from this thread's share
// of the partials of ||V~||^2 (ps, already including every entry) and of the
// breakdown scale (pm), with its breakdown test; then the plane rotation from
// beta_{j+1} (bnext), rhobar_j, phibar_j.  `first` records alpha_{j+1},
// rhobar_{j+1}, phibar_{j+1} and the stop flags.  Every thread of the block
// calls it (block reduction); (cx, cw) are the X and W update coefficients.
struct GkbUpd {
  double alpha, cx, cw;
  bool have_v;
};
__device__ inline GkbUpd gkb_update_scalars(KState* st, int j, double ps, double pm, double bnext, double rhob,
                                            double phib, double tol, int ss, int skind, double* sh, bool first) {
  const bool bbreak = (ss == j && skind == STOP_BETA);
  double alpha = 0.0;
  bool abreak = false, fin = true;
  if (!bbreak) {
    block_sum_max_all(ps, pm, sh);
    alpha = sqrt(ps);
    const double scale = fmax(pm, alpha);
    fin = isfinite(alpha);
    abreak = !fin || alpha <= kBreakFactor * 2.220446049250313e-16 * scale;
  }
  const double anext = bbreak ? 0.0 : alpha;
  const double rho = sqrt(rhob * rhob + bnext * bnext);
  const double c = rhob / rho, s = bnext / rho;
  const double theta = s * anext;
  const double phi = c * phib;
  const double phibar_new = -s * phib;
  const bool conv = !bbreak && !abreak && fabs(phibar_new) < tol;
  if (first) {
    if (!bbreak) {
      st->alpha[j] = alpha;
      st->steps = j;
    }
    st->rhobar[j] = c * anext;
    st->phibar[j] = phibar_new;
    if (abreak) {
      st->stop_step = j;
      st->stop_kind = STOP_ALPHA;
      st->status = fin ? DCTK_BREAKDOWN : DCTK_ENONFINITE;
    } else if (conv) {
      st->stop_step = j;
      st->stop_kind = STOP_CONV;
      st->converged = 1;
    }
  }
  return GkbUpd{alpha, phi / rho, theta / rho, !bbreak && !abreak};
}

// What a control block reads from memory.  ctl_load issues every load (the
// recorded scalar, this thread's share of the history that scales the
// breakdown test and of the partials, then the stop flags), none of them
// inside a branch -- on this target a load in a conditional block is waited
// for before the block ends; ctl_eval uses them.  A kernel that issues its own
// first loads, then calls ctl_load, waits for memory once.
struct CtlLoad {
  double ps, pm, rec;
  double bn, rb, pb, tol;  // the LSQR update (CTL_GKB_FWDU): beta_j, rhobar_{j-1}, phibar_{j-1}, tol
  double an;               // alpha_j (the normaliser of an unnormalised V_j source)
  int ss, kl, halt, sk;
};

__device__ inline CtlLoad ctl_load(const Ctl& c) {
  CtlLoad L{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -1, 0, 0, 0};
  if (c.kind == CTL_PLAIN) {
    if (c.st != nullptr) L.halt = ld_state(&c.st->halt);
    return L;
  }
  // Every load is unconditional, from an index computed (or clamped) into the
  // state or the partials; the kind only selects indices and, afterwards,
  // values.
  const KState* st = c.st;
  const double* sd = reinterpret_cast<const double*>(st);
  constexpr int oA = (int)(offsetof(KState, alpha) / sizeof(double));
  constexpr int oB = (int)(offsetof(KState, beta) / sizeof(double));
  constexpr int oH = (int)(offsetof(KState, H) / sizeof(double));
  constexpr int oRB = (int)(offsetof(KState, rhobar) / sizeof(double));
  constexpr int oPB = (int)(offsetof(KState, phibar) / sizeof(double));
  constexpr int oTol = (int)(offsetof(KState, tol) / sizeof(double));
  const int j = c.j, i = (int)threadIdx.x;
  const bool fs = c.from_state != 0;
  const bool fwd = c.kind == CTL_GKB_FWD, ini = c.kind == CTL_GKB_INIT, adj = c.kind == CTL_GKB_ADJ,
             arn = c.kind == CTL_ARN_FWD, fwdu = c.kind == CTL_GKB_FWDU;
  // the recorded scalar this kernel needs (beta_1 when none)
  int ri = oB;
  ri = (fs && arn && j > 1) ? oH + (j - 1) * kMaxK + j - 2 : ri;
  ri = (fs && adj) ? oB + j : ri;
  ri = (fwd || (fs && fwdu)) ? oA + j - 1 : ri;
  L.rec = sd[ri];
  // breakdown scale: max |alpha_1..alpha_na|, |beta_1..beta_j| (GKB adjoint:
  // na = j; LSQR update of step j-1: na = j - 1) or max_i |h_{i, j-1}|
  // (Arnoldi), one value of each per thread from a clamped index
  // (j <= kMaxK + 1 < kThreads; a repeated value does not change the max)
  static_assert(kMaxK + 2 <= kThreads, "one history value per thread");
  const int na = fwdu ? j - 1 : j;
  const int iaa = na > 1 ? (i < na ? i : na - 1) : 0, iab = j > 1 ? (i < j ? i : j - 1) : 0;
  const int ih = j > 2 ? (i < j - 1 ? i : j - 2) : 0, ch = j > 2 ? j - 2 : 0;
  const double av = sd[oA + iaa], bv = sd[oB + iab], hv = sd[oH + ih * kMaxK + ch];
  const double wab = (adj || fwdu) ? 1.0 : 0.0, wh = arn ? 1.0 : 0.0;
  L.pm = fmax(wab * fmax(fabs(av), fabs(bv)), wh * fabs(hv));
  // the recorded scalars of the LSQR update of step j - 1
  const int jp = j > 0 ? j - 1 : 0, jq = j > 1 ? j - 2 : 0;
  L.bn = sd[oB + jp];
  L.an = sd[oA + jp];
  L.rb = sd[oRB + jq];
  L.pb = sd[oPB + jq];
  L.tol = sd[oTol];
  // the partials of the norm (from beta_1, with no entries, when none)
  const bool sums = !fs && (ini || adj || fwdu || (arn && j > 1));
  L.ps = part_first(sums ? c.part_in : sd + oB, sums ? c.npart_in : 0);
  // the stop flags last: the compiler moves these uniform values to scalar
  // registers, which waits for them, and with them for every earlier load
  L.ss = ld_state(&st->stop_step);
  L.kl = ld_state(&st->k_limit);
  L.halt = ld_state(&st->halt);
  L.sk = ld_state(&st->stop_kind);
  return L;
}

// Evaluates the control block (all threads of every block call it).  Returns
// false when the kernel must do nothing.  Block (0, 0, 0) of the instance
// records the scalar it produced in the state.  `sh` holds kShCtl doubles
// (blocks of at most kThreads threads).
__device__ inline bool ctl_eval(const Ctl& c, const CtlLoad& L, double& a, double& b, double& sin, double* sh,
                                const VBlock& vb) {
  a = 1.0; b = 0.0; sin = 1.0;
  if (c.kind == CTL_PLAIN) {
    // a plain product inside a GMRES solve is skipped once the solve halted
    if (L.halt) return false;
    a = c.a; b = c.b; sin = c.s;
    return true;
  }
  // The loaded values are taken into registers here, in one wait: without
  // this use the compiler may sink each load into the branch that needs it,
  // where it would be waited for on its own.
  asm volatile("" ::"v"(L.ps), "v"(L.pm), "v"(L.rec), "v"(L.bn), "v"(L.an), "v"(L.ss), "v"(L.kl), "v"(L.halt));
  KState* st = c.st;
  const int j = c.j;
  const bool sums = !c.from_state && (c.kind == CTL_GKB_INIT || c.kind == CTL_GKB_ADJ || c.kind == CTL_GKB_FWDU ||
                                      (c.kind == CTL_ARN_FWD && j > 1));
  double ps = sums ? part_rest(L.ps, c.part_in, c.npart_in) : 0.0, pm = L.pm;
  const double rec = L.rec;
  const int ss = L.ss, kl = L.kl, halt = L.halt;
  const bool beyond = kl > 0 && j > kl;  // beyond a learned step limit
  const bool first = vb.x == 0 && vb.y == 0 && vb.z == 0 && threadIdx.x == 0;
  // an unnormalised source: beta_j U_j (forward kinds) or alpha_j V_j (adjoint)
  const double fdiv = c.src_div ? L.bn : 1.0, adiv = c.src_div ? L.an : 1.0;
  const double eps = 2.220446049250313e-16;
  switch (c.kind) {
    case CTL_GKB_INIT: {
      if (c.from_state) {
        if (ss == 0) return false;
        sin = 1.0 / rec;
        return true;
      }
      const double bt = sqrt(block_sum_all(ps, sh));
      const bool bad = !(bt > 0.0) || !isfinite(bt);
      if (first) {
        st->beta[0] = bt;
        st->steps = 0;
        if (bad) {
          st->stop_step = 0;
          st->stop_kind = STOP_BETA;
          st->status = isfinite(bt) ? DCTK_BREAKDOWN : DCTK_ENONFINITE;
        }
      }
      if (bad) return false;
      sin = 1.0 / bt;
      return true;
    }
    case CTL_GKB_FWD: {
      if (ss >= 0 || beyond) return false;  // stopped at an earlier step
      b = -rec / fdiv;
      return true;
    }
    case CTL_GKB_ADJ: {
      if ((ss >= 0 && ss < j) || beyond) return false;
      if (c.from_state) {
        if (ss == j) return false;
        sin = 1.0 / rec;
        b = -rec / adiv;
        return true;
      }
      block_sum_max_all(ps, pm, sh);
      const double bt = sqrt(ps);
      const double scale = fmax(pm, bt);
      const bool fin = isfinite(bt);
      const bool brk = !fin || bt <= kBreakFactor * eps * scale;
      if (first) {
        st->beta[j] = bt;
        st->steps = j;
        if (brk) {
          st->stop_step = j;
          st->stop_kind = STOP_BETA;
          st->status = fin ? DCTK_BREAKDOWN : DCTK_ENONFINITE;
        }
      }
      if (brk) return false;
      sin = 1.0 / bt;
      b = -bt / adiv;
      return true;
    }
    case CTL_GKB_FWDU: {
      if (c.from_state) {  // later kernels of an unfused product: as CTL_GKB_FWD
        if (ss >= 0 || beyond) return false;
        b = -rec / fdiv;
        return true;
      }
      const int jp = j - 1;  // the pending update
      if ((ss >= 0 && ss < jp) || (kl > 0 && jp > kl)) return false;
      const GkbUpd u = gkb_update_scalars(st, jp, ps, pm, L.bn, L.rb, L.pb, L.tol, ss, L.sk, sh, first);
      if (!u.have_v) return false;
      sin = 1.0 / u.alpha;
      b = -u.alpha / fdiv;
      return true;
    }
    case CTL_ARN_FWD: {
      if (halt) return false;
      if (ss >= 0 && ss < j) return false;
      if (j == 1) return true;  // V_1 was normalised by the cycle start
      const int r = j - 1, col = j - 2;   // h_{j, j-1} (1-based) at H[j-1][j-2]
      if (c.from_state) {
        if (ss == j - 1) return false;
        sin = 1.0 / rec;
        return true;
      }
      block_sum_max_all(ps, pm, sh);
      const double h = sqrt(ps);
      const double scale = fmax(pm, h);
      const bool fin = isfinite(h);
      const bool brk = !fin || h <= kBreakFactor * eps * scale;
      if (first) {
        st->H[r * kMaxK + col] = h;
        st->steps = j - 1;
        if (brk) {
          st->stop_step = j - 1;
          st->stop_kind = STOP_BETA;
          st->status = fin ? DCTK_BREAKDOWN : DCTK_ENONFINITE;
        }
      }
      if (brk) return false;
      sin = 1.0 / h;
      return true;
    }
    default:
      return false;
  }
}

__device__ inline bool ctl_begin(const Ctl& c, double& a, double& b, double& sin, double* sh, const VBlock& vb) {
  const CtlLoad L = ctl_load(c);
  return ctl_eval(c, L, a, b, sin, sh, vb);
}

// Gate of the plain kernels (GEMMs, reorthogonalisation passes) of a step:
// mode 0 runs while the process has not stopped before step j; mode 1 also
// requires that it did not stop at step j (its input exists).
struct Gate {
  const KState* st;  // nullptr: always open
  int j;
  int mode;
};

__device__ inline bool gate_open(const Gate& g) {
  if (g.st == nullptr) return true;
  const int halt = ld_state(&g.st->halt), kl = ld_state(&g.st->k_limit), ss = ld_state(&g.st->stop_step);
  if (halt) return false;
  if (kl > 0 && g.j > kl) return false;
  if (ss < 0) return true;
  return g.mode == 0 ? ss >= g.j : ss > g.j;
}

}  // namespace dctk

// ---- opaque handle definitions ---------------------------------------------
struct dctk_ctx_s {
  int device;
  hipStream_t stream;
  int last_hip_error;
  int num_cus;
  double* red_partials;   // kRedBlocks * kRedVals doubles: partials of standalone reductions
  void* prof;             // dctk::Profiler while profiling, else null
  void* rec;              // dctk::Recorder while a batch schedule is being planned, else null
  void* scratch;          // this device's copy of the no-allocation staging array (device address)
};

struct dctk_op_s {
  dctk_ctx ctx;
  int tube, gemm_dtype, vec_dtype;
  int64_t p, n1, n2, s;
  int two_sided;
  // product path per direction [0 forward, 1 adjoint]: {path, tile} with path
  // -1 by problem size, 0 unfused (transform, GEMM, transform), 1 fused; tile
  // 0 by problem size, else the output tile edge (set by dctk_op_autotune)
  int tune[2][2];
  void* Ah;       // p*n1*n2, gemm dtype
  void* AhT;      // p*n2*n1: slices of Ah transposed (FP32 and 16-bit gemm types), else null
  void* Bh;       // p*s*s, gemm dtype (two-sided)
  double* Gd;     // 4 matrices p*p (L, L^-1, L^-T, L^T), FP64 (null for a fast operator)
  float* Gf;      // same in FP32
  int fast;       // 1: tubes longer than kMaxTube, transformed in O(p log p) (power-of-two p)
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
  int last_npart;          // partials produced by the last enqueued norm (feeds the next step)
  // bit i set: V slot i holds alpha_{i+1} V_{i+1} (and U slot i beta_{i+1} U_{i+1}) unnormalised, as the
  // Tikhonov steps leave them; the combine divides y_i by alpha_{i+1}
  unsigned long long vmask;
  int64_t nvec;            // slot stride in elements (>= p*max(n1,n2)*s, 64-aligned)
  size_t vbytes;           // bytes of one slot
  void* U;                 // (k_max+1) slots (GKB U / Arnoldi V)
  void* V;                 // (k_max+1) slots (GKB V)
  void* X;                 // LSQR iterate
  void* W;                 // LSQR search direction
  void* T;                 // scratch vectors (2 slots)
  void* R;                 // GMRES residual
  double* partA;           // kNormParts partials (norms feeding the next product)
  double* partB;           // kNormParts partials
  double* partM;           // kRedBlocks * kRedVals partials of multi-dots
  dctk::KState* st;        // device state
};

namespace dctk {

// ---- profiling: HIP events around transform / GEMM launches -----------------
enum ProfKind : int {
  PROF_TUBE_FWD = 0,
  PROF_GEMM = 1,
  PROF_TUBE_INV = 2,
  PROF_FUSED_FWD = 3,
  PROF_FUSED_ADJ = 4,
  PROF_TUBE_PAIR = 5,
  PROF_KINDS = 6
};
void prof_begin(dctk_ctx ctx, int kind);  // no-ops unless profiling
void prof_end(dctk_ctx ctx, int kind);
// While profiling: creates a start/stop event pair for one kernel launch that
// records them itself (hipExtLaunchKernel) and registers it under kind; else
// sets both to null.
void prof_kernel(dctk_ctx ctx, int kind, hipEvent_t* start, hipEvent_t* stop);

// error plumbing
int hip_fail(dctk_ctx ctx, hipError_t e);
#define DCTK_HIP(ctx, call)                                   \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return ::dctk::hip_fail((ctx), e_); \
  } while (0)

// ---- launch recording (batch planning) ----------------------------------------
// While ctx->rec is set, the launchers of the batchable kernels append a record
// instead of launching: the kernel, the instance's grid and block, and the
// bytes of its argument struct.  `phase` is advanced by the planner between the
// steps of the schedule; `sub` numbers the records within a phase.
struct LaunchRec {
  const void* fn;        // the kernel's plain variant
  const void* fn_group;  // its grouped variant
  dim3 grid;
  unsigned threads;
  unsigned shmem;
  int phase, sub;
  std::vector<unsigned char> args;
};
struct Recorder {
  int phase = 0;
  int sub = 0;
  std::vector<LaunchRec> recs;
};
inline void rec_phase(dctk_ctx ctx) {
  if (ctx && ctx->rec) {
    Recorder* r = (Recorder*)ctx->rec;
    r->phase += 1;
    r->sub = 0;
  }
}

// Launch (or record) a kernel fn(A a, const A* grp, const int4* bmap) as a plain
// launch with grid `grid`; fn_group is the same kernel's grouped variant, which a
// batch plan uses when it merges this launch with other instances'.  The grid
// is stored in a.gx/gy/gz first.  Start and stop events (may be null) are
// recorded by the dispatch itself.
template <typename A>
hipError_t launch_kernel(dctk_ctx ctx, hipStream_t s, void (*fn)(A, const A*, const int4*),
                         void (*fn_group)(A, const A*, const int4*), dim3 grid, unsigned threads, unsigned shmem, A a,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  a.gx = (int)grid.x;
  a.gy = (int)grid.y;
  a.gz = (int)grid.z;
  if (ctx && ctx->rec) {
    Recorder* r = (Recorder*)ctx->rec;
    LaunchRec lr;
    lr.fn = (const void*)fn;
    lr.fn_group = (const void*)fn_group;
    lr.grid = grid;
    lr.threads = threads;
    lr.shmem = shmem;
    lr.phase = r->phase;
    lr.sub = r->sub++;
    lr.args.resize(sizeof(A));
    memcpy(lr.args.data(), &a, sizeof(A));
    r->recs.push_back(std::move(lr));
    return hipSuccess;
  }
  const A* grp = nullptr;
  const int4* bmap = nullptr;
  void* kargs[3] = {&a, &grp, &bmap};
  hipError_t e = hipExtLaunchKernel((const void*)fn, grid, dim3(threads), kargs, shmem, s, e0, e1, 0);
  return e != hipSuccess ? e : hipGetLastError();
}
// Launchers of kernels that cannot be recorded refuse while planning.
inline bool recording(dctk_ctx ctx) { return ctx && ctx->rec; }

// transform matrices (host, FP64): which = DCTK_MAT_*
int build_tube_matrix(int tube, int which, int64_t p, double* out);
size_t elem_size(int dt);
void set_num_cus(int n);
int num_cus();

// ---- product kernels ---------------------------------------------------------
// Streaming tube transform: out[k][e] = a * sum_t G[k][t] (s * in[t][e]) + b * src[k][e].
// `xnorm` (may be null) receives s * in.  Scalars come from the control block;
// ctl.part_out gets per-block sums of out^2.
hipError_t launch_tube(dctk_ctx ctx, hipStream_t st, int in_dtype, int out_dtype, int64_t p, int64_t count,
                       const void* in, void* out, const double* Gd, const float* Gf,
                       const void* src, void* xnorm, const Ctl& ctl, bool scale, bool epi, int* nblocks_out);

// Inverse transform of one product with its epilogue, y = a (G1 c) + b src (a scaled
// by the control block's input scale; partials of y^2 in ctl.part_out), paired with
// the next product's forward transform x = G1^T y in x_dtype (FP32 vectors, 16 <= p <= 64).
// G1 is L^{-1} after a forward product (then G1^T = L^{-T}), L^T after an adjoint (G1^T = L).
bool tube_pair_ok(int64_t p, int vec_dtype);
hipError_t launch_tube_pair(dctk_ctx ctx, hipStream_t s, int x_dtype, int64_t p, int64_t count, const float* c,
                            const float* src, float* y, void* x, const float* G1, const Ctl& ctl,
                            int* nblocks_out);

// C_k = op(A_k) op(B_k), batched over `batch`; tile 0: by problem size, else 32/64/128
hipError_t launch_gemm(dctk_ctx ctx, hipStream_t s, int in_dtype, int out_acc, int M, int N, int K,
                       const void* A, int64_t lda, int64_t sA, int ta,
                       const void* B, int64_t ldb, int64_t sB, int tb,
                       void* C, int64_t ldc, int64_t sC, int batch, Gate g, int tile = 0);

// Whether an operator can take the fused product, and whether it does in a direction.
bool fused_eligible(dctk_op op);
bool use_fused(dctk_op op, int adjoint);

// Fused c-product for one-sided operators with p <= kFusedMaxP.
hipError_t launch_fused(dctk_op op, hipStream_t s, int adjoint, const void* X, void* Y, const void* src,
                        void* xnorm, const Ctl& ctl, int* nblocks_out);

// The c-product / adjoint under a control block: Y = a*M(s X) + b*src; xnorm gets s X.
// Writes the number of partials produced to *nblocks_out (when ctl.part_out).
hipError_t apply_op(dctk_op op, hipStream_t s, int adjoint, const void* X, void* Y, const void* src,
                    void* xnorm, const Ctl& ctl, int* nblocks_out);

// Golub-Kahan steps with paired transforms (three-kernel products, FP32 vectors,
// 16 <= p <= 64): pair_eligible says whether op takes them; pair_first enqueues
// a product's forward transform (input X, scale from ctl) and its slice GEMMs;
// pair_gemm the slice GEMMs of a product whose transformed input is already in
// place; pair_transforms the product's inverse transform with its epilogue
// (Y = a M(.) + b src under ctl, partials of Y^2) paired with the forward
// transform of the next product (the other direction), whose input is Y.
bool pair_eligible(dctk_op op);
hipError_t pair_first(dctk_op op, hipStream_t s, int adjoint, const void* X, const Ctl& ctl);
hipError_t pair_gemm(dctk_op op, hipStream_t s, int adjoint, const Ctl& ctl);
hipError_t pair_transforms(dctk_op op, hipStream_t s, int adjoint, const void* src, void* Y, const Ctl& ctl,
                           int* nblocks_out);

// ---- streaming vector kernels (vec.hip) ------------------------------------
// partials of sum(x . z) (z null: x . x)
hipError_t launch_sumsq(dctk_ctx ctx, int dtype, int64_t n, const void* x, const void* z, double* part,
                        int* nblocks, Gate g);
// out = x + c*y with c = csign * cptr[0]; partials of out^2 (part may be null)
hipError_t launch_axpy_sumsq(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* x, const void* y,
                             const double* cptr, double csign, double* part, int* nblocks, Gate g);
// partials of <basis_i, w>, i < nb, laid out part[i * nblocks + block]
hipError_t launch_multidot(dctk_ctx ctx, int dtype, int64_t n, const void* basis, int64_t stride, int nb,
                           const void* w, double* part, int* nblocks, Gate g);
// one block: coef[i] = sum_b part[i*nblocks + b]; dst[i*dst_stride] += coef[i] when dst
hipError_t launch_coef_finalize(dctk_ctx ctx, const double* part, int nblocks, int nb, double* coef,
                                double* dst, int dst_stride, Gate g);
// w -= sum_i coef[i] basis_i
hipError_t launch_subtract(dctk_ctx ctx, int dtype, int64_t n, void* w, const void* basis, int64_t stride,
                           int nb, const double* coef, Gate g);
// out = (x0 ? x0 : 0) + sum_{i < min(nb, *nptr)} c_i basis_i with c_i = y[i], or y[i] / div[i] where bit i
// of `mask` is set (a basis vector stored unnormalised)
hipError_t launch_combine(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* x0, const void* basis,
                          int64_t stride, int nb, const int* nptr, const double* y, Gate g,
                          unsigned long long mask = 0, const double* div = nullptr);
// GMRES cycle start: beta = sqrt(sum part) -> st->beta0 (halt on 0); out = in / beta
hipError_t launch_arn_start(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* in, const double* part,
                            int npart, KState* st);
// Arnoldi MGS pass i of step j: when part_in, h = sum part_in is recorded at hdst and
// w -= h * vprev; then partials of <vi, w> (vi null: |w|^2) into part_out
hipError_t launch_mgs(dctk_ctx ctx, int dtype, int64_t n, void* w, const void* vprev, const void* vi,
                      const double* part_in, int npart_in, double* hdst, double* part_out, int* nblocks,
                      KState* st, int j);
// Arnoldi: record h_{j+1,j} = sqrt(sum part) with the breakdown test (one block)
hipError_t launch_arn_finish(dctk_ctx ctx, const double* part, int npart, KState* st, int j);
// GMRES: ||C - M(X)|| = sqrt(sum part) with the convergence test (one block)
hipError_t launch_gmres_res(dctk_ctx ctx, const double* part, int npart, KState* st);
// GKB start (Algorithm 6 step 2) and the per-step update (Algorithm 6 (c)-(g))
hipError_t launch_gkb_start(dctk_ctx ctx, int dtype, int64_t n, void* X, void* W, void* V1, const double* part,
                            int npart, KState* st);
// (U, if given: beta_{j+1} U_{j+1} normalised in place by the recorded beta_{j+1})
hipError_t launch_gkb_update(dctk_ctx ctx, int dtype, int64_t n, void* X, void* W, const void* Vin, void* Vn,
                             const double* part, int npart, KState* st, int j, void* U = nullptr);
hipError_t launch_state_reset(dctk_ctx ctx, KState* st, int full, double tol);
hipError_t launch_cast(dctk_ctx ctx, int64_t n, const double* in, int out_dtype, void* out);
// Transposing cast of p slices rows x cols (FP64) to cols x rows (FP32 and 16-bit types).
hipError_t launch_cast_t(dctk_ctx ctx, int64_t p, int64_t rows, int64_t cols, const double* in, int out_dtype,
                         void* out);

// ---- solves (api.hip) ------------------------------------------------------------
int check_solve_opts(const dctk_solve_opts* o, const dctk_krylov ws);
// everything dctk_lsqr_tik_solve enqueues, and its info once finished (synchronises)
hipError_t lsqr_enqueue(dctk_ctx ctx, dctk_krylov ws, const void* C, void* X, const dctk_solve_opts* opts);
int lsqr_info(dctk_ctx ctx, dctk_krylov ws, const dctk_solve_opts* opts, dctk_solve_info* info);

// projected FP64 problem (projected.hip): bidiag = 1 reads alpha/beta, else H.
// Writes st->y[0..k), st->lambda, st->gcv.
// k_use > 0 projects at min(k_use, steps); lam_cand > 0 (with GCV) is kept when its GCV
// value is <= gate * the minimum (st->gate_ok records the decision).
hipError_t launch_projected(dctk_ctx ctx, KState* st, int bidiag, int gcv_mode, double lambda, int k_use = 0,
                            double lam_cand = -1.0, double gate = 1.0, int cand_from_state = 0);
// device-side learned stop: st->k_limit and st->pred_lambda from the network (after step 8)
hipError_t launch_mlp_stop(dctk_ctx ctx, dctk_mlp m, KState* st, int kmin, int kmax);
// DC-GK with the device-side learned stop, fully asynchronous (recordable)
hipError_t learned_enqueue(dctk_ctx ctx, dctk_krylov ws, dctk_mlp m, const void* C, void* X,
                           const dctk_solve_opts* opts, double gate);

// learned stop (mlp.hip): features of st -> network -> host pred[5] =
// {t_lambda, t_k, lambda, k, valid}; synchronises
hipError_t mlp_predict(dctk_ctx ctx, dctk_mlp m, const KState* st, int kmin, int kmax, float* host_pred);

}  // namespace dctk
