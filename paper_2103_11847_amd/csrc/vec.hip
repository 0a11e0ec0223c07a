// Global inner products, Frobenius norms, axpys and basis combinations of the
// Krylov methods (Sec. 2.2 inner product; Algorithms 2, 4 and 6; the
// combination V (*) y of eq. ev1), as streaming kernels.
//
// Reductions are deterministic and need no fences: a reducing kernel writes
// one FP64 partial per block; the kernel that needs the value (the next one
// in stream order, after the kernel boundary has made the partials visible)
// sums them in block order in every block, so all blocks hold the same bits.
// Block 0 records the scalar in the device state (indexed by step).
#include <cfloat>
#include <cmath>

#include "internal.h"

namespace dctk {

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

__device__ inline bool first_thread() { return blockIdx.x == 0 && threadIdx.x == 0; }
__device__ inline bool first_thread(const VBlock& vb) { return vb.x == 0 && threadIdx.x == 0; }

#define DCTK_GRID_LOOP(e, n) \
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < (n); e += (int64_t)gridDim.x * blockDim.x * 4)
// the same over an instance's own 1-D grid (plain or grouped launch)
#define DCTK_VGRID_LOOP(e, n, vb, gx) \
  for (int64_t e = ((int64_t)(vb).x * blockDim.x + threadIdx.x) * 4; e < (n); e += (int64_t)(gx) * blockDim.x * 4)

// argument structs of the kernels that run in grouped launches
struct SumsqArgs {
  int gx, gy, gz;
  int vec;
  int64_t n;
  const void* x;
  const void* z;
  double* part;
  Gate g;
};
struct GkbArgs {  // start and per-step update of Algorithm 6
  int gx, gy, gz;
  int vec;
  int64_t n;
  void* X;          // LSQR iterate (null: not formed)
  void* W;          // LSQR search direction (null with X)
  void* V;          // the new basis vector (written)
  const void* Vin;  // its unnormalised input (update; null: V itself)
  void* U;          // update: beta_{j+1} U_{j+1}, normalised in place (null: none)
  const double* part;
  int npart;
  int j;
  KState* st;
};
struct CombineArgs {
  int gx, gy, gz;
  int vec;
  int64_t n;
  void* out;
  const void* x0;
  const void* basis;
  int64_t bstride;
  int nb;
  const int* nptr;
  const double* y;
  Gate g;
  unsigned long long mask;  // bit i: basis_i stored unnormalised, coefficient y[i] / div[i]
  const double* div;
};
struct GramArgs {  // reorthogonalisation passes: multi-dot, coefficient sums, subtraction
  int gx, gy, gz;
  int vec;
  int64_t n;
  const void* basis;
  int64_t bstride;
  int nb;
  int nblocks;       // coefficient sums: partials per coefficient
  void* w;
  double* part;
  double* coef;
  double* dst;       // coefficient sums: optional accumulation target (Arnoldi column)
  int dst_stride;
  Gate g;
};
struct ResetArgs {
  int gx, gy, gz;
  int full;
  KState* st;
  double tol;
};

// ---- reductions ----------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void k_sumsq_body(const SumsqArgs& a, const VBlock vb, const bool grouped) {
  if (!gate_open(a.g)) return;
  const int64_t n = a.n;
  const T* x = (const T*)a.x;
  const T* z = (const T*)a.z;
  const bool vec = a.vec;
  __shared__ double sh[kShCtl];
  double acc = 0.0;
  DCTK_VGRID_LOOP(e, n, vb, a.gx) {
    double xv[4];
    ld4(x, e, n, vec, xv);
    if (z) {
      double zv[4];
      ld4(z, e, n, vec, zv);
      for (int i = 0; i < 4; ++i) acc += xv[i] * zv[i];
    } else {
      for (int i = 0; i < 4; ++i) acc += xv[i] * xv[i];
    }
  }
  const double t = block_sum_all(acc, sh);
  if (threadIdx.x == 0) a.part[vb.x] = t;
}

template <typename T, bool GROUPED>
__global__ __launch_bounds__(kThreads) void k_sumsq(SumsqArgs a_, const SumsqArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_sumsq_body<T>(a_, hw_block(), false);
  } else {
    VBlock vb;
    const SumsqArgs g = group_args(grp, bmap, vb);
    k_sumsq_body<T>(g, vb, true);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_axpy_sumsq(int64_t n, T* out, const T* x, const T* y,
                                                         const double* cptr, double csign, double* part, bool vec,
                                                         Gate g) {
  if (!gate_open(g)) return;
  __shared__ double sh[kShCtl];
  const double c = csign * cptr[0];
  double acc = 0.0;
  DCTK_GRID_LOOP(e, n) {
    double xv[4], yv[4];
    ld4(x, e, n, vec, xv);
    ld4(y, e, n, vec, yv);
    for (int i = 0; i < 4; ++i) xv[i] = (double)(T)(xv[i] + c * yv[i]);
    st4(out, e, n, vec, xv);
    for (int i = 0; i < 4; ++i) acc += xv[i] * xv[i];
  }
  if (part) {
    const double t = block_sum_all(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

// partials of <basis_i, w> for i < nb: part[i * gridDim.x + block]
template <typename T>
__device__ __forceinline__ void k_multidot_body(const GramArgs& a, const VBlock vb, const bool grouped) {
  if (!gate_open(a.g)) return;
  const int64_t n = a.n, bstride = a.bstride;
  const T* basis = (const T*)a.basis;
  const T* w = (const T*)a.w;
  const int nb = a.nb;
  const bool vec = a.vec;
  __shared__ double sh[kShCtl];
  for (int i0 = 0; i0 < nb; i0 += 8) {
    double acc[8];
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    DCTK_VGRID_LOOP(e, n, vb, a.gx) {
      double wv[4];
      ld4(w, e, n, vec, wv);
      for (int u = 0; u < 8 && i0 + u < nb; ++u) {
        double bv[4];
        ld4(basis + (int64_t)(i0 + u) * bstride, e, n, vec, bv);
        acc[u] += bv[0] * wv[0] + bv[1] * wv[1] + bv[2] * wv[2] + bv[3] * wv[3];
      }
    }
    for (int u = 0; u < 8 && i0 + u < nb; ++u) {
      const double t = block_sum_all(acc[u], sh);
      if (threadIdx.x == 0) a.part[(int64_t)(i0 + u) * a.gx + vb.x] = t;
    }
  }
}

template <typename T, bool GROUPED>
__global__ __launch_bounds__(kThreads) void k_multidot(GramArgs a_, const GramArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_multidot_body<T>(a_, hw_block(), false);
  } else {
    VBlock vb;
    const GramArgs g = group_args(grp, bmap, vb);
    k_multidot_body<T>(g, vb, true);
  }
}

// one block: coef[i] = sum_b part[i * nblocks + b]; dst[i * dst_stride] += coef[i]
__device__ __forceinline__ void k_coef_finalize_body(const GramArgs& a, const VBlock vb, const bool grouped) {
  if (!gate_open(a.g)) return;
  const double* part = a.part;
  const int nblocks = a.nblocks, nb = a.nb, dst_stride = a.dst_stride;
  double* coef = a.coef;
  double* dst = a.dst;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = wid; i < nb; i += (int)(blockDim.x >> 6)) {
    double v = 0.0;
    for (int b = lane; b < nblocks; b += 64) v += part[(int64_t)i * nblocks + b];
    v = wave_sum(v);
    if (lane == 0) {
      coef[i] = v;
      if (dst) dst[i * dst_stride] += v;
    }
  }
}

template <bool GROUPED>
__global__ __launch_bounds__(kThreads) void k_coef_finalize(GramArgs a_, const GramArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_coef_finalize_body(a_, hw_block(), false);
  } else {
    VBlock vb;
    const GramArgs g = group_args(grp, bmap, vb);
    k_coef_finalize_body(g, vb, true);
  }
}

// w -= sum_i coef[i] basis_i
template <typename T>
__device__ __forceinline__ void k_subtract_body(const GramArgs& a, const VBlock vb, const bool grouped) {
  if (!gate_open(a.g)) return;
  const int64_t n = a.n, bstride = a.bstride;
  T* w = (T*)a.w;
  const T* basis = (const T*)a.basis;
  const int nb = a.nb;
  const bool vec = a.vec;
  __shared__ double sc[kRedVals];
  for (int i = threadIdx.x; i < nb; i += blockDim.x) sc[i] = a.coef[i];
  __syncthreads();
  DCTK_VGRID_LOOP(e, n, vb, a.gx) {
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

template <typename T, bool GROUPED>
__global__ __launch_bounds__(kThreads) void k_subtract(GramArgs a_, const GramArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_subtract_body<T>(a_, hw_block(), false);
  } else {
    VBlock vb;
    const GramArgs g = group_args(grp, bmap, vb);
    k_subtract_body<T>(g, vb, true);
  }
}

// out = x0 + sum_{i < cnt} y[i] basis_i
template <typename T>
__device__ __forceinline__ void k_combine_body(const CombineArgs& a, const VBlock vb, const bool grouped) {
  if (!gate_open(a.g)) return;
  const int64_t n = a.n, bstride = a.bstride;
  T* out = (T*)a.out;
  const T* x0 = (const T*)a.x0;
  const T* basis = (const T*)a.basis;
  const int nb = a.nb;
  const double* y = a.y;
  const bool vec = a.vec;
  __shared__ double sy[kRedVals];
  int cnt = a.nptr ? a.nptr[0] : nb;
  if (cnt > nb) cnt = nb;
  if (cnt < 0) cnt = 0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x)
    sy[i] = (i < 64 && ((a.mask >> i) & 1ull)) ? y[i] / a.div[i] : y[i];
  __syncthreads();
  if (vec) {
    // 16-byte rows (n a multiple of 4): eight basis rows in flight per thread,
    // loaded unconditionally from clamped indices, summed in basis order
    constexpr int U = 8;
    DCTK_VGRID_LOOP(e, n, vb, a.gx) {
      double o[4] = {0.0, 0.0, 0.0, 0.0};
      if (x0) V4<T>::ld(x0 + e, o);
      for (int i0 = 0; i0 < cnt; i0 += U) {
        double bv[U][4];
#pragma unroll
        for (int j = 0; j < U; ++j) V4<T>::ld(basis + (int64_t)min(i0 + j, cnt - 1) * bstride + e, bv[j]);
#pragma unroll
        for (int j = 0; j < U; ++j) {
          if (i0 + j < cnt) {
#pragma unroll
            for (int u = 0; u < 4; ++u) o[u] += sy[i0 + j] * bv[j][u];
          }
        }
      }
      V4<T>::st(out + e, o);
    }
    return;
  }
  DCTK_VGRID_LOOP(e, n, vb, a.gx) {
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

template <typename T, bool GROUPED>
__global__ __launch_bounds__(kThreads) void k_combine(CombineArgs a_, const CombineArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_combine_body<T>(a_, hw_block(), false);
  } else {
    VBlock vb;
    const CombineArgs g = group_args(grp, bmap, vb);
    k_combine_body<T>(g, vb, true);
  }
}

// ---- Golub-Kahan / LSQR ----------------------------------------------------------
// Algorithm 6 step 2 after M*(U_1): alpha_1 from the partials; V_1 = V~/alpha_1
// in place; W_1 = V_1; X_0 = 0.
template <typename T>
__device__ __forceinline__ void k_gkb_start_body(const GkbArgs& a, const VBlock vb, const bool grouped) {
  const int64_t n = a.n;
  T* X = (T*)a.X;
  T* W = (T*)a.W;
  T* V1 = (T*)a.V;
  const double* part = a.part;
  const int npart = a.npart;
  KState* st = a.st;
  const bool vec = a.vec;
  __shared__ double sh[kShCtl];
  // the partials and beta_1 are loaded before the stop flag: one memory latency
  const double ps = part_local(part, npart);
  const double b1 = st->beta[0];
  const bool ok = ld_state(&st->stop_step) < 0;
  bool brk = true;
  double alpha = 0.0;
  if (ok) {
    alpha = sqrt(block_sum_all(ps, sh));
    const double scale = fmax(b1, alpha);
    const bool fin = isfinite(alpha);
    brk = !fin || alpha <= kBreakFactor * DBL_EPSILON * scale;
    if (first_thread(vb)) {
      st->alpha[0] = alpha;
      st->rhobar[0] = alpha;
      st->phibar[0] = b1;
      if (brk) {
        st->stop_step = 0;
        st->stop_kind = STOP_ALPHA;
        st->status = fin ? DCTK_BREAKDOWN : DCTK_ENONFINITE;
      }
    }
  }
  const double ia = brk ? 0.0 : 1.0 / alpha;
  DCTK_VGRID_LOOP(e, n, vb, a.gx) {
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    if (X) st4(X, e, n, vec, z);
    if (!brk) {
      double v[4];
      ld4(V1, e, n, vec, v);
      for (int u = 0; u < 4; ++u) v[u] = (double)(T)(v[u] * ia);
      st4(V1, e, n, vec, v);
      if (W) st4(W, e, n, vec, v);
    } else if (W) {
      st4(W, e, n, vec, z);
    }
  }
}

template <typename T, bool GROUPED>
__global__ __launch_bounds__(kThreads) void k_gkb_start(GkbArgs a_, const GkbArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_gkb_start_body<T>(a_, hw_block(), false);
  } else {
    VBlock vb;
    const GkbArgs g = group_args(grp, bmap, vb);
    k_gkb_start_body<T>(g, vb, true);
  }
}

// Algorithm 4 (e)-(f) and Algorithm 6 (c)-(g) for step j: alpha_{j+1} from the
// partials of V~ (unless beta_{j+1} broke down), the plane rotation, then
// V_{j+1} = V~/alpha_{j+1} in place, X_j = X_{j-1} + (phi_j/rho_j) W_j,
// W_{j+1} = V_{j+1} - (theta_{j+1}/rho_j) W_j.
template <typename T>
__device__ __forceinline__ void k_gkb_update_body(const GkbArgs& a, const VBlock vb, const bool grouped) {
  const int64_t n = a.n;
  T* X = (T*)a.X;
  T* W = (T*)a.W;
  T* Vn = (T*)a.V;
  const T* Vi = a.Vin ? (const T*)a.Vin : Vn;
  const double* part = a.part;
  const int npart = a.npart, j = a.j;
  KState* st = a.st;
  const bool vec = a.vec;
  __shared__ double sh[kShCtl];
  // Every load of the prologue (recorded scalars, breakdown scale, partials,
  // stop flags) is issued before the first use, none inside a branch: one
  // memory latency.
  const double bnext = st->beta[j];
  const double rhob = st->rhobar[j - 1], phib = st->phibar[j - 1];
  const double tol = st->tol;
  const double pm = gkb_scale_local(st, j, j + 1);
  double ps = part_first(part, npart);
  // (the stop flags last: moved to scalar registers, they are waited for at once)
  const int ss = ld_state(&st->stop_step);
  const int skind = ld_state(&st->stop_kind);
  const int kl = ld_state(&st->k_limit);
  if ((ss >= 0 && ss < j) || (kl > 0 && j > kl)) return;
  ps = part_rest(ps, part, npart);
  const GkbUpd u = gkb_update_scalars(st, j, ps, pm, bnext, rhob, phib, tol, ss, skind, sh, first_thread(vb));
  const double cx = u.cx, cw = u.cw;
  const bool have_v = u.have_v;
  const double ia = have_v ? 1.0 / u.alpha : 0.0;
  T* Un = (T*)a.U;
  // U_{j+1} exists unless beta_{j+1} broke down (then it is never used)
  const bool have_u = Un != nullptr && !(ss == j && skind == STOP_BETA) && bnext > 0.0;
  const double ib = have_u ? 1.0 / bnext : 0.0;
  DCTK_VGRID_LOOP(e, n, vb, a.gx) {
    double xv[4], wv[4], vv[4];
    if (have_u) {
      double uv[4];
      ld4(Un, e, n, vec, uv);
      for (int q = 0; q < 4; ++q) uv[q] = (double)(T)(uv[q] * ib);
      st4(Un, e, n, vec, uv);
    }
    if (X) {
      ld4(X, e, n, vec, xv);
      ld4(W, e, n, vec, wv);
      for (int q = 0; q < 4; ++q) xv[q] += cx * wv[q];
      st4(X, e, n, vec, xv);
    }
    if (have_v) {
      ld4(Vi, e, n, vec, vv);
      for (int q = 0; q < 4; ++q) vv[q] = (double)(T)(vv[q] * ia);
      st4(Vn, e, n, vec, vv);
      if (X) {
        for (int q = 0; q < 4; ++q) wv[q] = vv[q] - cw * wv[q];
        st4(W, e, n, vec, wv);
      }
    }
  }
}

template <typename T, bool GROUPED>
__global__ __launch_bounds__(kThreads) void k_gkb_update(GkbArgs a_, const GkbArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_gkb_update_body<T>(a_, hw_block(), false);
  } else {
    VBlock vb;
    const GkbArgs g = group_args(grp, bmap, vb);
    k_gkb_update_body<T>(g, vb, true);
  }
}

// ---- Arnoldi / GMRES -----------------------------------------------------------
// cycle start: beta = ||R|| from the partials; V_1 = R / beta
template <typename T>
__global__ __launch_bounds__(kThreads) void k_arn_start(int64_t n, T* out, const T* in, const double* part, int npart,
                                                        KState* st, bool vec) {
  if (ld_state(&st->halt)) return;
  __shared__ double sh[kShCtl];
  const double beta = sqrt(block_sum_partials(part, npart, sh));
  const bool fin = isfinite(beta);
  const bool ok = fin && beta > 0.0;
  if (first_thread()) {
    st->beta0 = beta;
    st->steps = 0;
    if (!ok) {
      st->halt = 1;
      if (!fin) st->status = DCTK_ENONFINITE;
    }
  }
  if (!ok) return;
  const double ib = 1.0 / beta;
  DCTK_GRID_LOOP(e, n) {
    double v[4];
    ld4(in, e, n, vec, v);
    for (int u = 0; u < 4; ++u) v[u] *= ib;
    st4(out, e, n, vec, v);
  }
}

// One modified Gram-Schmidt pass of Algorithm 2 step 3(b) for step j: when
// part_in is given, h = sum(part_in) is recorded at hdst and w -= h vprev;
// then the partials of <vi, w> (vi null: of <w, w>) go to part_out.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mgs(int64_t n, T* w, const T* vprev, const T* vi, const double* part_in,
                                                  int npart_in, double* hdst, double* part_out, bool vec, Gate g) {
  if (!gate_open(g)) return;
  __shared__ double sh[kShCtl];
  double h = 0.0;
  if (part_in) {
    h = block_sum_partials(part_in, npart_in, sh);
    if (first_thread()) hdst[0] = h;
  }
  double acc = 0.0;
  DCTK_GRID_LOOP(e, n) {
    double wv[4];
    ld4(w, e, n, vec, wv);
    if (part_in) {
      double pv[4];
      ld4(vprev, e, n, vec, pv);
      for (int u = 0; u < 4; ++u) wv[u] = (double)(T)(wv[u] - h * pv[u]);
      st4(w, e, n, vec, wv);
    }
    if (vi) {
      double v[4];
      ld4(vi, e, n, vec, v);
      for (int u = 0; u < 4; ++u) acc += v[u] * wv[u];
    } else {
      for (int u = 0; u < 4; ++u) acc += wv[u] * wv[u];
    }
  }
  const double t = block_sum_all(acc, sh);
  if (threadIdx.x == 0) part_out[blockIdx.x] = t;
}

// one block: h_{j,j-1} from the partials (breakdown test) -- the prologue of the
// next Arnoldi product, for the last step of a cycle
__global__ __launch_bounds__(kThreads) void k_arn_finish(Ctl c) {
  __shared__ double sh[kShCtl];
  double a, b, s;
  (void)ctl_begin(c, a, b, s, sh, hw_block());
}

// one block: ||C - M(X)|| from the partials; cycle bookkeeping; convergence
__global__ __launch_bounds__(kThreads) void k_gmres_res(const double* part, int npart, KState* st) {
  if (ld_state(&st->halt)) return;
  __shared__ double sh[kShCtl];
  const double r = sqrt(block_sum_partials(part, npart, sh));
  if (threadIdx.x == 0) {
    st->resnorm = r;
    st->cycles += 1;
    st->total_steps += st->steps;
    if (!isfinite(r)) {
      st->status = DCTK_ENONFINITE;
      st->halt = 1;
    } else if (r < st->tol) {
      st->converged = 1;
      st->halt = 1;
    }
  }
}

template <typename TO>
__global__ __launch_bounds__(kThreads) void k_cast(int64_t n, const double* in, TO* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) out[e] = cvt<TO, double>(in[e]);
}

// out[k][c][r] = in[k][r][c] for p slices of rows x cols (operator setup only)
template <typename TO>
__global__ __launch_bounds__(kThreads) void k_cast_t(int64_t p, int64_t rows, int64_t cols, const double* in, TO* out) {
  const int64_t n = p * rows * cols, rc = rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const int64_t k = e / rc, rem = e - k * rc;
    const int64_t c = rem / rows, r = rem - c * rows;
    out[e] = cvt<TO, double>(in[k * rc + r * cols + c]);
  }
}

// full = 1: clear everything (new solve); full = 0: start a new GMRES cycle (unless halted)
__device__ __forceinline__ void k_state_reset_body(const ResetArgs& a, const VBlock vb, const bool grouped) {
  KState* st = a.st;
  const int full = a.full;
  const double tol = a.tol;
  if (full == 0 && ld_state(&st->halt)) return;
  if (full) {
    double* d = reinterpret_cast<double*>(st);
    const int nd = (int)(sizeof(KState) / sizeof(double));
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
    }
  }
}

template <bool GROUPED>
__global__ void k_state_reset(ResetArgs a_, const ResetArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_state_reset_body(a_, hw_block(), false);
  } else {
    VBlock vb;
    const ResetArgs g = group_args(grp, bmap, vb);
    k_state_reset_body(g, vb, true);
  }
}

// ---- launchers ---------------------------------------------------------------
static inline unsigned grid_for(int64_t n) {
  int64_t b = ((n + 3) / 4 + kThreads - 1) / kThreads;
  if (b > kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (unsigned)b;
}
static inline bool al(const void* p) { return p == nullptr || ((uintptr_t)p % 32) == 0; }

hipError_t launch_sumsq(dctk_ctx ctx, int dtype, int64_t n, const void* x, const void* z, double* part, int* nblocks,
                        Gate g) {
  const unsigned grid = grid_for(n);
  if (nblocks) *nblocks = (int)grid;
  SumsqArgs a{};
  a.vec = (n % 4 == 0) && al(x) && al(z);
  a.n = n;
  a.x = x;
  a.z = z;
  a.part = part;
  a.g = g;
  if (dtype == DCTK_F64) return launch_kernel(ctx, ctx->stream, k_sumsq<double, false>, k_sumsq<double, true>, dim3(grid), kThreads, 0, a);
  return launch_kernel(ctx, ctx->stream, k_sumsq<float, false>, k_sumsq<float, true>, dim3(grid), kThreads, 0, a);
}

hipError_t launch_axpy_sumsq(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* x, const void* y,
                             const double* cptr, double csign, double* part, int* nblocks, Gate g) {
  if (recording(ctx)) return hipErrorNotSupported;
  const unsigned grid = grid_for(n);
  if (nblocks) *nblocks = (int)grid;
  const bool vec = (n % 4 == 0) && al(out) && al(x) && al(y);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_axpy_sumsq<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)out,
                       (const double*)x, (const double*)y, cptr, csign, part, vec, g);
  else
    hipLaunchKernelGGL(k_axpy_sumsq<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)out,
                       (const float*)x, (const float*)y, cptr, csign, part, vec, g);
  return hipGetLastError();
}

hipError_t launch_multidot(dctk_ctx ctx, int dtype, int64_t n, const void* basis, int64_t stride, int nb,
                           const void* w, double* part, int* nblocks, Gate g) {
  const unsigned grid = grid_for(n);
  if (nblocks) *nblocks = (int)grid;
  if (nb <= 0) return hipSuccess;
  GramArgs a{};
  a.vec = (n % 4 == 0) && (stride % 4 == 0) && al(basis) && al(w);
  a.n = n;
  a.basis = basis;
  a.bstride = stride;
  a.nb = nb;
  a.w = const_cast<void*>(w);
  a.part = part;
  a.g = g;
  if (dtype == DCTK_F64) return launch_kernel(ctx, ctx->stream, k_multidot<double, false>, k_multidot<double, true>, dim3(grid), kThreads, 0, a);
  return launch_kernel(ctx, ctx->stream, k_multidot<float, false>, k_multidot<float, true>, dim3(grid), kThreads, 0, a);
}

hipError_t launch_coef_finalize(dctk_ctx ctx, const double* part, int nblocks, int nb, double* coef, double* dst,
                                int dst_stride, Gate g) {
  if (nb <= 0) return hipSuccess;
  GramArgs a{};
  a.part = const_cast<double*>(part);
  a.nblocks = nblocks;
  a.nb = nb;
  a.coef = coef;
  a.dst = dst;
  a.dst_stride = dst_stride;
  a.g = g;
  return launch_kernel(ctx, ctx->stream, k_coef_finalize<false>, k_coef_finalize<true>, dim3(1), kThreads, 0, a);
}

hipError_t launch_subtract(dctk_ctx ctx, int dtype, int64_t n, void* w, const void* basis, int64_t stride, int nb,
                           const double* coef, Gate g) {
  if (nb <= 0) return hipSuccess;
  const unsigned grid = grid_for(n);
  GramArgs a{};
  a.vec = (n % 4 == 0) && (stride % 4 == 0) && al(basis) && al(w);
  a.n = n;
  a.w = w;
  a.basis = basis;
  a.bstride = stride;
  a.nb = nb;
  a.coef = const_cast<double*>(coef);
  a.g = g;
  if (dtype == DCTK_F64) return launch_kernel(ctx, ctx->stream, k_subtract<double, false>, k_subtract<double, true>, dim3(grid), kThreads, 0, a);
  return launch_kernel(ctx, ctx->stream, k_subtract<float, false>, k_subtract<float, true>, dim3(grid), kThreads, 0, a);
}

hipError_t launch_combine(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* x0, const void* basis,
                          int64_t stride, int nb, const int* nptr, const double* y, Gate g,
                          unsigned long long mask, const double* div) {
  const unsigned grid = grid_for(n);
  CombineArgs a{};
  a.mask = div != nullptr ? mask : 0ull;
  a.div = div;
  a.vec = (n % 4 == 0) && (stride % 4 == 0) && al(out) && al(x0) && al(basis);
  a.n = n;
  a.out = out;
  a.x0 = x0;
  a.basis = basis;
  a.bstride = stride;
  a.nb = nb;
  a.nptr = nptr;
  a.y = y;
  a.g = g;
  if (dtype == DCTK_F64) return launch_kernel(ctx, ctx->stream, k_combine<double, false>, k_combine<double, true>, dim3(grid), kThreads, 0, a);
  return launch_kernel(ctx, ctx->stream, k_combine<float, false>, k_combine<float, true>, dim3(grid), kThreads, 0, a);
}

hipError_t launch_arn_start(dctk_ctx ctx, int dtype, int64_t n, void* out, const void* in, const double* part,
                            int npart, KState* st) {
  if (recording(ctx)) return hipErrorNotSupported;
  const unsigned grid = grid_for(n);
  const bool vec = (n % 4 == 0) && al(out) && al(in);
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_arn_start<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)out,
                       (const double*)in, part, npart, st, vec);
  else
    hipLaunchKernelGGL(k_arn_start<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)out,
                       (const float*)in, part, npart, st, vec);
  return hipGetLastError();
}

hipError_t launch_mgs(dctk_ctx ctx, int dtype, int64_t n, void* w, const void* vprev, const void* vi,
                      const double* part_in, int npart_in, double* hdst, double* part_out, int* nblocks, KState* st,
                      int j) {
  if (recording(ctx)) return hipErrorNotSupported;
  const unsigned grid = grid_for(n);
  if (nblocks) *nblocks = (int)grid;
  const bool vec = (n % 4 == 0) && al(w) && al(vprev) && al(vi);
  const Gate g{st, j - 1, 1};  // runs when the product of step j ran
  if (dtype == DCTK_F64)
    hipLaunchKernelGGL(k_mgs<double>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (double*)w,
                       (const double*)vprev, (const double*)vi, part_in, npart_in, hdst, part_out, vec, g);
  else
    hipLaunchKernelGGL(k_mgs<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, n, (float*)w,
                       (const float*)vprev, (const float*)vi, part_in, npart_in, hdst, part_out, vec, g);
  return hipGetLastError();
}

hipError_t launch_arn_finish(dctk_ctx ctx, const double* part, int npart, KState* st, int j) {
  if (recording(ctx)) return hipErrorNotSupported;
  Ctl c{};
  c.kind = CTL_ARN_FWD;
  c.j = j;
  c.st = st;
  c.part_in = part;
  c.npart_in = npart;
  hipLaunchKernelGGL(k_arn_finish, dim3(1), dim3(kThreads), 0, ctx->stream, c);
  return hipGetLastError();
}

hipError_t launch_gmres_res(dctk_ctx ctx, const double* part, int npart, KState* st) {
  if (recording(ctx)) return hipErrorNotSupported;
  hipLaunchKernelGGL(k_gmres_res, dim3(1), dim3(kThreads), 0, ctx->stream, part, npart, st);
  return hipGetLastError();
}

hipError_t launch_gkb_start(dctk_ctx ctx, int dtype, int64_t n, void* X, void* W, void* V1, const double* part,
                            int npart, KState* st) {
  const unsigned grid = grid_for(n);
  GkbArgs a{};
  a.vec = (n % 4 == 0) && al(X) && al(W) && al(V1);
  a.n = n;
  a.X = X;
  a.W = W;
  a.V = V1;
  a.part = part;
  a.npart = npart;
  a.j = 0;
  a.st = st;
  if (dtype == DCTK_F64) return launch_kernel(ctx, ctx->stream, k_gkb_start<double, false>, k_gkb_start<double, true>, dim3(grid), kThreads, 0, a);
  return launch_kernel(ctx, ctx->stream, k_gkb_start<float, false>, k_gkb_start<float, true>, dim3(grid), kThreads, 0, a);
}

hipError_t launch_gkb_update(dctk_ctx ctx, int dtype, int64_t n, void* X, void* W, const void* Vin, void* Vn,
                             const double* part, int npart, KState* st, int j, void* U) {
  const unsigned grid = grid_for(n);
  GkbArgs a{};
  a.vec = (n % 4 == 0) && al(X) && al(W) && al(Vn) && al(Vin) && al(U);
  a.U = U;
  a.n = n;
  a.X = X;
  a.W = W;
  a.V = Vn;
  a.Vin = Vin;
  a.part = part;
  a.npart = npart;
  a.j = j;
  a.st = st;
  if (dtype == DCTK_F64) return launch_kernel(ctx, ctx->stream, k_gkb_update<double, false>, k_gkb_update<double, true>, dim3(grid), kThreads, 0, a);
  return launch_kernel(ctx, ctx->stream, k_gkb_update<float, false>, k_gkb_update<float, true>, dim3(grid), kThreads, 0, a);
}

hipError_t launch_cast(dctk_ctx ctx, int64_t n, const double* in, int out_dtype, void* out) {
  if (recording(ctx)) return hipErrorNotSupported;
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

hipError_t launch_cast_t(dctk_ctx ctx, int64_t p, int64_t rows, int64_t cols, const double* in, int out_dtype,
                         void* out) {
  if (recording(ctx)) return hipErrorNotSupported;
  unsigned grid = grid_for(p * rows * cols * 4);
  switch (out_dtype) {
    case DCTK_F32: hipLaunchKernelGGL(k_cast_t<float>, dim3(grid), dim3(kThreads), 0, ctx->stream, p, rows, cols, in, (float*)out); break;
    case DCTK_BF16: hipLaunchKernelGGL(k_cast_t<bf16_t>, dim3(grid), dim3(kThreads), 0, ctx->stream, p, rows, cols, in, (bf16_t*)out); break;
    case DCTK_F16: hipLaunchKernelGGL(k_cast_t<f16_t>, dim3(grid), dim3(kThreads), 0, ctx->stream, p, rows, cols, in, (f16_t*)out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_state_reset(dctk_ctx ctx, KState* st, int full, double tol) {
  ResetArgs a{};
  a.full = full;
  a.st = st;
  a.tol = tol;
  return launch_kernel(ctx, ctx->stream, k_state_reset<false>, k_state_reset<true>, dim3(1), 256, 0, a);
}

}  // namespace dctk
