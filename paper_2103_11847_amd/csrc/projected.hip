// The small projected problem of DC-GMRES and DC-GK (Sec. 3.1, 3.2), in FP64
// on the device, one workgroup of 16 waves:
//   * SVD of the (k+1) x k projected matrix (Hessenberg H~_k or lower
//     bidiagonal C~_k) by one-sided (Hestenes) Jacobi: columns are rotated
//     pairwise until orthogonal, in a round-robin order; each pair of a round
//     belongs to a 16-lane row of a wave (rows of the matrix spread over the
//     lanes, dot products reduced with DPP row permutes), so a round of up to
//     64 pairs is one pass;
//   * the component of beta e_1 outside range(H), from the null vector z of
//     H^T (H^T z = 0 is a forward recurrence for a Hessenberg matrix), so it
//     does not suffer the cancellation of beta^2 - sum g_i^2;
//   * lambda by GCV: 400-point log grid on [1e-8 sigma_1, sigma_1] (one
//     point per thread), first minimum, golden-section refinement on
//     log10(lambda) in the neighbouring cells (bracket < 1e-10 or 200 steps),
//     keeping the better of the refined midpoint and the grid point;
//   * y_lambda = V diag(sigma / (sigma^2 + lambda^2)) g  (eq. leastsq / normeq2).
// The GCV function is that of the rectangular projected problem (mode 0) or
// the printed eq. (gcv2) (mode 1).
#include <cfloat>
#include <cmath>

#include "internal.h"

namespace dctk {

constexpr int kPT = 1024;            // threads
constexpr int kPW = kPT / 64;        // waves
constexpr int kGrid = 400;
constexpr int kLdG = kMaxK + 2;      // rows <= 65
static_assert(kPW * 4 >= (kMaxK + 1) / 2, "one Jacobi round must fit in one pass (4 pairs per wave)");

// ---- DPP helpers (64-bit values moved as two 32-bit halves) -------------------
template <int CTRL>
__device__ inline double dpp(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  const long long r = ((long long)(unsigned)lo) | ((long long)hi << 32);
  return __builtin_bit_cast(double, r);
}

// Sum over the 16 lanes of a row, returned to every lane of the row (identical
// bits: each step adds a commuted copy of the same partial sums).
__device__ inline double row16_sum(double v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return v;
}

__device__ inline double readlane_d(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Sum over the wave, uniform result.
__device__ inline double wave_sum_uniform(double v) {
  v = row16_sum(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// GCV at lambda, serial over the k singular values (one thread)
__device__ inline double gcv_serial(int mode, double lam, int k, const double* sig, const double* g, double gperp2) {
  const double l2 = lam * lam;
  if (mode == 0) {
    double num = gperp2, tr = 1.0;
    for (int i = 0; i < k; ++i) {
      const double f = l2 / (sig[i] * sig[i] + l2);
      num += (f * g[i]) * (f * g[i]);
      tr += f;
    }
    return num / (tr * tr);
  }
  double num = 0.0, den = 0.0;
  for (int i = 0; i < k; ++i) {
    const double d = sig[i] * sig[i] + l2;
    num += (g[i] / d) * (g[i] / d);
    den += 1.0 / d;
  }
  return num / (den * den);
}

// GCV at lambda, lanes over the singular values (one wave, uniform result)
__device__ inline double gcv_wave(int mode, double lam, int k, const double* sig, const double* g, double gperp2,
                                  int lane) {
  const double l2 = lam * lam;
  double t1 = 0.0, t2 = 0.0;
  if (lane < k) {
    const double s2 = sig[lane] * sig[lane];
    if (mode == 0) {
      const double f = l2 / (s2 + l2);
      t1 = (f * g[lane]) * (f * g[lane]);
      t2 = f;
    } else {
      const double d = s2 + l2;
      t1 = (g[lane] / d) * (g[lane] / d);
      t2 = 1.0 / d;
    }
  }
  t1 = wave_sum_uniform(t1);
  t2 = wave_sum_uniform(t2);
  if (mode == 0) {
    const double tr = 1.0 + t2;
    return (gperp2 + t1) / (tr * tr);
  }
  return t1 / (t2 * t2);
}

struct ProjArgs {
  int gx, gy, gz;
  int bidiag;
  int gcv_mode;
  int k_use;         // > 0: project at min(k_use, steps) instead of all steps taken
  KState* st;
  double lam_fixed;  // >= 0: this lambda; < 0: GCV
  double lam_cand;   // > 0 (with GCV): a proposed lambda, kept when GCV(lam_cand) <= gate * min GCV
  double gate;
  int cand_from_state;  // 1: the proposed lambda is st->pred_lambda (learned stop)
};

__global__ __launch_bounds__(kPT) void k_projected(ProjArgs a_, const ProjArgs* group, const int4* bmap) {
  VBlock vb;
  const ProjArgs a = pick_args(a_, group, bmap, vb);
  KState* st = a.st;
  const int bidiag = a.bidiag, gcv_mode = a.gcv_mode;
  const double lam_fixed = a.lam_fixed, gate = a.gate;
  const double lam_cand = a.cand_from_state ? ((volatile KState*)st)->pred_lambda : a.lam_cand;
  const int k_use = a.k_use;
  if (((volatile KState*)st)->halt) return;
  __shared__ double G[kMaxK * kLdG];      // G[c * kLdG + r]: column c of the matrix
  __shared__ double Vm[kMaxK * kMaxK];    // Vm[c * kMaxK + r]: right singular vectors
  __shared__ double sig[kMaxK], ssort[kMaxK], gs[kMaxK], g0s[kMaxK];
  __shared__ int order[kMaxK];
  __shared__ double z[kMaxK + 1];
  __shared__ double gridv[kGrid];
  __shared__ int rot_flag[2];
  __shared__ double s_gperp2, s_lam, s_gcv;
  __shared__ int s_ib;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int k = st->steps;
  if (k_use > 0 && k_use < k) k = k_use;
  if (k > kMaxK) k = kMaxK;
  if (tid == 0) st->gate_ok = 0.0;
  const int rows = k + 1;
  const double beta = bidiag ? st->beta[0] : st->beta0;
  if (k <= 0) {
    if (tid == 0) { st->lambda = 0.0; st->gcv = __builtin_nan(""); }
    return;
  }

  // load the matrix and V = I
  for (int i = tid; i < k * kLdG; i += kPT) {
    const int c = i / kLdG, r = i % kLdG;
    double v = 0.0;
    if (r < rows) {
      if (bidiag) v = (r == c) ? st->alpha[c] : (r == c + 1 ? st->beta[c + 1] : 0.0);
      else v = (r <= c + 1) ? st->H[r * kMaxK + c] : 0.0;
    }
    G[i] = v;
  }
  for (int i = tid; i < k * kMaxK; i += kPT) Vm[i] = ((i / kMaxK) == (i % kMaxK)) ? 1.0 : 0.0;
  if (tid == 0) { rot_flag[0] = 0; rot_flag[1] = 0; }
  __syncthreads();

  // component of beta e_1 outside range(H): z with H^T z = 0, z_0 = 1 (wave 0)
  if (wave == 0) {
    bool zero = false;
    double zl = (lane == 0) ? 1.0 : 0.0;   // lane l holds z_l (k <= 64: z_64 in z[64])
    if (lane == 0) z[0] = 1.0;
    for (int j = 0; j < k; ++j) {
      const double part = (lane <= j) ? G[j * kLdG + lane] * zl : 0.0;
      const double sum = wave_sum_uniform(part);
      const double h = G[j * kLdG + j + 1];
      if (h == 0.0) { zero = true; break; }
      double zn = -sum / h;
      if (fabs(zn) > 1e150) {
        zl *= 1e-150;
        zn *= 1e-150;
        if (lane == 0) {
          for (int i = 0; i <= j; ++i) z[i] *= 1e-150;
        }
      }
      if (lane == j + 1) zl = zn;
      if (lane == 0) z[j + 1] = zn;
    }
    double zz = 0.0;
    if (!zero) {
      for (int i = lane; i <= k; i += 64) zz += z[i] * z[i];
    }
    zz = wave_sum_uniform(zz);
    if (lane == 0) s_gperp2 = zero ? 0.0 : (beta * z[0]) * (beta * z[0]) / zz;
  }
  __syncthreads();

  // one-sided Jacobi: pair pi of a round belongs to row (lane / 16) of wave pi / 4
  const int cEven = k + (k & 1);
  const int npairs = cEven / 2;
  const int grp = lane >> 4, l16 = lane & 15;
  const int pi = wave * 4 + grp;
  // rotate while |g_p . g_q| > tol |g_p| |g_q|; below a few ulps per row the
  // columns are orthogonal to working precision
  const double tolJ = DBL_EPSILON * (double)rows;
  int sweeps = 0;
  for (int sweep = 0; sweep < 60 && cEven > 1; ++sweep) {
    const int flag = sweep & 1;
    sweeps = sweep + 1;
    for (int rr = 0; rr < cEven - 1; ++rr) {
      int p = 0, q = 0;
      bool valid = pi < npairs;
      if (valid) {
        const int pa = pi, pb = cEven - 1 - pi;
        const int ia = (pa == 0) ? 0 : 1 + ((pa - 1 + rr) % (cEven - 1));
        const int ib = (pb == 0) ? 0 : 1 + ((pb - 1 + rr) % (cEven - 1));
        p = ia < ib ? ia : ib;
        q = ia < ib ? ib : ia;
        valid = q < k;  // the dummy column of an odd k
      }
      // every lane takes part in the row reductions (zeros when idle)
      double xp[5], xq[5];
      double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
      for (int u = 0; u < 5; ++u) {
        const int r = l16 + 16 * u;
        const bool in = valid && r < rows;
        xp[u] = in ? G[p * kLdG + r] : 0.0;
        xq[u] = in ? G[q * kLdG + r] : 0.0;
        a += xp[u] * xp[u];
        b += xq[u] * xq[u];
        c += xp[u] * xq[u];
      }
      a = row16_sum(a);
      b = row16_sum(b);
      c = row16_sum(c);
      if (valid && c != 0.0 && c * c > (tolJ * tolJ) * (a * b)) {
        // tan of the rotation angle, the smaller root of t^2 + 2 zeta t - 1 = 0
        // with zeta = (b - a) / (2c), written with one square root and one division
        const double dba = b - a;
        const double t = (dba >= 0.0 ? 2.0 * c : -2.0 * c) / (fabs(dba) + sqrt(dba * dba + 4.0 * c * c));
        const double cs = rsqrt(1.0 + t * t);
        const double sn = cs * t;
#pragma unroll
        for (int u = 0; u < 5; ++u) {
          const int r = l16 + 16 * u;
          if (r < rows) {
            G[p * kLdG + r] = cs * xp[u] - sn * xq[u];
            G[q * kLdG + r] = sn * xp[u] + cs * xq[u];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = l16 + 16 * u;
          if (r < k) {
            const double vp = Vm[p * kMaxK + r], vq = Vm[q * kMaxK + r];
            Vm[p * kMaxK + r] = cs * vp - sn * vq;
            Vm[q * kMaxK + r] = sn * vp + cs * vq;
          }
        }
        if (l16 == 0) rot_flag[flag] = 1;
      }
      __syncthreads();
    }
    const int f = rot_flag[flag];
    if (tid == 0) rot_flag[flag ^ 1] = 0;
    __syncthreads();
    if (!f) break;
  }

  // singular values (column norms) and their descending order (rank sort, ties by index)
  if (tid < k) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += G[tid * kLdG + r] * G[tid * kLdG + r];
    sig[tid] = sqrt(s);
  }
  if (tid < k) order[tid] = tid;  // stays a valid index even if NaNs make ranks collide
  __syncthreads();
  if (tid < k) {
    const double si = sig[tid];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double sj = sig[j];
      rank += (sj > si || (sj == si && j < tid)) ? 1 : 0;
    }
    order[rank] = tid;
  }
  __syncthreads();
  if (tid < k) {
    const int c = order[tid];
    const double s = sig[c];
    ssort[tid] = s;
    g0s[tid] = beta * G[c * kLdG];                    // sigma_i g_i
    gs[tid] = s > 0.0 ? beta * G[c * kLdG] / s : 0.0; // g_i = beta (U^T e_1)_i
  }
  __syncthreads();

  // lambda
  if (lam_fixed >= 0.0) {
    if (tid == 0) { s_lam = lam_fixed; s_gcv = __builtin_nan(""); }
  } else if (!(ssort[0] > 0.0)) {
    if (tid == 0) { s_lam = 0.0; s_gcv = __builtin_nan(""); }
  } else {
    const double t0 = log10(ssort[0]) - 8.0;
    const double dt = 8.0 / (double)(kGrid - 1);
    if (tid < kGrid) gridv[tid] = gcv_serial(gcv_mode, pow(10.0, t0 + (double)tid * dt), k, ssort, gs, s_gperp2);
    __syncthreads();
    if (wave == 0) {
      // first index of the minimum: per-lane scan, then lanes in order
      int bi = -1;
      double bv = 0.0;
      for (int i = lane; i < kGrid; i += 64)
        if (bi < 0 || gridv[i] < bv) { bi = i; bv = gridv[i]; }
      if (lane == 0) s_ib = 0;
      for (int l = 0; l < 64; ++l) {
        const int li = __builtin_amdgcn_readlane(bi, l);
        const double lv = readlane_d(bv, l);
        if (lane == 0 && li >= 0) {
          const int cur = s_ib;
          if (lv < gridv[cur] || (lv == gridv[cur] && li < cur)) s_ib = li;
        }
      }
      const int ib = __builtin_amdgcn_readfirstlane(s_ib);
      double a = t0 + (double)(ib > 0 ? ib - 1 : 0) * dt;
      double b = t0 + (double)(ib < kGrid - 1 ? ib + 1 : kGrid - 1) * dt;
      const double invphi = (sqrt(5.0) - 1.0) / 2.0;
      double c = b - invphi * (b - a);
      double d = a + invphi * (b - a);
      double fc = gcv_wave(gcv_mode, pow(10.0, c), k, ssort, gs, s_gperp2, lane);
      double fd = gcv_wave(gcv_mode, pow(10.0, d), k, ssort, gs, s_gperp2, lane);
      int steps = 0;
      while ((b - a) > 1e-10 && steps < 200) {
        if (fc <= fd) {
          b = d; d = c; fd = fc;
          c = b - invphi * (b - a);
          fc = gcv_wave(gcv_mode, pow(10.0, c), k, ssort, gs, s_gperp2, lane);
        } else {
          a = c; c = d; fc = fd;
          d = a + invphi * (b - a);
          fd = gcv_wave(gcv_mode, pow(10.0, d), k, ssort, gs, s_gperp2, lane);
        }
        ++steps;
      }
      const double tm = 0.5 * (a + b);
      const double fm = gcv_wave(gcv_mode, pow(10.0, tm), k, ssort, gs, s_gperp2, lane);
      if (lane == 0) {
        if (fm <= gridv[ib]) { s_lam = pow(10.0, tm); s_gcv = fm; }
        else { s_lam = pow(10.0, t0 + (double)ib * dt); s_gcv = gridv[ib]; }
      }
      // a proposed lambda is kept when its GCV value is within the gate of the minimum
      if (lam_cand > 0.0) {
        const double fcand = gcv_wave(gcv_mode, lam_cand, k, ssort, gs, s_gperp2, lane);
        if (lane == 0) {
          const bool keep = fcand <= gate * s_gcv;
          st->gate_ok = keep ? 1.0 : 0.0;
          if (keep) { s_lam = lam_cand; s_gcv = fcand; }
        }
      }
    }
  }
  __syncthreads();

  // y = sum_i v_i sigma_i g_i / (sigma_i^2 + lambda^2)
  const double lam = s_lam;
  if (tid < k) {
    double acc = 0.0;
    for (int i = 0; i < k; ++i) {
      const double dd = ssort[i] * ssort[i] + lam * lam;
      if (dd > 0.0) acc += Vm[order[i] * kMaxK + tid] * (g0s[i] / dd);
    }
    st->y[tid] = acc;
  }
  if (tid == 0) {
    st->lambda = lam;
    st->gcv = s_gcv;
    st->sweeps = (double)sweeps;
  }
}

hipError_t launch_projected(dctk_ctx ctx, KState* st, int bidiag, int gcv_mode, double lambda, int k_use,
                            double lam_cand, double gate, int cand_from_state) {
  ProjArgs a{};
  a.cand_from_state = cand_from_state;
  a.bidiag = bidiag;
  a.gcv_mode = gcv_mode;
  a.k_use = k_use;
  a.st = st;
  a.lam_fixed = lambda;
  a.lam_cand = lam_cand;
  a.gate = gate;
  return launch_kernel(ctx, ctx->stream, k_projected, dim3(1), kPT, 0, a);
}

}  // namespace dctk
