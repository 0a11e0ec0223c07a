// The small projected problem of DC-GMRES and DC-GK (Sec. 3.1, 3.2), in FP64
// on the device, one workgroup:
//   * SVD of the (k+1) x k projected matrix (Hessenberg H~_k or lower
//     bidiagonal C~_k) by one-sided (Hestenes) Jacobi: columns are rotated
//     pairwise until orthogonal, in a round-robin order that lets 16 waves
//     rotate disjoint pairs at once (each wave reduces over the rows);
//   * the component of beta e_1 outside range(H), from the null vector z of
//     H^T (H^T z = 0 is a forward recurrence for a Hessenberg matrix), so it
//     does not suffer the cancellation of beta^2 - sum g_i^2;
//   * lambda by GCV: 400-point log grid on [1e-8 sigma_1, sigma_1], first
//     minimum, golden-section refinement on log10(lambda) in the neighbouring
//     cells (bracket < 1e-10 or 200 steps), keep the better of the refined
//     midpoint and the grid point;
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

__device__ inline double wave_bcast_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return __shfl(v, 0, 64);
}

__device__ inline double gcv_eval(int mode, double lam, int k, const double* sig, const double* g, double gperp2,
                                  int lane) {
  // lane-parallel over i (k <= 64): one term per lane
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
  t1 = wave_bcast_sum(t1);
  t2 = wave_bcast_sum(t2);
  if (mode == 0) {
    const double num = gperp2 + t1;
    const double tr = 1.0 + t2;
    return num / (tr * tr);
  }
  return t1 / (t2 * t2);
}

__global__ __launch_bounds__(kPT) void k_projected(KState* st, int bidiag, int gcv_mode, double lam_fixed) {
  if (st->halt) return;
  __shared__ double G[kMaxK * kLdG];      // G[c * kLdG + r]: column c of the matrix
  __shared__ double Vm[kMaxK * kMaxK];    // Vm[c * kMaxK + r]: right singular vectors
  __shared__ double sig[kMaxK], gs[kMaxK], g0s[kMaxK];
  __shared__ int order[kMaxK];
  __shared__ double z[kMaxK + 1];
  __shared__ double gridv[kGrid];
  __shared__ int rot_flag;
  __shared__ double s_gperp2, s_lam, s_gcv;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int k = st->steps;
  if (k > kMaxK) k = kMaxK;
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
  if (tid == 0) rot_flag = 0;
  __syncthreads();

  // component of beta e_1 outside range(H): z with H^T z = 0, z_0 = 1
  if (wave == 0) {
    bool zero = false;
    if (lane == 0) z[0] = 1.0;
    for (int j = 0; j < k; ++j) {
      const double part = (lane <= j) ? G[j * kLdG + lane] * z[lane] : 0.0;
      const double sum = wave_bcast_sum(part);
      const double h = G[j * kLdG + j + 1];
      if (h == 0.0) { zero = true; break; }
      const double zn = -sum / h;
      if (lane == 0) z[j + 1] = zn;
      if (fabs(zn) > 1e150) {
        for (int i = lane; i <= j + 1; i += 64) z[i] *= 1e-150;
      }
    }
    // ||z|| (scaled) and g_perp^2 = beta^2 z_0^2 / ||z||^2
    double zz = 0.0;
    if (!zero) {
      for (int i = lane; i <= k; i += 64) zz += z[i] * z[i];
    }
    zz = wave_bcast_sum(zz);
    if (lane == 0) s_gperp2 = zero ? 0.0 : (beta * z[0]) * (beta * z[0]) / zz;
  }
  __syncthreads();

  // one-sided Jacobi
  const int cEven = k + (k & 1);
  const int npairs = cEven / 2;
  const double tolJ = 1e-15;
  for (int sweep = 0; sweep < 60 && cEven > 1; ++sweep) {
    for (int rr = 0; rr < cEven - 1; ++rr) {
      for (int pi = wave; pi < npairs; pi += kPW) {
        const int pa = pi, pb = cEven - 1 - pi;
        int ia = (pa == 0) ? 0 : 1 + ((pa - 1 + rr) % (cEven - 1));
        int ib = (pb == 0) ? 0 : 1 + ((pb - 1 + rr) % (cEven - 1));
        int p = ia < ib ? ia : ib, q = ia < ib ? ib : ia;
        if (q >= k) continue;  // dummy column of an odd k
        double* gp = &G[p * kLdG];
        double* gq = &G[q * kLdG];
        double xp0 = lane < rows ? gp[lane] : 0.0;
        double xq0 = lane < rows ? gq[lane] : 0.0;
        double xp1 = (lane + 64) < rows ? gp[lane + 64] : 0.0;
        double xq1 = (lane + 64) < rows ? gq[lane + 64] : 0.0;
        const double a = wave_bcast_sum(xp0 * xp0 + xp1 * xp1);
        const double b = wave_bcast_sum(xq0 * xq0 + xq1 * xq1);
        const double c = wave_bcast_sum(xp0 * xq0 + xp1 * xq1);
        if (c == 0.0 || !(fabs(c) > tolJ * sqrt(a) * sqrt(b))) continue;
        const double zeta = (b - a) / (2.0 * c);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t);
        const double sn = cs * t;
        if (lane < rows) { gp[lane] = cs * xp0 - sn * xq0; gq[lane] = sn * xp0 + cs * xq0; }
        if (lane + 64 < rows) { gp[lane + 64] = cs * xp1 - sn * xq1; gq[lane + 64] = sn * xp1 + cs * xq1; }
        double* vp = &Vm[p * kMaxK];
        double* vq = &Vm[q * kMaxK];
        if (lane < k) {
          const double vpl = vp[lane], vql = vq[lane];
          vp[lane] = cs * vpl - sn * vql;
          vq[lane] = sn * vpl + cs * vql;
        }
        if (lane == 0) rot_flag = 1;
      }
      __syncthreads();
    }
    const int f = rot_flag;
    __syncthreads();
    if (tid == 0) rot_flag = 0;
    __syncthreads();
    if (!f) break;
  }

  // singular values (column norms), descending order
  if (tid < k) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += G[tid * kLdG + r] * G[tid * kLdG + r];
    sig[tid] = sqrt(s);
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < k; ++i) order[i] = i;
    for (int i = 0; i < k; ++i) {
      int best = i;
      for (int j2 = i + 1; j2 < k; ++j2)
        if (sig[order[j2]] > sig[order[best]]) best = j2;
      int tmp = order[i]; order[i] = order[best]; order[best] = tmp;
    }
  }
  __syncthreads();
  __shared__ double ssort[kMaxK];
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
  } else {
    const double s1 = ssort[0];
    if (!(s1 > 0.0)) {
      if (tid == 0) { s_lam = 0.0; s_gcv = __builtin_nan(""); }
    } else {
      const double t0 = log10(s1) - 8.0;
      const double dt = 8.0 / (double)(kGrid - 1);
      // grid: one wave per 64 points would need the lane-parallel evaluator; each wave
      // evaluates points w, w + 16, ... with its lanes over the singular values
      for (int i = wave; i < kGrid; i += kPW) {
        const double v = gcv_eval(gcv_mode, pow(10.0, t0 + (double)i * dt), k, ssort, gs, s_gperp2, lane);
        if (lane == 0) gridv[i] = v;
      }
      __syncthreads();
      if (wave == 0) {
        int ib = 0;
        for (int i = 1; i < kGrid; ++i)
          if (gridv[i] < gridv[ib]) ib = i;
        double a = t0 + (double)(ib > 0 ? ib - 1 : 0) * dt;
        double b = t0 + (double)(ib < kGrid - 1 ? ib + 1 : kGrid - 1) * dt;
        const double invphi = (sqrt(5.0) - 1.0) / 2.0;
        double c = b - invphi * (b - a);
        double d = a + invphi * (b - a);
        double fc = gcv_eval(gcv_mode, pow(10.0, c), k, ssort, gs, s_gperp2, lane);
        double fd = gcv_eval(gcv_mode, pow(10.0, d), k, ssort, gs, s_gperp2, lane);
        int steps = 0;
        while ((b - a) > 1e-10 && steps < 200) {
          if (fc <= fd) {
            b = d; d = c; fd = fc;
            c = b - invphi * (b - a);
            fc = gcv_eval(gcv_mode, pow(10.0, c), k, ssort, gs, s_gperp2, lane);
          } else {
            a = c; c = d; fc = fd;
            d = a + invphi * (b - a);
            fd = gcv_eval(gcv_mode, pow(10.0, d), k, ssort, gs, s_gperp2, lane);
          }
          ++steps;
        }
        const double tm = 0.5 * (a + b);
        const double fm = gcv_eval(gcv_mode, pow(10.0, tm), k, ssort, gs, s_gperp2, lane);
        if (lane == 0) {
          if (fm <= gridv[ib]) { s_lam = pow(10.0, tm); s_gcv = fm; }
          else { s_lam = pow(10.0, t0 + (double)ib * dt); s_gcv = gridv[ib]; }
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
      const double d = ssort[i] * ssort[i] + lam * lam;
      if (d > 0.0) acc += Vm[order[i] * kMaxK + tid] * (g0s[i] / d);
    }
    st->y[tid] = acc;
  }
  if (tid == 0) {
    st->lambda = lam;
    st->gcv = s_gcv;
  }
}

hipError_t launch_projected(dctk_ctx ctx, KState* st, int bidiag, int gcv_mode, double lambda) {
  hipLaunchKernelGGL(k_projected, dim3(1), dim3(kPT), 0, ctx->stream, st, bidiag, gcv_mode, lambda);
  return hipGetLastError();
}

}  // namespace dctk
