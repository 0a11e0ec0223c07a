// The small projected problem of DC-GMRES and DC-GK (Sec. 3.1, 3.2), in FP64
// on the device, one workgroup of 16 waves.  Two kernels:
//
// k_projected (the Hessenberg matrix of DC-GMRES, and the printed GCV form
// eq. (gcv2) of either method):
//   * SVD of the (k+1) x k projected matrix by one-sided (Hestenes) Jacobi:
//     columns are rotated pairwise until orthogonal, in a round-robin order;
//     each pair of a round belongs to an 8-lane group of a wave (rows of the
//     matrix spread over the lanes, dot products reduced with DPP permutes),
//     so a round of up to 32 pairs is one pass of at most four waves, one per
//     SIMD;
//   * the component of beta e_1 outside range(H), from the null vector z of
//     H^T (H^T z = 0 is a forward recurrence for a Hessenberg matrix), so it
//     does not suffer the cancellation of beta^2 - sum g_i^2;
//   * lambda by GCV: 400-point log grid on [1e-8 sigma_1, sigma_1] (one
//     point per thread), first minimum, then the neighbouring cells are
//     subdivided in passes of 64 points (one 16-lane row each) around the
//     first smallest value until the bracket on log10(lambda) is below 1e-10,
//     keeping the better of the refined point and the grid point;
//   * y_lambda (eq. leastsq / normeq2): for the bidiagonal matrix by plane
//     rotations of [C~_k; lambda I], for the Hessenberg matrix as
//     V diag(sigma / (sigma^2 + lambda^2)) g.
//
// k_projected_gk (the lower bidiagonal C~_k of DC-GK with the GCV function of
// the rectangular projected problem, or a fixed lambda): no SVD, see below.
#include <cfloat>
#include <cmath>

#include "internal.h"
#include "projected.h"

namespace dctk {

constexpr int kPT = 1024;            // threads
constexpr int kPW = kPT / 64;        // waves
constexpr int kGrid = 400;
// Column strides of G (rows <= 65) and V: 72 doubles = 144 dwords, 16 more than a
// multiple of 64 banks, so that the 8-lane groups of a wave, which read
// 8 consecutive rows of mostly consecutive columns, fall in distinct bank windows.
constexpr int kLdG = 72;
constexpr int kLdV = 72;
constexpr int kJR = (kMaxK + 1 + 7) / 8;   // rows of G (and V) per lane of an 8-lane group
constexpr int kRef = kPW * 4;              // GCV refinement points per pass (16-lane rows)
static_assert(kPW * 8 >= (kMaxK + 1) / 2, "one Jacobi round must fit in one pass (8 pairs per wave)");
static_assert(kRef == 64, "the refinement pass reduces one value per lane of a wave");
static_assert(kLdV >= kMaxK, "V columns hold kMaxK rows");
static_assert(kJR * 8 <= kLdG && kLdG >= kMaxK + 1, "a lane reads rows l, l + 8, ... < kLdG of G");

// Sum over the 8 lanes of a half row, returned to every lane of it (identical bits).
__device__ inline double row8_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  return v;
}

// (value, index) of the first smallest value over the wave, in every lane
__device__ inline void first_min64(double& v, int& i) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const double ov = __shfl_xor(v, m);
    const int oi = __shfl_xor(i, m);
    if (ov < v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
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
  t1 = wave_sum(t1);
  t2 = wave_sum(t2);
  if (mode == 0) {
    const double tr = 1.0 + t2;
    return (gperp2 + t1) / (tr * tr);
  }
  return t1 / (t2 * t2);
}

// GCV at lambda, the 16 lanes of a row over the singular values (result in every lane of the row)
__device__ inline double gcv_row16(int mode, double lam, int k, const double* sig, const double* g, double gperp2,
                                   int l16) {
  const double l2 = lam * lam;
  double t1 = 0.0, t2 = 0.0;
  for (int i = l16; i < k; i += 16) {
    const double s2 = sig[i] * sig[i];
    if (mode == 0) {
      const double f = l2 / (s2 + l2);
      t1 += (f * g[i]) * (f * g[i]);
      t2 += f;
    } else {
      const double d = s2 + l2;
      t1 += (g[i] / d) * (g[i] / d);
      t2 += 1.0 / d;
    }
  }
  t1 = row16_sum(t1);
  t2 = row16_sum(t2);
  if (mode == 0) {
    const double tr = 1.0 + t2;
    return (gperp2 + t1) / (tr * tr);
  }
  return t1 / (t2 * t2);
}

// One round of the one-sided Jacobi method for the pair (p, q) of this 8-lane
// group: each lane holds rows l8, l8 + 8, ... (NR of them) of the two columns
// of G and, when V is accumulated, of V.  Every load is issued before the
// first use, from addresses inside the arrays: rows past the matrix read the
// zero rows below it, and the columns of an idle pair are replaced by zeros
// after the load.
template <int NR, bool WITHV>
__device__ inline void jacobi_round(double* G, double* Vm, int p, int q, bool valid, int l8, int rows, int k,
                                    double tolJ, int* rot_flag) {
  static_assert(8 * NR <= kLdG && 8 * NR <= kLdV, "rows of a lane inside the column strides");
  double xp[NR], xq[NR], vp[NR], vq[NR];
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int r = l8 + 8 * u;
    xp[u] = G[p * kLdG + r];
    xq[u] = G[q * kLdG + r];
  }
  if constexpr (WITHV) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      vp[u] = Vm[p * kLdV + l8 + 8 * u];
      vq[u] = Vm[q * kLdV + l8 + 8 * u];
    }
  }
  double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const double x = valid ? xp[u] : 0.0, y = valid ? xq[u] : 0.0;
    a += x * x;
    b += y * y;
    c += x * y;
  }
  a = row8_sum(a);
  b = row8_sum(b);
  c = row8_sum(c);
  if (valid && c != 0.0 && c * c > (tolJ * tolJ) * (a * b)) {
    // The smaller of the two rotations that make g_p . g_q zero, through the
    // double angle: with h = sqrt((b - a)^2 + 4c^2), cos 2th = |b - a| / h and
    // sin 2th = sign(b - a) 2c / h; then cos th = sqrt((1 + cos 2th) / 2) and
    // sin th = sin 2th / (2 cos th), with 1 + cos 2th >= 1 (no cancellation):
    // two reciprocal square roots, no division.
    const double dba = b - a;
    const double ih = rsqrt(dba * dba + 4.0 * c * c);
    const double c2 = fabs(dba) * ih;
    const double s2 = (dba >= 0.0 ? 2.0 * c : -2.0 * c) * ih;
    const double w = 0.5 + 0.5 * c2;
    const double iw = rsqrt(w);
    const double cs = w * iw;
    const double sn = 0.5 * s2 * iw;
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int r = l8 + 8 * u;
      if (r < rows) {
        G[p * kLdG + r] = cs * xp[u] - sn * xq[u];
        G[q * kLdG + r] = sn * xp[u] + cs * xq[u];
      }
    }
    if constexpr (WITHV) {
#pragma unroll
      for (int u = 0; u < NR; ++u) {
        const int r = l8 + 8 * u;
        if (r < k) {
          Vm[p * kLdV + r] = cs * vp[u] - sn * vq[u];
          Vm[q * kLdV + r] = sn * vp[u] + cs * vq[u];
        }
      }
    }
    if (l8 == 0) *rot_flag = 1;
  }
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
  double target;        // gcv_mode 2 (discrepancy principle): the residual norm lambda is chosen for
};

__device__ __forceinline__ void k_projected_body(const ProjArgs& a, const VBlock vb, const bool grouped) {
  KState* st = a.st;
  const int bidiag = a.bidiag, gcv_mode = a.gcv_mode;
  const double lam_fixed = a.lam_fixed, gate = a.gate;
  const double lam_cand = a.cand_from_state ? ld_state(&st->pred_lambda) : a.lam_cand;
  const int k_use = a.k_use;
  if (ld_state(&st->halt)) return;
  __shared__ double G[kMaxK * kLdG];      // G[c * kLdG + r]: column c of the matrix
  __shared__ double Vm[kMaxK * kLdV];     // Vm[c * kLdV + r]: right singular vectors
  __shared__ double sig[kMaxK], ssort[kMaxK], gs[kMaxK], g0s[kMaxK];
  __shared__ int order[kMaxK];
  __shared__ double z[kMaxK + 1];
  __shared__ double gridv[kGrid];
  __shared__ double refv[kRef];
  __shared__ double wcoef[kMaxK];
  __shared__ double ab_a[kMaxK], ab_b[kMaxK];   // bidiagonal: alpha_1..alpha_k, beta_2..beta_{k+1}
  __shared__ int rot_flag[2];
  __shared__ double s_gperp2, s_lam, s_gcv;
  __shared__ double s_ra, s_rb, s_rt, s_rf;
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
  if (bidiag) {
    if (tid < k) {
      ab_a[tid] = st->alpha[tid];
      ab_b[tid] = st->beta[tid + 1];
    }
  } else {
    for (int i = tid; i < k * kLdV; i += kPT) Vm[i] = ((i / kLdV) == (i % kLdV)) ? 1.0 : 0.0;
  }
  if (tid == 0) { rot_flag[0] = 0; rot_flag[1] = 0; }
  __syncthreads();

  // component of beta e_1 outside range(H): z with H^T z = 0, z_0 = 1 (wave 0)
  if (wave == 0) {
    if (bidiag) {
      // lower bidiagonal: alpha_j z_j + beta_{j+1} z_{j+1} = 0, one lane
      if (lane == 0) {
        bool zero = false;
        double z0 = 1.0, zj = 1.0, zz = 1.0;
        for (int j = 0; j < k; ++j) {
          const double h = G[j * kLdG + j + 1];
          if (h == 0.0) { zero = true; break; }
          double zn = -(G[j * kLdG + j] * zj) / h;
          if (fabs(zn) > 1e150) {
            z0 *= 1e-150;
            zz *= 1e-300;
            zn *= 1e-150;
          }
          zz += zn * zn;
          zj = zn;
        }
        s_gperp2 = zero ? 0.0 : (beta * z0) * (beta * z0) / zz;
      }
    } else {
      bool zero = false;
      double zl = (lane == 0) ? 1.0 : 0.0;   // lane l holds z_l (k <= 64: z_64 in z[64])
      if (lane == 0) z[0] = 1.0;
      for (int j = 0; j < k; ++j) {
        const double part = (lane <= j) ? G[j * kLdG + lane] * zl : 0.0;
        const double sum = wave_sum(part);
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
      zz = wave_sum(zz);
      if (lane == 0) s_gperp2 = zero ? 0.0 : (beta * z[0]) * (beta * z[0]) / zz;
    }
  }
  __syncthreads();

  // One-sided Jacobi.  Pair pi of a round belongs to an 8-lane group (lane / 8)
  // of wave pi / 8, so at most four waves (one per SIMD) do the work of a round.
  // V is accumulated only for the Hessenberg matrix.
  const int cEven = k + (k & 1);
  const int npairs = cEven / 2;
  const int grp = lane >> 3, l8 = lane & 7;
  const int pi = wave * 8 + grp;
  // positions of this group's pair and their (pos - 1 + rr) mod (cEven - 1),
  // advanced by one per round (a sweep of cEven - 1 rounds returns them)
  const int pa = pi, pb = cEven - 1 - pi;
  int ma = pa > 0 ? pa - 1 : 0, mb = pb > 0 ? pb - 1 : 0;
  // rotate while |g_p . g_q| > tol |g_p| |g_q|; below a few ulps per row the
  // columns are orthogonal to working precision
  const double tolJ = DBL_EPSILON * (double)rows;
  const bool small = rows <= 48;  // six rows per lane suffice
  int sweeps = 0;
  for (int sweep = 0; sweep < 60 && cEven > 1; ++sweep) {
    const int flag = sweep & 1;
    sweeps = sweep + 1;
    for (int rr = 0; rr < cEven - 1; ++rr) {
      // waves without a pair this round go straight to the barrier
      if (wave * 8 >= npairs) {
        __syncthreads();
        continue;
      }
      const int ia = pa == 0 ? 0 : 1 + ma, ib = pb == 0 ? 0 : 1 + mb;
      ma = ma + 1 == cEven - 1 ? 0 : ma + 1;
      mb = mb + 1 == cEven - 1 ? 0 : mb + 1;
      const bool live = pi < npairs;
      const int p = live ? min(ia, ib) : 0, q = live ? max(ia, ib) : 0;
      const bool valid = live && q < k;  // the dummy column of an odd k
      // every lane takes part in the group reductions (zeros when idle); the
      // bidiagonal case needs no V (y comes from the damped recurrence below)
      if (bidiag) {
        if (small) jacobi_round<6, false>(G, Vm, p, q, valid, l8, rows, k, tolJ, &rot_flag[flag]);
        else jacobi_round<kJR, false>(G, Vm, p, q, valid, l8, rows, k, tolJ, &rot_flag[flag]);
      } else {
        if (small) jacobi_round<6, true>(G, Vm, p, q, valid, l8, rows, k, tolJ, &rot_flag[flag]);
        else jacobi_round<kJR, true>(G, Vm, p, q, valid, l8, rows, k, tolJ, &rot_flag[flag]);
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
    if (tid < kGrid) gridv[tid] = gcv_serial(gcv_mode, exp10(t0 + (double)tid * dt), k, ssort, gs, s_gperp2);
    __syncthreads();
    if (wave == 0) {
      // first index of the minimum (NaN counts as +inf)
      int bi = kGrid;
      double bv = __builtin_inf();
      for (int i = lane; i < kGrid; i += 64) {
        const double v = gridv[i] == gridv[i] ? gridv[i] : __builtin_inf();
        if (bi == kGrid || v < bv) { bi = i; bv = v; }
      }
      first_min64(bv, bi);
      const int ib = bi < kGrid ? bi : 0;
      if (lane == 0) {
        s_ib = ib;
        s_ra = t0 + (double)(ib > 0 ? ib - 1 : 0) * dt;
        s_rb = t0 + (double)(ib < kGrid - 1 ? ib + 1 : kGrid - 1) * dt;
        s_rt = __builtin_nan("");
        s_rf = __builtin_inf();
      }
    }
    __syncthreads();
    // Refine on t = log10(lambda) inside the grid cells next to the minimum:
    // each pass evaluates kRef points evenly inside [a, b] (one 16-lane row
    // of the workgroup per point) and keeps the two cells next to the first
    // smallest value, until the bracket is narrower than 1e-10.
    const int row = wave * 4 + (lane >> 4), l16 = lane & 15;
    for (int pass = 0; pass < 40; ++pass) {
      const double ra = s_ra, rb = s_rb;
      if (!((rb - ra) > 1e-10)) break;
      const double h = (rb - ra) / (double)(kRef + 1);
      const double tq = ra + (double)(row + 1) * h;
      const double f = gcv_row16(gcv_mode, exp10(tq), k, ssort, gs, s_gperp2, l16);
      if (l16 == 0) refv[row] = f;
      __syncthreads();
      if (wave == 0) {
        const double v = refv[lane] == refv[lane] ? refv[lane] : __builtin_inf();
        int mi = lane;
        double mv = v;
        first_min64(mv, mi);
        if (lane == 0) {
          s_ra = ra + (double)mi * h;          // point mi - 1 (or a)
          s_rb = ra + (double)(mi + 2) * h;    // point mi + 1 (or b)
          s_rt = ra + (double)(mi + 1) * h;
          s_rf = mv;
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int ib = s_ib;
      if (s_rf <= gridv[ib]) { s_lam = exp10(s_rt); s_gcv = s_rf; }
      else { s_lam = exp10(t0 + (double)ib * dt); s_gcv = gridv[ib]; }
    }
    __syncthreads();
    // a proposed lambda is kept when its GCV value is within the gate of the minimum
    if (lam_cand > 0.0 && wave == 0) {
      const double fcand = gcv_wave(gcv_mode, lam_cand, k, ssort, gs, s_gperp2, lane);
      if (lane == 0) {
        const bool keep = fcand <= gate * s_gcv;
        st->gate_ok = keep ? 1.0 : 0.0;
        if (keep) { s_lam = lam_cand; s_gcv = fcand; }
      }
    }
  }
  __syncthreads();

  const double lam = s_lam;
  if (bidiag) {
    // y_lambda = argmin ||C~ y - beta_1 e_1||^2 + lambda^2 ||y||^2 by plane
    // rotations of [C~; lambda I] (the damped bidiagonal recurrence of LSQR):
    // at step i the damping row is rotated into rhobar_i, then beta_{i+1}
    // below it, which leaves R upper bidiagonal (rho_i, theta_{i+1}) and its
    // right-hand side phi_i; then R y = phi by back substitution.  One lane.
    if (tid == 0) {
      double* rho = wcoef;
      double* phi = gs;
      double* th = ssort;
      double rbar = ab_a[0], fbar = beta;
      for (int i = 0; i < k; ++i) {
        const double rhat = sqrt(rbar * rbar + lam * lam);
        const double c1 = rhat > 0.0 ? rbar / rhat : 1.0;
        const double fhat = c1 * fbar;
        const double bn = ab_b[i];
        const double r = sqrt(rhat * rhat + bn * bn);
        const double c = r > 0.0 ? rhat / r : 1.0, sn = r > 0.0 ? bn / r : 0.0;
        rho[i] = r;
        phi[i] = c * fhat;
        if (i + 1 < k) {
          th[i] = sn * ab_a[i + 1];
          rbar = -c * ab_a[i + 1];
        }
        fbar = sn * fhat;
      }
      double yn = 0.0;
      for (int i = k - 1; i >= 0; --i) {
        const double rhs = phi[i] - (i + 1 < k ? th[i] * yn : 0.0);
        yn = rho[i] > 0.0 ? rhs / rho[i] : 0.0;
        st->y[i] = yn;
      }
    }
  } else {
    // y = sum_i v_i sigma_i g_i / (sigma_i^2 + lambda^2)
    if (tid < k) {
      const double dd = ssort[tid] * ssort[tid] + lam * lam;
      wcoef[tid] = dd > 0.0 ? g0s[tid] / dd : 0.0;
    }
    __syncthreads();
    if (tid < k) {
      double acc = 0.0;
      for (int i = 0; i < k; ++i) acc += Vm[order[i] * kLdV + tid] * wcoef[i];
      st->y[tid] = acc;
    }
  }
  if (tid == 0) {
    st->lambda = lam;
    st->gcv = s_gcv;
    st->sweeps = (double)sweeps;
  }
}

template <bool GROUPED>
__global__ __launch_bounds__(kPT) void k_projected(ProjArgs a_, const ProjArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_projected_body(a_, hw_block(), false);
  } else {
    VBlock vb;
    const ProjArgs g = group_args(grp, bmap, vb);
    k_projected_body(g, vb, true);
  }
}

// ---- DC-GK projected problem without an SVD ---------------------------------
// For the lower bidiagonal C~_k with the GCV function of the rectangular
// projected problem (or a fixed lambda) no singular vectors are needed:
//   * sigma_1 (which fixes the GCV grid) by multisection with Sturm counts on
//     the Golub-Kahan form of C~_k;
//   * GCV(lambda) = ||beta e_1 - C~ y_lambda||^2 / (1 + lambda^2 ||R^-1||_F^2)^2,
//     where [C~; lambda I] = Q [R; 0] by the damped bidiagonal recurrence: the
//     sum over the singular values of lambda^2 / (sigma_i^2 + lambda^2) is
//     lambda^2 trace((C~^T C~ + lambda^2 I)^-1) = lambda^2 ||R^-1||_F^2, whose
//     column norms follow a forward recurrence, and the residual is formed
//     from y_lambda = R^-1 f directly (no cancellation against beta^2);
//   * the same grid and gate as the SVD path; the refinement is one pass of
//     up to 256 points and a step to the vertex of the parabola through the
//     smallest value and its neighbours.
constexpr int kRecD = 18432;  // doubles of per-lambda recurrence rows (144 KB)
constexpr int kMS = 256;      // multisection points per round
constexpr int kRP = 256;      // most refinement points per pass
static_assert(kRecD / (2 * kMaxK) >= 64, "a pass keeps at least 64 lambdas' rows");

// Eigenvalues below x > 0 of the Golub-Kahan tridiagonal of C~_k (order
// 2k + 1, zero diagonal, off-diagonals alpha_1, beta_2, ..., alpha_k,
// beta_{k+1}; eigenvalues +-sigma_i and 0): by Sylvester's law of inertia the
// number of negative pivots of T - x I, i.e. of sign changes between
// consecutive leading principal minors d_i = -x d_{i-1} - e_{i-1}^2 d_{i-2}.
// e2 holds the squared off-diagonals in order, padded with zeros to n2 (a
// multiple of 8) entries: each zero decouples one more row, an eigenvalue 0,
// which adds one to the count.  No division: with x and the off-diagonals
// divided by a bound g of the spectrum (ig = 1 / g) a minor grows at most
// twofold per step, so rescaling by powers of two (exact) every eight minors
// keeps them in range.  Sign changes are counted from the sign bits (a zero
// minor of either sign is followed by one that restores the count).
__device__ inline int gk_count_below(double x, int n2, const double* e2, double ig) {
  const double ig2 = ig * ig;
  x *= ig;
  double d0 = 1.0, d1 = -x;
  unsigned cnt = 1;  // d1 < 0 for x > 0
  unsigned sg = 1;
  for (int j = 0; j < n2; j += 8) {
    double ev[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) ev[u] = e2[j + u] * ig2;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double d2 = fma(-x, d1, -ev[u] * d0);
      const unsigned s2 = (unsigned)((unsigned long long)__double_as_longlong(d2) >> 63);
      cnt += s2 ^ sg;
      sg = s2;
      d0 = d1;
      d1 = d2;
    }
    const double m = fmax(fabs(d0), fabs(d1));
    const double sc = m > 0x1p256 ? 0x1p-256 : (m < 0x1p-256 ? 0x1p256 : 1.0);
    d0 *= sc;
    d1 *= sc;
  }
  return (int)cnt;
}

// GCV of the rectangular projected problem at lambda > 0, one thread.  Plane
// rotations of [C~; lambda I] (the damping row into rhobar_i, then beta_{i+1}
// below it) give R = bidiag(rho_i, theta_{i+1}) and f; with reciprocal square
// roots, no division.  Column j of R^-1 has squared norm
// T_j = (1 + theta_j^2 T_{j-1}) / rho_j^2.  The rows f_i / rho_i and
// theta_{i+1} / rho_i go to q[i * ld] and w[i * ld] for the back substitution
// y = R^-1 f, which also forms the residual rows of beta e_1 - C~ y (and
// writes y to yout when it is not null).  Each step's operands are loaded one
// step ahead, off the recurrence's dependency chain.
__device__ inline double gk_gcv(double lam, int k, const double* a, const double* b, double beta, double* q,
                                double* w, int ld, double* yout, double* res2 = nullptr) {
  const double l2 = lam * lam;
  double rbar = a[0], fbar = beta, th = 0.0, tcol = 0.0, tr = 0.0;
  double bn = b[0], an = a[min(1, k - 1)];
  for (int i = 0; i < k; ++i) {
    const double bc = bn, ac = an;
    bn = b[min(i + 1, k - 1)];
    an = a[min(i + 2, k - 1)];
    const double x1 = fma(rbar, rbar, l2);
    const double i1 = rsqrt(x1);
    const double i2 = rsqrt(fma(bc, bc, x1));  // 1 / rho_i
    const double rhat = x1 * i1;
    const double fhat = (rbar * i1) * fbar;
    const double c = rhat * i2, sn = bc * i2;
    tcol = fma(th * th, tcol, 1.0) * (i2 * i2);
    tr += tcol;
    q[i * ld] = (c * fhat) * i2;
    th = sn * ac;       // theta_{i+1} (unused after the last step)
    w[i * ld] = th * i2;
    rbar = -c * ac;
    fbar = sn * fhat;
  }
  double yn = 0.0, rr = 0.0;
  double qn = q[(k - 1) * ld], wn = 0.0, bb = b[k - 1], aa = 0.0;  // operands of step k - 1
  for (int i = k - 1; i >= 0; --i) {
    const double qc = qn, wc = wn, bc = bb, ac = aa;  // q_i, w_i, b_i, a_{i+1} (w, a: 0 at i = k - 1)
    const int ip = max(i - 1, 0);
    qn = q[ip * ld];
    wn = w[ip * ld];
    bb = b[ip];
    aa = a[i];
    const double y = fma(-wc, yn, qc);
    const double row = fma(bc, y, ac * yn);  // row i + 1 of C~ y
    rr = fma(row, row, rr);
    yn = y;
    if (yout != nullptr) yout[i] = y;
  }
  const double r0 = fma(-a[0], yn, beta);
  rr = fma(r0, r0, rr);
  if (res2 != nullptr) *res2 = rr;
  const double den = fma(l2, tr, 1.0);
  return rr / (den * den);
}

__device__ __forceinline__ void k_projected_gk_body(const ProjArgs& a, const VBlock vb, const bool grouped) {
  KState* st = a.st;
  const double lam_fixed = a.lam_fixed, gate = a.gate;
  const double lam_cand = a.cand_from_state ? ld_state(&st->pred_lambda) : a.lam_cand;
  const int k_use = a.k_use;
  if (ld_state(&st->halt)) return;
  __shared__ double rec[kRecD];
  __shared__ double ab_a[kMaxK], ab_b[kMaxK], e2[2 * kMaxK + 8];
  __shared__ double gridv[kGrid];
  __shared__ double refv[kRP];
  __shared__ int wfirst[kPW];
  __shared__ double s_lo, s_hi, s_ra, s_rb, s_rt, s_rf, s_fl, s_fr;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int k = st->steps;
  if (k_use > 0 && k_use < k) k = k_use;
  if (k > kMaxK) k = kMaxK;
  if (tid == 0) st->gate_ok = 0.0;
  const double beta = st->beta[0];
  if (k <= 0) {
    if (tid == 0) { st->lambda = 0.0; st->gcv = __builtin_nan(""); }
    return;
  }
  const int n2 = (2 * k + 7) & ~7;  // padded length of e2
  if (tid < k) {
    const double al = st->alpha[tid], be = st->beta[tid + 1];
    ab_a[tid] = al;
    ab_b[tid] = be;
    e2[2 * tid] = al * al;
    e2[2 * tid + 1] = be * be;
  } else if (tid >= 2 * k && tid < n2) {
    e2[tid] = 0.0;
  }
  __syncthreads();

  double lam = lam_fixed, gcv = __builtin_nan("");
  bool y_done = false;
  if (lam_fixed < 0.0) {
    // sigma_1: Gershgorin bound, then rounds of kMS evenly spaced Sturm counts
    // (one wave per SIMD); the first point above sigma_1 (count 2k + 1, plus
    // the padding) and the one before it bound the next round (seven rounds
    // reach a few ulps)
    if (wave == 0) {
      double gb = 0.0;
      for (int r = lane; r <= 2 * k; r += 64) {
        const double el = r > 0 ? (((r - 1) & 1) ? fabs(ab_b[(r - 1) >> 1]) : fabs(ab_a[(r - 1) >> 1])) : 0.0;
        const double er = r < 2 * k ? ((r & 1) ? fabs(ab_b[r >> 1]) : fabs(ab_a[r >> 1])) : 0.0;
        gb = fmax(gb, el + er);
      }
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) gb = fmax(gb, __shfl_xor(gb, m));
      if (lane == 0) { s_lo = 0.0; s_hi = gb * (1.0 + 8.0 * DBL_EPSILON); }
    }
    __syncthreads();
    for (int round = 0; round < 12; ++round) {
      const double lo = s_lo, hi = s_hi;
      if (!(hi - lo > 4.0 * DBL_EPSILON * hi)) break;
      const double h = (hi - lo) / (double)(kMS + 1);
      if (tid < kMS) {
        const bool above = gk_count_below(lo + h * (double)(tid + 1), n2, e2, 1.0 / hi) >= n2 + 1;
        const unsigned long long m = __ballot(above);
        if (lane == 0) wfirst[wave] = m ? wave * 64 + __builtin_ctzll(m) : kMS;
      }
      __syncthreads();
      if (tid == 0) {
        int j = kMS;
        for (int w = 0; w < kMS / 64; ++w) j = min(j, wfirst[w]);
        s_lo = j == 0 ? lo : lo + h * (double)j;
        s_hi = j == kMS ? hi : lo + h * (double)(j + 1);
      }
      __syncthreads();
    }
    const double sig1 = 0.5 * (s_lo + s_hi);
    if (!(sig1 > 0.0)) {
      lam = 0.0;
    } else if (a.gcv_mode == 2) {
      // The discrepancy principle: lambda with ||beta e_1 - C~ y_lambda|| equal
      // to the target.  The residual increases with lambda: the range
      // [1e-8 sigma_1, sigma_1] of t = log10(lambda) is cut in passes of np
      // points (one per thread), keeping the cell where the residual first
      // reaches the target, until it is narrower than 1e-12; the ends of the
      // range are returned for targets outside it.
      const double tt2 = a.target * a.target;
      const int nb = min(kRP, kRecD / (2 * k));
      const double t1 = log10(sig1), t0 = t1 - 8.0;
      if (tid < 2) {
        double r2;
        (void)gk_gcv(exp10(tid == 0 ? t0 : t1), k, ab_a, ab_b, beta, rec + tid, rec + k * 2 + tid, 2, nullptr, &r2);
        refv[tid] = r2;
      }
      __syncthreads();
      const double r2a = refv[0], r2b = refv[1];
      if (!(r2a < tt2)) {
        lam = exp10(t0);
      } else if (!(r2b > tt2)) {
        lam = exp10(t1);
      } else {
        if (tid == 0) { s_ra = t0; s_rb = t1; }
        __syncthreads();
        for (int pass = 0; pass < 12; ++pass) {
          const double ra = s_ra, rb = s_rb;
          if (!(rb - ra > 1e-12)) break;
          const double h = (rb - ra) / (double)(nb + 1);
          __syncthreads();  // every thread has read the bracket
          if (tid < nb) {
            double r2;
            (void)gk_gcv(exp10(ra + (double)(tid + 1) * h), k, ab_a, ab_b, beta, rec + tid, rec + k * nb + tid, nb,
                         nullptr, &r2);
            refv[tid] = r2;
          }
          __syncthreads();
          if (tid < 64) {
            // first point whose residual reaches the target (nb: none)
            int fi = nb;
            for (int i = lane; i < nb; i += 64)
              if (!(refv[i] < tt2)) { fi = i; break; }
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) fi = min(fi, __shfl_xor(fi, m));
            if (lane == 0) {
              s_ra = fi == 0 ? ra : ra + (double)fi * h;
              s_rb = fi == nb ? rb : ra + (double)(fi + 1) * h;
            }
          }
          __syncthreads();
        }
        lam = exp10(0.5 * (s_ra + s_rb));
      }
    } else {
      // the 400-point grid, as many lambdas per pass as the row storage holds
      // (each thread reuses its own slot: no barrier between passes)
      const double t0 = log10(sig1) - 8.0;
      const double dt = 8.0 / (double)(kGrid - 1);
      const int nb = min(kGrid, kRecD / (2 * k));
      for (int base = 0; base < kGrid; base += nb) {
        const int i = base + tid;
        if (tid < nb && i < kGrid)
          gridv[i] = gk_gcv(exp10(t0 + (double)i * dt), k, ab_a, ab_b, beta, rec + tid, rec + k * nb + tid, nb,
                            nullptr);
      }
      __syncthreads();
      // first index of the grid minimum (NaN counts as +inf)
      if (wave == 0) {
        int bi = kGrid;
        double bv = __builtin_inf();
        for (int i = lane; i < kGrid; i += 64) {
          const double v = gridv[i] == gridv[i] ? gridv[i] : __builtin_inf();
          if (bi == kGrid || v < bv) { bi = i; bv = v; }
        }
        first_min64(bv, bi);
        const int ib = bi < kGrid ? bi : 0;
        if (lane == 0) {
          wfirst[0] = ib;
          s_ra = t0 + (double)(ib > 0 ? ib - 1 : 0) * dt;
          s_rb = t0 + (double)(ib < kGrid - 1 ? ib + 1 : kGrid - 1) * dt;
          s_rt = __builtin_nan("");
          s_rf = __builtin_inf();
        }
      }
      __syncthreads();
      const int ib = wfirst[0];
      // Refinement on t = log10(lambda) inside the grid cells next to the
      // minimum: one pass of np points evenly inside [a, b] (one per thread),
      // keeping the two cells next to the first smallest value (a bracket of
      // ~1/100 of a grid cell), then the vertex of the parabola through the
      // smallest value and its two neighbours (its error, third order in the
      // spacing, leaves the GCV value at the minimum's to ~1e-15).
      const int np = min(nb, kRP);
      for (int pass = 0; pass < 1; ++pass) {
        const double ra = s_ra, rb = s_rb;
        const double h = (rb - ra) / (double)(np + 1);
        if (tid < np) {
          const double f = gk_gcv(exp10(ra + (double)(tid + 1) * h), k, ab_a, ab_b, beta, rec + tid,
                                  rec + k * np + tid, np, nullptr);
          refv[tid] = f == f ? f : __builtin_inf();
        }
        __syncthreads();
        if (tid < 64) {
          int mi = np;
          double mv = __builtin_inf();
          for (int i = lane; i < np; i += 64) {
            if (mi == np || refv[i] < mv) { mi = i; mv = refv[i]; }
          }
          first_min64(mv, mi);
          if (lane == 0) {
            mi = mi < np ? mi : 0;
            s_ra = ra + (double)mi * h;          // point mi - 1 (or a)
            s_rb = ra + (double)(mi + 2) * h;    // point mi + 1 (or b)
            s_rt = ra + (double)(mi + 1) * h;
            s_rf = refv[mi];
            s_fl = mi > 0 ? refv[mi - 1] : __builtin_nan("");
            s_fr = mi + 1 < np ? refv[mi + 1] : __builtin_nan("");
          }
        }
        __syncthreads();
      }
      if (tid != 0) return;
      double rt = s_rt, rf = s_rf;
      double y_t = __builtin_nan("");  // t whose y st->y holds
      {
        // parabola through (rt - h, fl), (rt, rf), (rt + h, fr): vertex offset
        // h (fl - fr) / (2 (fl - 2 rf + fr)) when the curvature is positive and
        // the vertex lies inside the bracket; kept if its value is smaller.
        // Its evaluation also writes y, kept when the vertex is the result.
        const double h = 0.5 * (s_rb - s_ra), fl = s_fl, fr = s_fr;
        const double cu = fl - 2.0 * rf + fr;
        if (cu > 0.0) {
          const double dv = 0.5 * h * (fl - fr) / cu;
          if (fabs(dv) < h) {
            const double tv = rt + dv;
            const double fv = gk_gcv(exp10(tv), k, ab_a, ab_b, beta, rec, rec + kMaxK, 1, st->y);
            y_t = tv;
            if (fv <= rf) { rt = tv; rf = fv; }
          }
        }
      }
      const double gv = gridv[ib];
      if (rf <= gv) { lam = exp10(rt); gcv = rf; y_done = (rt == y_t); }
      else { lam = exp10(t0 + (double)ib * dt); gcv = gv; }
      // a proposed lambda is kept when its GCV value is within the gate of the minimum
      if (lam_cand > 0.0) {
        const double fcand = gk_gcv(lam_cand, k, ab_a, ab_b, beta, rec, rec + kMaxK, 1, st->y);
        const bool keep = fcand <= gate * gcv;
        st->gate_ok = keep ? 1.0 : 0.0;
        if (keep) { lam = lam_cand; gcv = fcand; }
        y_done = keep;
      }
    }
  }
  if (tid != 0) return;
  if (y_done) {
  } else if (lam > 0.0) {
    // y_lambda from the same rotations as the GCV values (one lane)
    (void)gk_gcv(lam, k, ab_a, ab_b, beta, rec, rec + kMaxK, 1, st->y);
  } else {
    // lambda = 0: the recurrence with square roots and guarded divisions
    double* rho = rec;
    double* phi = rec + kMaxK;
    double* th = rec + 2 * kMaxK;
    double rbar = ab_a[0], fbar = beta;
    for (int i = 0; i < k; ++i) {
      const double rhat = fabs(rbar);
      const double fhat = rbar < 0.0 ? -fbar : fbar;
      const double bn = ab_b[i];
      const double r = sqrt(rhat * rhat + bn * bn);
      const double c = r > 0.0 ? rhat / r : 1.0, sn = r > 0.0 ? bn / r : 0.0;
      rho[i] = r;
      phi[i] = c * fhat;
      if (i + 1 < k) {
        th[i] = sn * ab_a[i + 1];
        rbar = -c * ab_a[i + 1];
      }
      fbar = sn * fhat;
    }
    double yn = 0.0;
    for (int i = k - 1; i >= 0; --i) {
      const double rhs = phi[i] - (i + 1 < k ? th[i] * yn : 0.0);
      yn = rho[i] > 0.0 ? rhs / rho[i] : 0.0;
      st->y[i] = yn;
    }
  }
  st->lambda = lam;
  st->gcv = gcv;
  st->sweeps = 0.0;
}

template <bool GROUPED>
__global__ __launch_bounds__(kPT) void k_projected_gk(ProjArgs a_, const ProjArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_projected_gk_body(a_, hw_block(), false);
  } else {
    VBlock vb;
    const ProjArgs g = group_args(grp, bmap, vb);
    k_projected_gk_body(g, vb, true);
  }
}

// ---- the L-curve of the stopping index -------------------------------------
// For k = 1..K (K = steps taken) the least-squares solution y_k of the leading
// (k+1) x k block of C~ (the LSQR iterate X_k = V_k y_k) by plane rotations,
// its residual |phibar_{k+1}| and norm ||y_k|| (one lane per k, the rows of
// the back substitution in LDS); the corner of (log ||R_k||, log ||X_k||) is
// the interior point of largest curvature of the circle through it and its
// neighbours (taken with the sign of a right turn, the curve being traced
// with the residual decreasing); y of the corner goes to st->y, zero beyond it.
__device__ inline void gk_ls(int k, const double* a, const double* b, double beta, double* q, double* w, int ld,
                             double& res, double& ynorm, double* yout) {
  double rbar = a[0], fbar = beta;
  for (int i = 0; i < k; ++i) {
    const double bn = b[i];
    const double r = sqrt(rbar * rbar + bn * bn);
    const double c = r > 0.0 ? rbar / r : 1.0, sn = r > 0.0 ? bn / r : 0.0;
    const double ir = r > 0.0 ? 1.0 / r : 0.0;
    q[i * ld] = (c * fbar) * ir;
    if (i + 1 < k) {
      w[i * ld] = (sn * a[i + 1]) * ir;
      rbar = -c * a[i + 1];
    }
    fbar = sn * fbar;
  }
  res = fabs(fbar);
  double yn = 0.0, nn = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    const double y = (i + 1 < k) ? q[i * ld] - w[i * ld] * yn : q[i * ld];
    nn = fma(y, y, nn);
    if (yout != nullptr) yout[i] = y;
    yn = y;
  }
  ynorm = sqrt(nn);
}

struct LcurveArgs {
  int gx, gy, gz;
  KState* st;
};

__device__ __forceinline__ void k_lcurve_body(const LcurveArgs& a, const VBlock vb, const bool grouped) {
  KState* st = a.st;
  if (ld_state(&st->halt)) return;
  __shared__ double rows[2 * kMaxK * 64];
  __shared__ double ab_a[kMaxK], ab_b[kMaxK], px[kMaxK], py[kMaxK];
  const int tid = threadIdx.x, lane = tid & 63;
  int K = st->steps;
  if (K > kMaxK) K = kMaxK;
  if (K <= 0) return;
  const double beta = st->beta[0];
  if (tid < K) {
    ab_a[tid] = st->alpha[tid];
    ab_b[tid] = st->beta[tid + 1];
  }
  __syncthreads();
  if (tid >= 64) return;
  if (lane < K) {
    double res, yn;
    gk_ls(lane + 1, ab_a, ab_b, beta, rows + lane, rows + kMaxK * 64 + lane, 64, res, yn, nullptr);
    px[lane] = log10(res);
    py[lane] = log10(yn);
  }
  // wave 0 only from here: its lanes' writes complete before any lane reads
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  double kap = 0.0;
  if (lane >= 1 && lane + 1 < K) {
    const double ax = px[lane] - px[lane - 1], ay = py[lane] - py[lane - 1];
    const double bx = px[lane + 1] - px[lane], by = py[lane + 1] - py[lane];
    const double cx = px[lane + 1] - px[lane - 1], cy = py[lane + 1] - py[lane - 1];
    const double den = sqrt(ax * ax + ay * ay) * sqrt(bx * bx + by * by) * sqrt(cx * cx + cy * cy);
    const double m = den > 0.0 ? 2.0 * (ax * by - ay * bx) / den : 0.0;
    kap = -m;
  }
  double bv = (kap > 0.0) ? kap : 0.0;  // NaN and non-positive: no corner
  int bi = (kap > 0.0) ? lane : 64;
  for (int m = 32; m >= 1; m >>= 1) {
    const double ov = __shfl_xor(bv, m);
    const int oi = __shfl_xor(bi, m);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  const int kopt = bi < 64 ? bi + 1 : K;  // 1-based
  if (lane == 0) {
    double res, yn;
    gk_ls(kopt, ab_a, ab_b, beta, rows, rows + kMaxK * 64, 1, res, yn, st->y);
    for (int i = kopt; i < K; ++i) st->y[i] = 0.0;
    st->lambda = 0.0;
    st->gcv = __builtin_nan("");
    st->sweeps = (double)kopt;
    st->resnorm = res;
  }
}

template <bool GROUPED>
__global__ __launch_bounds__(kPT) void k_lcurve(LcurveArgs a_, const LcurveArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    k_lcurve_body(a_, hw_block(), false);
  } else {
    VBlock vb;
    const LcurveArgs g = group_args(grp, bmap, vb);
    k_lcurve_body(g, vb, true);
  }
}

hipError_t launch_lcurve(dctk_ctx ctx, KState* st) {
  LcurveArgs a{};
  a.st = st;
  return launch_kernel(ctx, ctx->stream, k_lcurve<false>, k_lcurve<true>, dim3(1), kPT, 0, a);
}

hipError_t launch_projected_disc(dctk_ctx ctx, KState* st, double target, int k_use) {
  ProjArgs a{};
  a.bidiag = 1;
  a.gcv_mode = 2;
  a.k_use = k_use;
  a.st = st;
  a.lam_fixed = -1.0;
  a.lam_cand = -1.0;
  a.gate = 1.0;
  a.target = target;
  return launch_kernel(ctx, ctx->stream, k_projected_gk<false>, k_projected_gk<true>, dim3(1), kPT, 0, a);
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
  if (bidiag && (gcv_mode == 0 || lambda >= 0.0))
    return launch_kernel(ctx, ctx->stream, k_projected_gk<false>, k_projected_gk<true>, dim3(1), kPT, 0, a);
  return launch_kernel(ctx, ctx->stream, k_projected<false>, k_projected<true>, dim3(1), kPT, 0, a);
}

}  // namespace dctk
