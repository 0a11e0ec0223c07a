// The whole c-product of Algorithm 1 in one kernel, for one-sided operators
// with n3 = p <= 8 (colour images, short tubes):
//
//   step 1  X~_k = sum_t Lin[k][t] (s X_t)      computed while the X tile is
//           staged into LDS (each thread holds the p entries of its tubes);
//   step 2  C~_k = op(A~_k) X~_k                 16x16 MFMA blocks, all p slices
//           of an output tile in one workgroup, accumulated in registers;
//   step 3  Y_t  = a sum_k Lout[t][k] C~_k + b src_t    applied to the
//           accumulators (each lane holds the same (row, col) of every slice),
//           with per-workgroup partial sums of Y^2 for the next Krylov norm.
//
// The forward transform of the input and the inverse transform of the output
// never touch HBM, so one product reads A~, X (and src) once and writes Y once.
// Small problems (fewer 32x32 tiles than CUs) use 16x16 tiles with the 4 waves
// splitting the contraction (reduced through LDS) so every CU has work;
// larger ones use 32x32 or 64x64 tiles with 2x2 waves.
#include "mfma.h"

namespace dctk {

struct FusedArgs {
  int gx, gy, gz;          // this instance's grid (tiles along N, M)
  int p, M, N, K;          // output rows, columns, contraction length
  int64_t lda, sA;         // A~ slice: row stride and slice stride
  const void* A;
  const void* X;           // p x K x N vector type
  void* Y;                 // p x M x N vector type
  const void* src;         // p x M x N or null
  void* xnorm;             // p x K x N or null: receives s X
  const void* Gin;         // p x p, vector type
  const void* Gout;        // p x p, vector type
  Ctl ctl;
};

// XCD-aware tile order.  Workgroups are dealt to the 8 XCDs round robin in
// dispatch order (x fastest), and each XCD has its own L2.  When the grid
// splits into 2 x 4 equal regions, XCD r is given region r, so an XCD reads
// half of the A~ rows and a quarter of the X columns instead of all A~ rows;
// otherwise (and in grouped launches, whose workgroups are not aligned to the
// XCD rotation) the plain order is kept.
__device__ inline void xcd_tile(const VBlock& vb, bool grouped, int gx, int gy, int& tx, int& ty) {
  tx = vb.x;
  ty = vb.y;
  if (grouped || gx % 4 != 0 || gy % 2 != 0) return;
  const int lin = vb.y * gx + vb.x;
  const int xcd = lin & 7, slot = lin >> 3;
  const int rw = gx / 4, rh = gy / 2;  // region size in tiles; rw * rh = slots per XCD
  tx = (xcd & 3) * rw + slot % rw;
  ty = (xcd >> 2) * rh + slot / rw;
}

// EXACT: p == PMAX (no slice guards); otherwise p <= PMAX at run time.
// The A~ operand always has its contraction index contiguous in memory: the
// forward product reads the slices of A~, the adjoint the transposed copy the
// operator keeps for 16-bit GEMM types, so both stage 16-byte rows of 8
// consecutive k.  VEC: those rows, and X along n, move as 16-byte vectors (K
// and the A~ strides multiples of 8, N a multiple of 4, 16-byte aligned
// bases); else element by element.
template <typename TI, typename TV, int PMAX, bool EXACT, int BM, int BN, int WK, int BK, bool VEC>
__device__ __forceinline__ void cprod_fused_kernel_body(const FusedArgs& fa, const VBlock vb, const bool grouped) {
  typedef Mfma<TI> MF;
  typedef typename MF::acc_t acc_t;
  typedef typename MF::frag_t frag_t;
  constexpr int KSTEP = MF::KSTEP;
  static_assert(sizeof(TI) == 2 && MF::EPL == 8, "16-bit MFMA operands");
  static_assert(BK % KSTEP == 0, "BK");
  constexpr int BKT = BK * WK;                // contraction chunk staged per iteration
  constexpr int PAD = 8;                      // 16-byte row padding
  constexpr int LD = BKT + PAD;
  constexpr int WGM = (WK == 1) ? 2 : 1;      // waves along M / N
  constexpr int WGN = (WK == 1) ? 2 : 1;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(WK == 1 || WK == 4, "WK");
  static_assert(FM >= 1 && FN >= 1, "tile");
  static_assert(BKT % 8 == 0, "chunk");

  // both operands as [slice][row][k] with k contiguous: each lane's MFMA
  // operand (8 consecutive k of one row) is one 16-byte LDS read
  // (one buffer, reused by the cross-wave reduction)
  __shared__ __attribute__((aligned(16))) TI smem[PMAX * (BM + BN) * LD];
  TI* const As = smem;
  TI* const Bs = smem + PMAX * BM * LD;
  __shared__ TV sGin[PMAX * PMAX], sGout[PMAX * PMAX];
  __shared__ double sh[kShCtl];

  static_assert(PMAX * PMAX <= 256, "one transform entry per thread");
  const int p = EXACT ? PMAX : fa.p;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // The transform matrices (to registers, stored to LDS after the control
  // block), the first chunk and the control block's values are loaded in one
  // go, so the kernel waits for memory once before the first store.
  const bool gown = tid < p * p;
  const TV gin_r = ((const TV*)fa.Gin)[gown ? tid : 0];
  const TV gout_r = ((const TV*)fa.Gout)[gown ? tid : 0];

  // offsets are 32-bit from the base pointers (the host checks that every
  // tensor has < 2^31 elements)
  const int M = fa.M, N = fa.N, K = fa.K;
  const int sA = (int)fa.sA, lda = (int)fa.lda;
  int tx, ty;
  xcd_tile(vb, grouped, fa.gx, fa.gy, tx, ty);
  const int m0 = ty * BM, n0 = tx * BN;
  const TI* A = (const TI*)fa.A;
  const TV* X = (const TV*)fa.X;
  TV* xnorm = (ty == 0) ? (TV*)fa.xnorm : nullptr;

  const int wk = (WK == 1) ? 0 : wave;
  const int wmn = (WK == 1) ? wave : 0;
  const int wm = wmn >> 1, wn = wmn & 1;
  const int lr = lane & 15;
  const int lk = (lane >> 4) * MF::EPL;

  frag_t acc[PMAX][FM][FN];
#pragma unroll
  for (int k = 0; k < PMAX; ++k)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[k][i][j][r] = (acc_t)0;

  // Staging.  A~: units of 8 consecutive k of one row of one slice (one
  // 16-byte row segment).  X: units of 4 consecutive n x 4 consecutive k of
  // all p tubes (16-byte loads along n, coalesced across lanes), transformed,
  // rounded and written to LDS as 8-byte row segments of the p slices.  All
  // global loads of the next chunk are issued into registers before the
  // current chunk is multiplied.
  struct H4 { TI v[4]; };
  constexpr int KG = BKT / 8;
  constexpr int A_UN = PMAX * BM * KG, X_UN = (BKT / 4) * (BN / 4);
  constexpr int A_PER = (A_UN + 255) / 256, X_PER = (X_UN + 255) / 256;
  uint4 ra[A_PER];
  TV rx[X_PER][4][PMAX][4];
  TV sc = (TV)1;  // input scale, set by the control block before the first store
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int u = 0; u < A_PER; ++u) {
      const int idx = tid + u * 256;
      const int k = idx / (BM * KG);
      const int rem = idx - k * (BM * KG);
      const int r = rem / KG, kg = rem - r * KG;
      const int gm = m0 + r, gk = k0 + kg * 8;
      // clamped address + select: every load is issued, none is out of bounds
      const bool ok = (A_UN % 256 == 0 || idx < A_UN) && k < p && gm < M && gk < K;
      const int off = ok ? k * sA + gm * lda + gk : 0;
      if constexpr (VEC) {
        const uint4 v = *reinterpret_cast<const uint4*>(A + off);
        ra[u] = ok ? v : make_uint4(0u, 0u, 0u, 0u);
      } else {
        struct { TI v[8]; } h;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const bool oki = ok && gk + i < K;
          const TI v = A[oki ? off + i : 0];
          h.v[i] = oki ? v : (TI)0;
        }
        ra[u] = __builtin_bit_cast(uint4, h);
      }
    }
#pragma unroll
    for (int u = 0; u < X_PER; ++u) {
      const int idx = tid + u * 256;
      const int kq = idx / (BN / 4), nq = idx - kq * (BN / 4);
      const int gk = k0 + kq * 4, gn = n0 + nq * 4;
      const bool in = (X_UN % 256 == 0 || idx < X_UN) && gn < N;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int t = 0; t < PMAX; ++t) {
          const bool ok = in && t < p && gk + kk < K;
          const int off = ok ? (t * K + gk + kk) * N + gn : 0;
          if constexpr (VEC) {
            VecIO<TV, 4>::ld(X + off, rx[u][kk][t]);
            if (!ok) {
#pragma unroll
              for (int v = 0; v < 4; ++v) rx[u][kk][t][v] = (TV)0;
            }
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const bool okv = ok && gn + v < N;
              const TV x = X[okv ? off + v : 0];
              rx[u][kk][t][v] = okv ? x : (TV)0;
            }
          }
        }
    }
  };
  auto store_chunk = [&](int k0) {
#pragma unroll
    for (int u = 0; u < A_PER; ++u) {
      const int idx = tid + u * 256;
      if (A_UN % 256 == 0 || idx < A_UN) {
        const int k = idx / (BM * KG);
        const int rem = idx - k * (BM * KG);
        const int r = rem / KG, kg = rem - r * KG;
        *reinterpret_cast<uint4*>(&As[(k * BM + r) * LD + kg * 8]) = ra[u];
      }
    }
#pragma unroll
    for (int u = 0; u < X_PER; ++u) {
      const int idx = tid + u * 256;
      if (X_UN % 256 == 0 || idx < X_UN) {
        const int kq = idx / (BN / 4), nq = idx - kq * (BN / 4);
        const int gk = k0 + kq * 4, gn = n0 + nq * 4;
        TV xv[4][PMAX][4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int t = 0; t < PMAX; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) xv[kk][t][v] = sc * rx[u][kk][t][v];
        if (xnorm != nullptr && gn < N) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            if (gk + kk < K) {
#pragma unroll
              for (int t = 0; t < PMAX; ++t) {
                if (t < p) {
                  TV* q = xnorm + (t * K + gk + kk) * N + gn;
                  if constexpr (VEC) {
                    VecIO<TV, 4>::st(q, xv[kk][t]);
                  } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                      if (gn + v < N) q[v] = xv[kk][t][v];
                  }
                }
              }
            }
        }
#pragma unroll
        for (int k = 0; k < PMAX; ++k) {
          if (k < p) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              H4 h;
#pragma unroll
              for (int kk = 0; kk < 4; ++kk) {
                TV s = (TV)0;
#pragma unroll
                for (int t = 0; t < PMAX; ++t)
                  if (t < p) s += sGin[k * p + t] * xv[kk][t][v];
                h.v[kk] = cvt<TI, TV>(s);
              }
              *reinterpret_cast<uint2*>(&Bs[(k * BN + nq * 4 + v) * LD + kq * 4]) = __builtin_bit_cast(uint2, h);
            }
          }
        }
      }
    }
  };

  load_chunk(0);
  const CtlLoad cl = ctl_load(fa.ctl);
  double a_d, b_d, s_d;
  if (!ctl_eval(fa.ctl, cl, a_d, b_d, s_d, sh, vb)) return;
  sc = (TV)s_d;
  if (gown) {
    sGin[tid] = gin_r;
    sGout[tid] = gout_r;
  }
  for (int k0 = 0; k0 < K; k0 += BKT) {
    __syncthreads();
    store_chunk(k0);
    __syncthreads();
    if (k0 + BKT < K) load_chunk(k0 + BKT);
    const int kb = wk * BK, ke = (WK == 1) ? BKT : kb + BK;
    for (int ks = kb; ks < ke; ks += KSTEP) {
#pragma unroll
      for (int k = 0; k < PMAX; ++k) {
        if (k < p) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
              const TI* ap = &As[(k * BM + wm * WM + i * 16 + lr) * LD + ks + lk];
              const TI* bp = &Bs[(k * BN + wn * WN + j * 16 + lr) * LD + ks + lk];
              acc[k][i][j] = MF::mac(ap, bp, acc[k][i][j]);
            }
        }
      }
    }
  }

  // Epilogue.  Output element (i, j, r) of this lane: row m0 + wm WM + 16 i +
  // 4 (lane / 16) + r, column n0 + wn WN + 16 j + lane % 16.  With a split
  // contraction (WK = 4) the four waves' partial accumulators are summed
  // through LDS and wave w finishes register r = w, so all four waves share
  // the epilogue.
  constexpr int RN = (WK == 4) ? 1 : 4;  // accumulator registers finished by this wave
  auto out_row = [&](int i, int r) { return m0 + wm * WM + i * 16 + (lane >> 4) * 4 + r; };
  const int rbase = (WK == 4) ? wave : 0;
  const TV a = (TV)a_d, b = (TV)b_d;
  const TV* src = (const TV*)fa.src;
  TV* Y = (TV*)fa.Y;
  // prefetch the epilogue's src values (independent of the accumulators).  src
  // is null whenever b = 0, so the loads are issued only when both are set;
  // inside, out-of-range positions load element 0 of the (non-null) src.
  TV sv[FM][FN][RN][PMAX];
  const bool use_src = src != nullptr && b != (TV)0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int rr = 0; rr < RN; ++rr)
#pragma unroll
        for (int t = 0; t < PMAX; ++t) sv[i][j][rr][t] = (TV)0;
  if (use_src) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int col = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
        for (int rr = 0; rr < RN; ++rr) {
          const int row = out_row(i, rbase + rr);
#pragma unroll
          for (int t = 0; t < PMAX; ++t) {
            const bool ok = t < p && row < M && col < N;
            const TV v = src[ok ? (t * M + row) * N + col : 0];
            sv[i][j][rr][t] = ok ? v : (TV)0;
          }
        }
      }
  }

  TV accf[PMAX][FM][FN][RN];
  if constexpr (WK == 4) {
    constexpr int SLOT = 64 * 4;  // one slice of one wave: 64 lanes x 4 registers
    static_assert(sizeof(smem) >= sizeof(acc_t) * 4 * PMAX * SLOT, "LDS too small for the cross-wave reduction");
    acc_t* red = reinterpret_cast<acc_t*>(smem);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(wave * PMAX + k) * SLOT + r * 64 + lane] = acc[k][0][0][r];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      acc_t v = (acc_t)0;
#pragma unroll
      for (int w = 0; w < 4; ++w) v += red[(w * PMAX + k) * SLOT + wave * 64 + lane];
      accf[k][0][0][0] = (TV)v;
    }
  } else {
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) accf[k][i][j][r] = (TV)acc[k][i][j][r];
  }

  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int rr = 0; rr < RN; ++rr) {
        const int row = out_row(i, rbase + rr);
        if (row < M && col < N) {
#pragma unroll
          for (int t = 0; t < PMAX; ++t) {
            if (t >= p) break;
            TV y = (TV)0;
#pragma unroll
            for (int k = 0; k < PMAX; ++k)
              if (k < p) y += sGout[t * p + k] * accf[k][i][j][rr];
            const TV v = a * y + b * sv[i][j][rr][t];
            Y[(t * M + row) * N + col] = v;
            sq += (double)v * (double)v;
          }
        }
      }
    }
  if (fa.ctl.part_out != nullptr) {
    // one partial per wave (no block-wide exchange), by tile: the same order
    // under any tile mapping
    const double tot = wave_sum(sq);
    if (lane == 0) fa.ctl.part_out[(ty * fa.gx + tx) * 4 + wave] = tot;
  }
}

template <typename TI, typename TV, int PMAX, bool EXACT, int BM, int BN, int WK, int BK, bool VEC, bool GROUPED>
__global__ __launch_bounds__(256) void cprod_fused_kernel(FusedArgs fa_, const FusedArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    cprod_fused_kernel_body<TI, TV, PMAX, EXACT, BM, BN, WK, BK, VEC>(fa_, hw_block(), false);
  } else {
    VBlock vb;
    const FusedArgs g = group_args(grp, bmap, vb);
    cprod_fused_kernel_body<TI, TV, PMAX, EXACT, BM, BN, WK, BK, VEC>(g, vb, true);
  }
}

// ---- FP32 / FP64: row-index-contiguous staging with 16-byte vectors ---------
// The A~ and X~ tiles are staged as [slice][k][m] and [slice][k][n], so the
// MFMA operand reads (16 consecutive rows per lane group) are conflict free and
// X, whose rows are contiguous in n, moves as VW-element vectors from HBM to
// LDS with the tube transform applied in between.  Offsets are 32-bit from the
// base pointers (the host checks that every tensor has < 2^31 elements).

template <typename T, int PMAX, bool EXACT, int BM, int BN, int WK, int BK, bool TA, int VW>
__device__ __forceinline__ void cprod_fused_mn_kernel_body(const FusedArgs& fa, const VBlock vb, const bool grouped) {
  typedef Mfma<T> MF;
  typedef typename MF::acc_t acc_t;
  typedef typename MF::frag_t frag_t;
  constexpr int KSTEP = MF::KSTEP;
  static_assert(KSTEP == 4 && MF::EPL == 1, "32/64-bit MFMA only");
  static_assert(BK % KSTEP == 0, "BK");
  constexpr int BKT = BK * WK;
  constexpr int PADM = (BM == 16 || sizeof(T) == 8) ? 0 : 16;  // bank offset between k rows
  constexpr int PADN = (BN == 16 || sizeof(T) == 8) ? 0 : 16;
  constexpr int LDM = BM + PADM, LDN = BN + PADN;
  constexpr int WGM = (WK == 1) ? 2 : 1, WGN = (WK == 1) ? 2 : 1;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(WK == 1 || WK == 4, "WK");
  static_assert(FM >= 1 && FN >= 1, "tile");
  static_assert(BM % VW == 0 && BN % VW == 0 && BKT % VW == 0, "vector width");

  // one LDS buffer: the A~ and X~ tiles, reused by the cross-wave reduction.
  // A~ layout: TA -> [slice][k][m] (rows of A~_k read along m); else
  // [slice][m][k] with a pad of 16 bytes per row, so that both the 16-byte
  // row stores and the MFMA operand reads (16 rows x 4 k per instruction)
  // fall in distinct banks.
  constexpr int LDK = BKT + 16 / (int)sizeof(T);
  constexpr int A_LDS = TA ? PMAX * BKT * LDM : PMAX * BM * LDK;
  constexpr int ASTEP = TA ? 16 : 16 * LDK;  // next 16 output rows
  __shared__ __attribute__((aligned(16))) T smem[A_LDS + PMAX * BKT * LDN];
  T* const As = smem;
  T* const Bs = smem + A_LDS;
  __shared__ T sGin[PMAX * PMAX], sGout[PMAX * PMAX];
  __shared__ double sh[kShCtl];

  const int p = EXACT ? PMAX : fa.p;
  const int M = fa.M, N = fa.N, K = fa.K;
  const int lda = (int)fa.lda, sA = (int)fa.sA;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // The transform matrices (to registers, stored to LDS after the control
  // block), the first chunk and the control block's values are loaded in one
  // go, so the kernel waits for memory once before the first store.
  static_assert(PMAX * PMAX <= 256, "one transform entry per thread");
  const bool gown = tid < p * p;
  const T gin_r = ((const T*)fa.Gin)[gown ? tid : 0];
  const T gout_r = ((const T*)fa.Gout)[gown ? tid : 0];
  int tx, ty;
  xcd_tile(vb, grouped, fa.gx, fa.gy, tx, ty);
  const int m0 = ty * BM, n0 = tx * BN;
  const T* A = (const T*)fa.A;
  const T* X = (const T*)fa.X;
  T* xnorm = (ty == 0) ? (T*)fa.xnorm : nullptr;

  const int wk = (WK == 1) ? 0 : wave;
  const int wmn = (WK == 1) ? wave : 0;
  const int wm = wmn >> 1, wn = wmn & 1;
  const int lr = lane & 15;
  const int lk = lane >> 4;

  frag_t acc[PMAX][FM][FN];
#pragma unroll
  for (int k = 0; k < PMAX; ++k)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[k][i][j][r] = (acc_t)0;

  // A~ vectors: TA -> along m ([k][m] rows of the transposed slice); else along k
  constexpr int AV_ROW = TA ? BM / VW : BKT / VW;            // vectors per contiguous row
  constexpr int A_V = PMAX * (TA ? BKT : BM) * AV_ROW;       // vectors per chunk
  constexpr int A_PER = (A_V + 255) / 256;
  constexpr int X_V = BKT * (BN / VW);                       // tube-vector positions per chunk
  constexpr int X_PER = (X_V + 255) / 256;
  T ra[A_PER][VW];
  T rx[X_PER][PMAX][VW];

  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int u = 0; u < A_PER; ++u) {
      const int idx = tid + u * 256;
      const int k = idx / ((TA ? BKT : BM) * AV_ROW);
      const int rem = idx - k * ((TA ? BKT : BM) * AV_ROW);
      const int row = rem / AV_ROW, cv = (rem - row * AV_ROW) * VW;
      // TA: row = kk, cv = m offset; else row = m, cv = kk offset
      const int gm = m0 + (TA ? cv : row), gk = k0 + (TA ? row : cv);
      const bool ok = (A_V % 256 == 0 || idx < A_V) && k < p && gm < M && gk < K;
      const int off = ok ? k * sA + (TA ? gk * lda + gm : gm * lda + gk) : 0;
      VecIO<T, VW>::ld(A + off, ra[u]);
      if (!ok) {
#pragma unroll
        for (int v = 0; v < VW; ++v) ra[u][v] = (T)0;
      }
    }
#pragma unroll
    for (int u = 0; u < X_PER; ++u) {
      const int idx = tid + u * 256;
      const int kk = idx / (BN / VW), nv = (idx - kk * (BN / VW)) * VW;
      const int gk = k0 + kk, gn = n0 + nv;
      const bool in = (X_V % 256 == 0 || idx < X_V) && gk < K && gn < N;
#pragma unroll
      for (int t = 0; t < PMAX; ++t) {
        const bool ok = in && t < p;
        VecIO<T, VW>::ld(X + (ok ? (t * K + gk) * N + gn : 0), rx[u][t]);
        if (!ok) {
#pragma unroll
          for (int v = 0; v < VW; ++v) rx[u][t][v] = (T)0;
        }
      }
    }
  };
  T sc = (T)1;  // input scale, set by the control block before the first store
  auto store_chunk = [&](int k0) {
#pragma unroll
    for (int u = 0; u < A_PER; ++u) {
      const int idx = tid + u * 256;
      if (A_V % 256 == 0 || idx < A_V) {
        const int k = idx / ((TA ? BKT : BM) * AV_ROW);
        const int rem = idx - k * ((TA ? BKT : BM) * AV_ROW);
        const int row = rem / AV_ROW, cv = (rem - row * AV_ROW) * VW;
        if (TA)
          VecIO<T, VW>::st(&As[(k * BKT + row) * LDM + cv], ra[u]);
        else
          VecIO<T, VW>::st(&As[(k * BM + row) * LDK + cv], ra[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < X_PER; ++u) {
      const int idx = tid + u * 256;
      if (X_V % 256 == 0 || idx < X_V) {
        const int kk = idx / (BN / VW), nv = (idx - kk * (BN / VW)) * VW;
        const int gk = k0 + kk, gn = n0 + nv;
        T xv[PMAX][VW];
#pragma unroll
        for (int t = 0; t < PMAX; ++t)
#pragma unroll
          for (int v = 0; v < VW; ++v) xv[t][v] = sc * rx[u][t][v];
        if (xnorm != nullptr && gk < K && gn < N) {
#pragma unroll
          for (int t = 0; t < PMAX; ++t)
            if (t < p) VecIO<T, VW>::st(xnorm + (t * K + gk) * N + gn, xv[t]);
        }
#pragma unroll
        for (int k = 0; k < PMAX; ++k) {
          if (k < p) {
            T h[VW];
#pragma unroll
            for (int v = 0; v < VW; ++v) h[v] = (T)0;
#pragma unroll
            for (int t = 0; t < PMAX; ++t) {
              if (t < p) {
                const T g = sGin[k * p + t];
#pragma unroll
                for (int v = 0; v < VW; ++v) h[v] += g * xv[t][v];
              }
            }
            VecIO<T, VW>::st(&Bs[(k * BKT + kk) * LDN + nv], h);
          }
        }
      }
    }
  };

  load_chunk(0);
  const CtlLoad cl = ctl_load(fa.ctl);
  double a_d, b_d, s_d;
  if (!ctl_eval(fa.ctl, cl, a_d, b_d, s_d, sh, vb)) return;
  sc = (T)s_d;
  if (gown) {
    sGin[tid] = gin_r;
    sGout[tid] = gout_r;
  }
  for (int k0 = 0; k0 < K; k0 += BKT) {
    __syncthreads();
    store_chunk(k0);
    __syncthreads();
    if (k0 + BKT < K) load_chunk(k0 + BKT);
    const int kb = wk * BK, ke = (WK == 1) ? BKT : kb + BK;
    for (int ks = kb; ks < ke; ks += KSTEP) {
#pragma unroll
      for (int k = 0; k < PMAX; ++k) {
        if (k < p) {
          const T* arow = TA ? &As[(k * BKT + ks + lk) * LDM + wm * WM + lr]
                             : &As[(k * BM + wm * WM + lr) * LDK + ks + lk];
          const T* brow = &Bs[(k * BKT + ks + lk) * LDN + wn * WN + lr];
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[k][i][j] = MF::mac(arow + i * ASTEP, brow + j * 16, acc[k][i][j]);
        }
      }
    }
  }

  // Epilogue.  Output element (i, j, r) of this lane: row m0 + wm WM + 16 i + rr(r),
  // column n0 + wn WN + 16 j + lane % 16.  With a split contraction (WK = 4) the
  // four waves' partial accumulators are summed through LDS and wave w finishes
  // register r = w, so all four waves share the epilogue.
  constexpr int RN = (WK == 4) ? 1 : 4;  // accumulator registers finished by this wave
  auto out_row = [&](int i, int r) {
    return m0 + wm * WM + i * 16 + (MF::ROWS_STRIDED ? (lane >> 4) + 4 * r : (lane >> 4) * 4 + r);
  };
  const int rbase = (WK == 4) ? wave : 0;
  const T a = (T)a_d, b = (T)b_d;
  const T* src = (const T*)fa.src;
  T* Y = (T*)fa.Y;
  // prefetch the epilogue's src values (independent of the accumulators).  src
  // is null whenever b = 0, so the loads are issued only when both are set;
  // inside, out-of-range positions load element 0 of the (non-null) src.
  T sv[FM][FN][RN][PMAX];
  const bool use_src = src != nullptr && b != (T)0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int rr = 0; rr < RN; ++rr)
#pragma unroll
        for (int t = 0; t < PMAX; ++t) sv[i][j][rr][t] = (T)0;
  if (use_src) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int col = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
        for (int rr = 0; rr < RN; ++rr) {
          const int row = out_row(i, rbase + rr);
#pragma unroll
          for (int t = 0; t < PMAX; ++t) {
            const bool ok = t < p && row < M && col < N;
            const T v = src[ok ? (t * M + row) * N + col : 0];
            sv[i][j][rr][t] = ok ? v : (T)0;
          }
        }
      }
  }

  T accf[PMAX][FM][FN][RN];
  if constexpr (WK == 4) {
    constexpr int SLOT = 64 * 4;  // one slice of one wave: 64 lanes x 4 registers
    static_assert(sizeof(smem) >= sizeof(acc_t) * 4 * PMAX * SLOT, "LDS too small for the cross-wave reduction");
    acc_t* red = reinterpret_cast<acc_t*>(smem);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(wave * PMAX + k) * SLOT + r * 64 + lane] = acc[k][0][0][r];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      acc_t v = (acc_t)0;
#pragma unroll
      for (int w = 0; w < 4; ++w) v += red[(w * PMAX + k) * SLOT + wave * 64 + lane];
      accf[k][0][0][0] = (T)v;
    }
  } else {
#pragma unroll
    for (int k = 0; k < PMAX; ++k)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) accf[k][i][j][r] = (T)acc[k][i][j][r];
  }

  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int rr = 0; rr < RN; ++rr) {
        const int row = out_row(i, rbase + rr);
        if (row < M && col < N) {
#pragma unroll
          for (int t = 0; t < PMAX; ++t) {
            if (t >= p) break;
            T y = (T)0;
#pragma unroll
            for (int k = 0; k < PMAX; ++k)
              if (k < p) y += sGout[t * p + k] * accf[k][i][j][rr];
            const T v = a * y + b * sv[i][j][rr][t];
            Y[(t * M + row) * N + col] = v;
            sq += (double)v * (double)v;
          }
        }
      }
    }
  if (fa.ctl.part_out != nullptr) {
    // one partial per wave (no block-wide exchange), by tile: the same order
    // under any tile mapping
    const double tot = wave_sum(sq);
    if (lane == 0) fa.ctl.part_out[(ty * fa.gx + tx) * 4 + wave] = tot;
  }
}

template <typename T, int PMAX, bool EXACT, int BM, int BN, int WK, int BK, bool TA, int VW, bool GROUPED>
__global__ __launch_bounds__(256) void cprod_fused_mn_kernel(FusedArgs fa_, const FusedArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    cprod_fused_mn_kernel_body<T, PMAX, EXACT, BM, BN, WK, BK, TA, VW>(fa_, hw_block(), false);
  } else {
    VBlock vb;
    const FusedArgs g = group_args(grp, bmap, vb);
    cprod_fused_mn_kernel_body<T, PMAX, EXACT, BM, BN, WK, BK, TA, VW>(g, vb, true);
  }
}

// Where a fused product goes: the context (recording or not), its stream, and
// start/stop events (null unless the context is profiling) that the dispatch
// itself records, so the measured interval is the kernel's execution alone.
struct FusedLaunch {
  dctk_ctx ctx;
  hipStream_t s;
  hipEvent_t e0, e1;
  int tile;  // output tile edge chosen by the autotuner (16, 32, 64), 0: by problem size
};

template <typename T, int PMAX, bool EXACT, int BM, int BN, int WK, int BK>
static hipError_t launch_fused_mn_cfg(const FusedLaunch& L, const FusedArgs& fa, int ta, bool vec, int* nblocks_out) {
  dim3 grid((unsigned)((fa.N + BN - 1) / BN), (unsigned)((fa.M + BM - 1) / BM));
  // one norm partial per wave (256 threads: 4 waves)
  if (nblocks_out) *nblocks_out = (int)(grid.x * grid.y * 4);
  if ((int64_t)grid.x * grid.y * 4 > kNormParts && fa.ctl.part_out != nullptr) return hipErrorInvalidConfiguration;
  constexpr int VW = 16 / (int)sizeof(T);
#define DCTK_MN_LAUNCH(TA_, VW_) \
  launch_kernel(L.ctx, L.s, cprod_fused_mn_kernel<T, PMAX, EXACT, BM, BN, WK, BK, TA_, VW_, false>, cprod_fused_mn_kernel<T, PMAX, EXACT, BM, BN, WK, BK, TA_, VW_, true>, grid, 256, 0, fa, L.e0, L.e1)
  if (ta) return vec ? DCTK_MN_LAUNCH(true, VW) : DCTK_MN_LAUNCH(true, 1);
  return vec ? DCTK_MN_LAUNCH(false, VW) : DCTK_MN_LAUNCH(false, 1);
#undef DCTK_MN_LAUNCH
}

template <typename T, int PMAX, bool EXACT>
static hipError_t launch_fused_mn_p(const FusedLaunch& L, const FusedArgs& fa, int ta, bool vec, int* nblocks_out) {
  constexpr int BK = (sizeof(T) == 8) ? 8 : 16;
  // 16x16 tiles (small problems, latency bound): the whole contraction of a
  // 256-long K in one staged chunk when it fits in ~130 KB of LDS
  constexpr int BK16 = PMAX > 4 ? BK : (sizeof(T) == 8 ? 32 : 64);
  const int64_t t32 = (int64_t)((fa.M + 31) / 32) * ((fa.N + 31) / 32);
  const int64_t t64 = (int64_t)((fa.M + 63) / 64) * ((fa.N + 63) / 64);
  const int ncu = num_cus();
  if (L.tile == 16 || (L.tile == 0 && t32 < ncu))
    return launch_fused_mn_cfg<T, PMAX, EXACT, 16, 16, 4, BK16>(L, fa, ta, vec, nblocks_out);
  if (L.tile == 32 || (L.tile == 0 && (t64 < ncu || sizeof(T) == 8 || PMAX > 4)) || t64 > kRedBlocks)
    return launch_fused_mn_cfg<T, PMAX, EXACT, 32, 32, 1, BK>(L, fa, ta, vec, nblocks_out);
  return launch_fused_mn_cfg<T, PMAX, EXACT, 64, 64, 1, BK>(L, fa, ta, vec, nblocks_out);
}

template <typename T>
static hipError_t launch_fused_mn(const FusedLaunch& L, const FusedArgs& fa, int ta, int* nblocks_out) {
  constexpr int VW = 16 / (int)sizeof(T);
  const bool vec = fa.M % VW == 0 && fa.N % VW == 0 && fa.K % VW == 0 && fa.lda % VW == 0 &&
                   ((uintptr_t)fa.A % 16) == 0 && ((uintptr_t)fa.X % 16) == 0 &&
                   (fa.xnorm == nullptr || ((uintptr_t)fa.xnorm % 16) == 0);
  if (fa.p == 3) return launch_fused_mn_p<T, 3, true>(L, fa, ta, vec, nblocks_out);
  if (fa.p <= 4) return launch_fused_mn_p<T, 4, false>(L, fa, ta, vec, nblocks_out);
  return launch_fused_mn_p<T, 8, false>(L, fa, ta, vec, nblocks_out);
}

template <typename TI, typename TV, int PMAX, bool EXACT, int BM, int BN, int WK, int BK>
static hipError_t launch_fused_cfg(const FusedLaunch& L, const FusedArgs& fa, bool va, int* nblocks_out) {
  dim3 grid((unsigned)((fa.N + BN - 1) / BN), (unsigned)((fa.M + BM - 1) / BM));
  // one norm partial per wave (256 threads: 4 waves)
  if (nblocks_out) *nblocks_out = (int)(grid.x * grid.y * 4);
  if ((int64_t)grid.x * grid.y * 4 > kNormParts && fa.ctl.part_out != nullptr) return hipErrorInvalidConfiguration;
  if (va) return launch_kernel(L.ctx, L.s, cprod_fused_kernel<TI, TV, PMAX, EXACT, BM, BN, WK, BK, true, false>, cprod_fused_kernel<TI, TV, PMAX, EXACT, BM, BN, WK, BK, true, true>, grid, 256, 0, fa, L.e0, L.e1);
  return launch_kernel(L.ctx, L.s, cprod_fused_kernel<TI, TV, PMAX, EXACT, BM, BN, WK, BK, false, false>, cprod_fused_kernel<TI, TV, PMAX, EXACT, BM, BN, WK, BK, false, true>, grid, 256, 0, fa, L.e0, L.e1);
}

// Tile choice: 16x16 with a split contraction while 32x32 tiles would not
// cover the CUs, then 32x32, then 64x64 (p > 4 stays at 32x32, also under a
// tuned 64, to bound the registers).  Chunks: the whole 256-long contraction of the
// colour and batch shapes in one staged chunk of 16x16 tiles (p <= 4), LDS
// under ~85 KB everywhere.
template <typename TI, typename TV, int PMAX, bool EXACT>
static hipError_t launch_fused_p(const FusedLaunch& L, const FusedArgs& fa, bool va, int* nblocks_out) {
  static_assert(Mfma<TI>::KSTEP == 32, "16-bit MFMA");
  constexpr int BK16 = PMAX > 4 ? 32 : 64;
  constexpr int BK32 = 64;
  constexpr int BK64 = 64;
  const int64_t t32 = (int64_t)((fa.M + 31) / 32) * ((fa.N + 31) / 32);
  const int64_t t64 = (int64_t)((fa.M + 63) / 64) * ((fa.N + 63) / 64);
  const int ncu = num_cus();
  if (L.tile == 16 || (L.tile == 0 && t32 < ncu))
    return launch_fused_cfg<TI, TV, PMAX, EXACT, 16, 16, 4, BK16>(L, fa, va, nblocks_out);
  if (PMAX > 4 || L.tile == 32 || (L.tile == 0 && t64 < ncu) || t64 > kRedBlocks)
    return launch_fused_cfg<TI, TV, PMAX, EXACT, 32, 32, 1, BK32>(L, fa, va, nblocks_out);
  if constexpr (PMAX <= 4) return launch_fused_cfg<TI, TV, PMAX, EXACT, 64, 64, 1, BK64>(L, fa, va, nblocks_out);
  return hipErrorInvalidValue;
}

template <typename TI, typename TV>
static hipError_t launch_fused_t(const FusedLaunch& L, const FusedArgs& fa, int* nblocks_out) {
  const bool va = fa.K % 8 == 0 && fa.lda % 8 == 0 && fa.sA % 8 == 0 && ((uintptr_t)fa.A % 16) == 0 &&
                  fa.N % 4 == 0 && ((uintptr_t)fa.X % 16) == 0 &&
                  (fa.xnorm == nullptr || ((uintptr_t)fa.xnorm % 16) == 0);
  if (fa.p == 3) return launch_fused_p<TI, TV, 3, true>(L, fa, va, nblocks_out);  // colour images
  if (fa.p <= 4) return launch_fused_p<TI, TV, 4, false>(L, fa, va, nblocks_out);
  return launch_fused_p<TI, TV, 8, false>(L, fa, va, nblocks_out);
}

hipError_t launch_fused(dctk_op op, hipStream_t s, int adjoint, const void* X, void* Y, const void* src,
                        void* xnorm, const Ctl& ctl, int* nblocks_out) {
  FusedArgs fa;
  fa.p = (int)op->p;
  fa.M = (int)(adjoint ? op->n2 : op->n1);
  fa.K = (int)(adjoint ? op->n1 : op->n2);
  fa.N = (int)op->s;
  fa.lda = op->n2;
  fa.sA = op->n1 * op->n2;
  fa.A = op->Ah;
  const bool half = op->gemm_dtype == DCTK_BF16 || op->gemm_dtype == DCTK_F16;
  if (half && adjoint) {
    // 16-bit operands: the adjoint reads the transposed slices (n2 x n1)
    if (op->AhT == nullptr) return hipErrorInvalidValue;
    fa.A = op->AhT;
    fa.lda = op->n1;
  }
  fa.X = X;
  fa.Y = Y;
  fa.src = src;
  fa.xnorm = xnorm;
  const int64_t pp = op->p * op->p;
  const int gi = adjoint ? 2 : 0, go = adjoint ? 3 : 1;
  if (op->vec_dtype == DCTK_F64) {
    fa.Gin = op->Gd + gi * pp;
    fa.Gout = op->Gd + go * pp;
  } else {
    fa.Gin = op->Gf + gi * pp;
    fa.Gout = op->Gf + go * pp;
  }
  fa.ctl = ctl;
  FusedLaunch L{op->ctx, s, nullptr, nullptr, op->tune[adjoint ? 1 : 0][1]};
  if (!recording(op->ctx)) prof_kernel(op->ctx, adjoint ? PROF_FUSED_ADJ : PROF_FUSED_FWD, &L.e0, &L.e1);
  switch (op->gemm_dtype) {
    case DCTK_F64: return launch_fused_mn<double>(L, fa, adjoint, nblocks_out);
    case DCTK_F32: return launch_fused_mn<float>(L, fa, adjoint, nblocks_out);
    case DCTK_BF16: return launch_fused_t<bf16_t, float>(L, fa, nblocks_out);
    case DCTK_F16: return launch_fused_t<f16_t, float>(L, fa, nblocks_out);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dctk
