// Transform-domain frontal-slice products (Algorithm 1 step 2): the one
// dense contraction of the c-product, C~_k = op(A~_k) op(B~_k) for k < p,
// as batched GEMMs on the gfx950 matrix cores.
//
// Tile: BM x BN outputs per workgroup of 4 waves arranged 2 x 2, each wave
// owning (BM/2) x (BN/2) as 16 x 16 MFMA blocks.  Operands are staged through
// LDS as [rows][BK + pad] (contraction index contiguous) so each lane's MFMA
// operand is one LDS read: 1 element for the K = 4 FP32/FP64 instructions,
// 8 packed 16-bit elements for the K = 32 BF16/FP16 instructions of gfx950.
// Global loads are ordered along each operand's contiguous dimension; the
// next K-chunk is prefetched into registers while the current one is
// multiplied.  Ragged edges are zero-filled on load and masked on store.
#include <type_traits>

#include "fastdct.h"
#include "mfma.h"

namespace dctk {

// batches of at least this many slices are placed per XCD (slice_block)
constexpr int kSliceXcdMin = 16;

// threads of a 16-bit GEMM workgroup: 512 for 256 x 256 tiles, else 256
__host__ __device__ constexpr int gemm_threads(int bm, int bn) { return bm * bn >= 65536 ? 512 : 256; }

struct GemmArgs {
  int gx, gy, gz;
  int M, N, K;
  const void* A;
  int64_t lda, sA;
  const void* B;
  int64_t ldb, sB;
  void* C;
  int64_t ldc, sC;
  Gate g;
  int nbatch;   // > 0: slices placed per XCD (see slice_block); the grid's z is padded to 8 ceil(nbatch / 8)
};

// XCD-aware slice placement of a plain batched launch.  Workgroups are dealt to
// the 8 XCDs round robin in dispatch order, and each XCD has its own L2.  With
// T = gx gy tiles per slice, dispatch slot `lin` goes to XCD lin % 8 and is
// given tile (lin / 8) % T of slice 8 ((lin / 8) / T) + lin % 8: every tile of
// a slice runs on one XCD, in consecutive slots, so the slice's operands are
// fetched into one L2 instead of eight.  Padding slots (slice >= nbatch) exit.
__device__ inline bool slice_block(const GemmArgs& ga, VBlock& vb) {
  if (ga.nbatch <= 0) return true;
  const int64_t T = (int64_t)ga.gx * ga.gy;
  const int64_t lin = vb.x + (int64_t)ga.gx * (vb.y + (int64_t)ga.gy * vb.z);
  const int64_t slot = lin >> 3;
  const int64_t z = (slot / T) * 8 + (lin & 7);
  if (z >= ga.nbatch) return false;
  const int64_t t = slot % T;
  vb.x = (int)(t % ga.gx);
  vb.y = (int)(t / ga.gx);
  vb.z = (int)z;
  return true;
}

// VEC (16-bit types): operands move as 16-byte vectors of 8 elements along
// their contiguous dimension (multiples of 8, 16-byte aligned): an operand
// contiguous in k goes to its LDS rows as one 16-byte store, one contiguous
// in m (or n) is transposed on the way, as eight 2-byte stores into eight
// rows at one k.  All loads are issued from clamped addresses and selected.
template <typename TI, typename TO, int BM, int BN, bool TA, bool TB, bool VEC>
__device__ __forceinline__ void gemm_kernel_body(const GemmArgs& ga, const VBlock vb, const bool grouped) {
  const int M = ga.M, N = ga.N, K = ga.K;
  const TI* __restrict__ A = (const TI*)ga.A;
  const TI* __restrict__ B = (const TI*)ga.B;
  TO* __restrict__ C = (TO*)ga.C;
  const int64_t lda = ga.lda, sA = ga.sA, ldb = ga.ldb, sB = ga.sB, ldc = ga.ldc, sC = ga.sC;
  const Gate g = ga.g;
  typedef Mfma<TI> MF;
  typedef typename MF::acc_t acc_t;
  typedef typename MF::frag_t frag_t;
  constexpr int KSTEP = MF::KSTEP;
  // 256-row tiles: 32-wide contraction chunks (the two operand tiles of a
  // 256 x 128 chunk are 30 KB of LDS, so two workgroups share a CU)
  constexpr int BK = (KSTEP == 4) ? 16 : (BM >= 256 ? 32 : 64);
  constexpr int PAD = (sizeof(TI) == 2) ? 8 : (sizeof(TI) == 4 ? 4 : 2);  // 16 bytes
  constexpr int LDS_LD = BK + PAD;
  constexpr int NT = gemm_threads(BM, BN), WGM = 2, WGN = NT / 128;   // threads, wave grid
  constexpr int A_PER = (BM * BK + NT - 1) / NT;  // elements of the A tile per thread
  constexpr int B_PER = (BN * BK + NT - 1) / NT;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(A_PER >= 1 && B_PER >= 1, "tile too small");

  if (!gate_open(g)) return;

  __shared__ __attribute__((aligned(16))) TI As[BM * LDS_LD];
  __shared__ __attribute__((aligned(16))) TI Bs[BN * LDS_LD];

  const int bz = vb.z;
  const int m0 = vb.y * BM;
  const int n0 = vb.x * BN;
  A += (int64_t)bz * sA;
  B += (int64_t)bz * sB;
  C += (int64_t)bz * sC;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;

  // element (r, kk) of the A tile (r < BM, kk < BK) handled by this thread, slot u
  auto a_coord = [&](int u, int& r, int& kk) {
    int idx = tid + u * NT;
    if (!TA) { r = idx / BK; kk = idx % BK; }   // contiguous along k
    else     { kk = idx / BM; r = idx % BM; }   // contiguous along m
  };
  auto b_coord = [&](int u, int& c, int& kk) {
    int idx = tid + u * NT;
    if (!TB) { kk = idx / BN; c = idx % BN; }   // contiguous along n
    else     { c = idx / BK; kk = idx % BK; }   // contiguous along k
  };

  TI ra[A_PER], rb[B_PER];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int u = 0; u < A_PER; ++u) {
      int r, kk;
      a_coord(u, r, kk);
      int gm = m0 + r, gk = k0 + kk;
      TI v = (TI)0;
      if (gm < M && gk < K) v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < B_PER; ++u) {
      int c, kk;
      b_coord(u, c, kk);
      int gn = n0 + c, gk = k0 + kk;
      TI v = (TI)0;
      if (gn < N && gk < K) v = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      rb[u] = v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int u = 0; u < A_PER; ++u) {
      int r, kk;
      a_coord(u, r, kk);
      As[r * LDS_LD + kk] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < B_PER; ++u) {
      int c, kk;
      b_coord(u, c, kk);
      Bs[c * LDS_LD + kk] = rb[u];
    }
  };

  // vector staging (VEC).  An operand contiguous in k moves in units of 8 k
  // of one row (one 16-byte load and LDS store); an operand contiguous in its
  // rows moves in units of 8 rows x KU k (KU 16-byte loads), transposed in
  // registers into 8 rows of KU consecutive k (eight LDS stores of KU
  // elements).
  constexpr int KU = 8;
  struct H8 { TI v[8]; };
  struct HK { TI v[KU]; };
  typedef typename std::conditional<KU == 8, uint4, uint2>::type kvec_t;
  constexpr int A_NK = TA ? BM * BK / (8 * KU) : BM * BK / 8;   // units of the A tile
  constexpr int B_NK = TB ? BN * BK / 8 : BN * BK / (8 * KU);
  constexpr int A_UV = (A_NK + NT - 1) / NT, B_UV = (B_NK + NT - 1) / NT;
  constexpr int A_L = TA ? KU : 1, B_L = TB ? 1 : KU;       // 16-byte loads per unit
  uint4 va[A_UV][A_L], vbv[B_UV][B_L];
  // unit u of an operand tile of R rows: its first (row, k)
  auto unit = [&](int u, int R, bool kcontig, int& r, int& kk) {
    const int idx = tid + u * NT;
    if (kcontig) { r = idx / (BK / 8); kk = (idx % (BK / 8)) * 8; }
    else         { kk = (idx / (R / 8)) * KU; r = (idx % (R / 8)) * 8; }
  };
  auto load_vec = [&](int k0) {
#pragma unroll
    for (int u = 0; u < A_UV; ++u) {
      int r, kk;
      unit(u, BM, !TA, r, kk);
      const bool ok = A_NK % NT == 0 || tid + u * NT < A_NK;
#pragma unroll
      for (int l = 0; l < A_L; ++l) {
        const int gm = m0 + r, gk = k0 + kk + l;
        const bool in = ok && gm < M && gk < K;
        const int64_t off = in ? (TA ? (int64_t)gk * lda + gm : (int64_t)gm * lda + gk) : 0;
        const uint4 v = *reinterpret_cast<const uint4*>(A + off);
        va[u][l] = in ? v : make_uint4(0u, 0u, 0u, 0u);
      }
    }
#pragma unroll
    for (int u = 0; u < B_UV; ++u) {
      int c, kk;
      unit(u, BN, TB, c, kk);
      const bool ok = B_NK % NT == 0 || tid + u * NT < B_NK;
#pragma unroll
      for (int l = 0; l < B_L; ++l) {
        const int gn = n0 + c, gk = k0 + kk + l;
        const bool in = ok && gn < N && gk < K;
        const int64_t off = in ? (TB ? (int64_t)gn * ldb + gk : (int64_t)gk * ldb + gn) : 0;
        const uint4 v = *reinterpret_cast<const uint4*>(B + off);
        vbv[u][l] = in ? v : make_uint4(0u, 0u, 0u, 0u);
      }
    }
  };
  // 8 rows x KU k held as KU 16-byte rows along the operand's rows -> LDS
  auto put_t = [&](TI* S, int r, int kk, const uint4 (&q)[KU]) {
    H8 h[KU];
#pragma unroll
    for (int l = 0; l < KU; ++l) h[l] = __builtin_bit_cast(H8, q[l]);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      HK w;
#pragma unroll
      for (int l = 0; l < KU; ++l) w.v[l] = h[l].v[j];
      *reinterpret_cast<kvec_t*>(&S[(r + j) * LDS_LD + kk]) = __builtin_bit_cast(kvec_t, w);
    }
  };
  auto store_vec = [&]() {
#pragma unroll
    for (int u = 0; u < A_UV; ++u) {
      if (A_NK % NT != 0 && tid + u * NT >= A_NK) continue;
      int r, kk;
      unit(u, BM, !TA, r, kk);
      if constexpr (!TA) *reinterpret_cast<uint4*>(&As[r * LDS_LD + kk]) = va[u][0];
      else put_t(As, r, kk, va[u]);
    }
#pragma unroll
    for (int u = 0; u < B_UV; ++u) {
      if (B_NK % NT != 0 && tid + u * NT >= B_NK) continue;
      int c, kk;
      unit(u, BN, TB, c, kk);
      if constexpr (TB) *reinterpret_cast<uint4*>(&Bs[c * LDS_LD + kk]) = vbv[u][0];
      else put_t(Bs, c, kk, vbv[u]);
    }
  };

  frag_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = (acc_t)0;

  const int lr = lane & 15;          // row (A) / column (B) within a 16-block
  const int lk = (lane >> 4) * MF::EPL;  // first contraction index of this lane

  if constexpr (VEC) load_vec(0);
  else load_tiles(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    if constexpr (VEC) store_vec();
    else store_tiles();
    __syncthreads();
    // prefetch the next chunk into registers
    if constexpr (VEC) {
      if (k0 + BK < K) load_vec(k0 + BK);
    } else {
      if (k0 + BK < K) load_tiles(k0 + BK);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += KSTEP) {
      const TI* ap[FM];
      const TI* bp[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) ap[i] = &As[(wm * WM + i * 16 + lr) * LDS_LD + ks + lk];
#pragma unroll
      for (int j = 0; j < FN; ++j) bp[j] = &Bs[(wn * WN + j * 16 + lr) * LDS_LD + ks + lk];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = MF::mac(ap[i], bp[j], acc[i][j]);
    }
  }

  // D layout of the 16x16 instructions: column lane % 16; rows 4 (lane/16) + r, or
  // lane/16 + 4 r for FP64.
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * WN + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + (MF::ROWS_STRIDED ? (lane >> 4) + 4 * r : (lane >> 4) * 4 + r);
        if (row < M) C[(int64_t)row * ldc + col] = out_cvt<TO, acc_t>(acc[i][j][r]);
      }
    }
}

template <typename TI, typename TO, int BM, int BN, bool TA, bool TB, bool VEC, bool GROUPED>
__global__ __launch_bounds__(gemm_threads(BM, BN)) void gemm_kernel(GemmArgs ga_, const GemmArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    VBlock vb = hw_block();
    if (!slice_block(ga_, vb)) return;
    gemm_kernel_body<TI, TO, BM, BN, TA, TB, VEC>(ga_, vb, false);
  } else {
    VBlock vb;
    const GemmArgs g = group_args(grp, bmap, vb);
    if (!slice_block(g, vb)) return;   // the instance's grid may be padded
    gemm_kernel_body<TI, TO, BM, BN, TA, TB, VEC>(g, vb, true);
  }
}

// FP32 / FP64 slice GEMM with 16-byte global loads (VW elements) along each
// operand's contiguous dimension and LDS tiles kept in that same orientation:
// A~ as [m][k] (or [k][m] when transposed), the right operand as [k][n] (or
// [n][k]).  Rows of the [.][k] tiles carry a 16-byte pad and those of the
// [k][.] tiles a 64-byte pad, so the 16-byte stores and the MFMA operand reads
// (16 rows x 4 k per instruction) hit distinct banks.  4 waves in 2 x 2, each
// owning (BM/2) x (BN/2) as 16 x 16 blocks; the next chunk is prefetched into
// registers while the current one is multiplied.  Out-of-range elements are
// loaded from a clamped address and replaced by zero (no branches per load).
template <typename T, int BM, int BN, int BK, bool TA, bool TB, int VW>
__device__ __forceinline__ void gemm_mn_kernel_body(const GemmArgs& ga, const VBlock vb, const bool grouped) {
  typedef Mfma<T> MF;
  typedef typename MF::frag_t frag_t;
  constexpr int KSTEP = MF::KSTEP;
  static_assert(KSTEP == 4 && MF::EPL == 1, "32/64-bit MFMA only");
  constexpr int PADK = 16 / (int)sizeof(T), PADR = 64 / (int)sizeof(T);
  constexpr int LDAK = BK + PADK, LDAM = BM + PADR;   // A as [m][k] / [k][m]
  constexpr int LDBK = BK + PADK, LDBN = BN + PADR;   // B as [n][k] / [k][n]
  constexpr int A_LDS = TA ? BK * LDAM : BM * LDAK;
  constexpr int B_LDS = TB ? BN * LDBK : BK * LDBN;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  // vectors per chunk and per thread
  constexpr int A_V = BM * BK / VW, B_V = BN * BK / VW;
  constexpr int A_PER = (A_V + 255) / 256, B_PER = (B_V + 255) / 256;
  static_assert(FM >= 1 && FN >= 1, "tile");
  static_assert(BK % KSTEP == 0 && BK % VW == 0 && BM % VW == 0 && BN % VW == 0, "chunk");

  if (!gate_open(ga.g)) return;
  __shared__ __attribute__((aligned(16))) T As[A_LDS];
  __shared__ __attribute__((aligned(16))) T Bs[B_LDS];

  const int M = ga.M, N = ga.N, K = ga.K;
  const T* __restrict__ A = (const T*)ga.A + (int64_t)vb.z * ga.sA;
  const T* __restrict__ B = (const T*)ga.B + (int64_t)vb.z * ga.sB;
  T* __restrict__ C = (T*)ga.C + (int64_t)vb.z * ga.sC;
  const int64_t lda = ga.lda, ldb = ga.ldb, ldc = ga.ldc;
  const int m0 = vb.y * BM, n0 = vb.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;

  // chunk coordinates of vector u of this thread: (row r, contiguous offset c)
  // A: TA -> rows are k (BK of them), vectors along m; else rows m, vectors along k
  constexpr int A_ROWV = TA ? BM / VW : BK / VW;
  constexpr int B_ROWV = TB ? BK / VW : BN / VW;
  T ra[A_PER][VW], rb[B_PER][VW];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int u = 0; u < A_PER; ++u) {
      const int idx = tid + u * 256;
      const int r = idx / A_ROWV, c = (idx - r * A_ROWV) * VW;
      const int gm = m0 + (TA ? c : r), gk = k0 + (TA ? r : c);
      const bool ok = (A_V % 256 == 0 || idx < A_V) && gm < M && gk < K;
      const int64_t off = ok ? (TA ? (int64_t)gk * lda + gm : (int64_t)gm * lda + gk) : 0;
      VecIO<T, VW>::ld(A + off, ra[u]);
      if (!ok) {
#pragma unroll
        for (int v = 0; v < VW; ++v) ra[u][v] = (T)0;
      }
    }
#pragma unroll
    for (int u = 0; u < B_PER; ++u) {
      const int idx = tid + u * 256;
      const int r = idx / B_ROWV, c = (idx - r * B_ROWV) * VW;
      const int gn = n0 + (TB ? r : c), gk = k0 + (TB ? c : r);
      const bool ok = (B_V % 256 == 0 || idx < B_V) && gn < N && gk < K;
      const int64_t off = ok ? (TB ? (int64_t)gn * ldb + gk : (int64_t)gk * ldb + gn) : 0;
      VecIO<T, VW>::ld(B + off, rb[u]);
      if (!ok) {
#pragma unroll
        for (int v = 0; v < VW; ++v) rb[u][v] = (T)0;
      }
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int u = 0; u < A_PER; ++u) {
      const int idx = tid + u * 256;
      if (A_V % 256 == 0 || idx < A_V) {
        const int r = idx / A_ROWV, c = (idx - r * A_ROWV) * VW;
        VecIO<T, VW>::st(&As[r * (TA ? LDAM : LDAK) + c], ra[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < B_PER; ++u) {
      const int idx = tid + u * 256;
      if (B_V % 256 == 0 || idx < B_V) {
        const int r = idx / B_ROWV, c = (idx - r * B_ROWV) * VW;
        VecIO<T, VW>::st(&Bs[r * (TB ? LDBK : LDBN) + c], rb[u]);
      }
    }
  };

  frag_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = (T)0;

  load_chunk(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    store_chunk();
    __syncthreads();
    if (k0 + BK < K) load_chunk(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += KSTEP) {
      const T* ap[FM];
      const T* bp[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int m = wm * WM + i * 16 + lr;
        ap[i] = TA ? &As[(ks + lk) * LDAM + m] : &As[m * LDAK + ks + lk];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int n = wn * WN + j * 16 + lr;
        bp[j] = TB ? &Bs[n * LDBK + ks + lk] : &Bs[(ks + lk) * LDBN + n];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = MF::mac(ap[i], bp[j], acc[i][j]);
    }
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * WN + j * 16 + lr;
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + (MF::ROWS_STRIDED ? lk + 4 * r : lk * 4 + r);
        if (row < M) C[(int64_t)row * ldc + col] = acc[i][j][r];
      }
    }
}

template <typename T, int BM, int BN, int BK, bool TA, bool TB, int VW, bool GROUPED>
__global__ __launch_bounds__(256) void gemm_mn_kernel(GemmArgs ga_, const GemmArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    VBlock vb = hw_block();
    if (!slice_block(ga_, vb)) return;
    gemm_mn_kernel_body<T, BM, BN, BK, TA, TB, VW>(ga_, vb, false);
  } else {
    VBlock vb;
    const GemmArgs g = group_args(grp, bmap, vb);
    if (!slice_block(g, vb)) return;   // the instance's grid may be padded
    gemm_mn_kernel_body<T, BM, BN, BK, TA, TB, VW>(g, vb, true);
  }
}

template <typename T, int BM, int BN, int BK>
static hipError_t launch_gemm_mn(dctk_ctx ctx, hipStream_t s, GemmArgs ga, int ta, int tb, bool vec,
                                 int batch) {
  ga.nbatch = batch >= kSliceXcdMin ? batch : 0;
  const int gz = ga.nbatch > 0 ? (batch + 7) / 8 * 8 : batch;
  const dim3 grid((unsigned)((ga.N + BN - 1) / BN), (unsigned)((ga.M + BM - 1) / BM), (unsigned)gz);
  constexpr int VW = 16 / (int)sizeof(T);
#define DCTK_GMN(TA_, TB_, VW_) return launch_kernel(ctx, s, gemm_mn_kernel<T, BM, BN, BK, TA_, TB_, VW_, false>, gemm_mn_kernel<T, BM, BN, BK, TA_, TB_, VW_, true>, grid, 256, 0, ga)
#define DCTK_GMN_V(TA_, TB_)    \
  do {                          \
    if (vec) DCTK_GMN(TA_, TB_, VW); \
    DCTK_GMN(TA_, TB_, 1);      \
  } while (0)
  if (!ta && !tb) DCTK_GMN_V(false, false);
  if (ta && !tb) DCTK_GMN_V(true, false);
  if (!ta && tb) DCTK_GMN_V(false, true);
  DCTK_GMN_V(true, true);
#undef DCTK_GMN_V
#undef DCTK_GMN
}

// FP32 / FP64 GEMMs with the output in the input type: 128 x 128 tiles while
// they give every CU two tiles, then 64 x 64 while they cover the CUs, else 32 x 32.
template <typename T>
static hipError_t launch_gemm_vec(dctk_ctx ctx, hipStream_t s, int M, int N, int K, const void* A, int64_t lda,
                                  int64_t sA, int ta, const void* B, int64_t ldb, int64_t sB, int tb, void* C,
                                  int64_t ldc, int64_t sC, int batch, Gate g, int num_cus, int tile) {
  GemmArgs ga{};
  ga.M = M;
  ga.N = N;
  ga.K = K;
  ga.A = A;
  ga.lda = lda;
  ga.sA = sA;
  ga.B = B;
  ga.ldb = ldb;
  ga.sB = sB;
  ga.C = C;
  ga.ldc = ldc;
  ga.sC = sC;
  ga.g = g;
  constexpr int VW = 16 / (int)sizeof(T);
  const bool vec = M % VW == 0 && N % VW == 0 && K % VW == 0 && lda % VW == 0 && ldb % VW == 0 &&
                   sA % VW == 0 && sB % VW == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)B % 16) == 0;
  const int64_t t128 = (int64_t)((M + 127) / 128) * ((N + 127) / 128) * batch;
  const int64_t t64 = (int64_t)((M + 63) / 64) * ((N + 63) / 64) * batch;
  constexpr int BK = sizeof(T) == 8 ? 16 : 32;
  if (sizeof(T) == 4 && (tile == 128 || (tile == 0 && t128 >= 2 * (int64_t)num_cus)))
    return launch_gemm_mn<T, 128, 128, 16>(ctx, s, ga, ta, tb, vec, batch);
  if (tile == 64 || tile == 128 || (tile == 0 && t64 >= (int64_t)num_cus))
    return launch_gemm_mn<T, 64, 64, BK>(ctx, s, ga, ta, tb, vec, batch);
  return launch_gemm_mn<T, 32, 32, BK>(ctx, s, ga, ta, tb, vec, batch);
}

template <typename TI, typename TO, int BM, int BN>
static hipError_t launch_gemm_tile(dctk_ctx ctx, hipStream_t s, int M, int N, int K, const void* A, int64_t lda,
                                   int64_t sA, int ta, const void* B, int64_t ldb, int64_t sB, int tb,
                                   void* C, int64_t ldc, int64_t sC, int batch, Gate g) {
  GemmArgs ga{};
  ga.nbatch = batch >= kSliceXcdMin ? batch : 0;
  const int gz = ga.nbatch > 0 ? (batch + 7) / 8 * 8 : batch;
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)gz);
  ga.M = M;
  ga.N = N;
  ga.K = K;
  ga.A = A;
  ga.lda = lda;
  ga.sA = sA;
  ga.B = B;
  ga.ldb = ldb;
  ga.sB = sB;
  ga.C = C;
  ga.ldc = ldc;
  ga.sC = sC;
  ga.g = g;
  // 16-byte vectors: 8 elements along each operand's contiguous dimension
  const bool va = (ta ? M % 8 == 0 : K % 8 == 0) && lda % 8 == 0 && sA % 8 == 0 && ((uintptr_t)A % 16) == 0;
  const bool vb = (tb ? K % 8 == 0 : N % 8 == 0) && ldb % 8 == 0 && sB % 8 == 0 && ((uintptr_t)B % 16) == 0;
  const bool vec = sizeof(TI) == 2 && va && vb;
#define DCTK_GEMM_LAUNCH(TA_, TB_) \
  do { \
    if (vec) return launch_kernel(ctx, s, gemm_kernel<TI, TO, BM, BN, TA_, TB_, true, false>, gemm_kernel<TI, TO, BM, BN, TA_, TB_, true, true>, grid, gemm_threads(BM, BN), 0, ga); \
    return launch_kernel(ctx, s, gemm_kernel<TI, TO, BM, BN, TA_, TB_, false, false>, gemm_kernel<TI, TO, BM, BN, TA_, TB_, false, true>, grid, gemm_threads(BM, BN), 0, ga); \
  } while (0)
  if (!ta && !tb) DCTK_GEMM_LAUNCH(false, false);
  if (ta && !tb) DCTK_GEMM_LAUNCH(true, false);
  if (!ta && tb) DCTK_GEMM_LAUNCH(false, true);
  DCTK_GEMM_LAUNCH(true, true);
#undef DCTK_GEMM_LAUNCH
}

template <typename TI, typename TO>
static hipError_t launch_gemm_t(dctk_ctx ctx, hipStream_t s, int M, int N, int K, const void* A, int64_t lda, int64_t sA,
                                int ta, const void* B, int64_t ldb, int64_t sB, int tb, void* C, int64_t ldc,
                                int64_t sC, int batch, Gate g, int num_cus, int tile) {
  // 128 x 128 tiles while they give every CU two, then 64 x 64 when they
  // fill the chip, 32 x 32 otherwise.
  const int64_t tiles256 = (int64_t)((M + 255) / 256) * ((N + 255) / 256) * batch;
  const int64_t tiles128 = (int64_t)((M + 127) / 128) * ((N + 127) / 128) * batch;
  int64_t tiles64 = (int64_t)((M + 63) / 64) * ((N + 63) / 64) * batch;
  // 256 x 128 while 256 x 256 blocks still give every CU one (each operand
  // byte staged serves 4/3 the flops of a 128 x 128 tile, and two workgroups
  // of 4 waves per CU hide more latency than one of 8 with 256 x 256 tiles)
  if (tile == 256 || (tile == 0 && M >= 256 && N >= 256 && tiles256 >= (int64_t)num_cus))
    return launch_gemm_tile<TI, TO, 256, 128>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g);
  if (tile == 128 || (tile == 0 && tiles128 >= 2 * (int64_t)num_cus))
    return launch_gemm_tile<TI, TO, 128, 128>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g);
  if (tile == 64 || (tile == 0 && tiles64 >= 2 * (int64_t)num_cus))
    return launch_gemm_tile<TI, TO, 64, 64>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g);
  return launch_gemm_tile<TI, TO, 32, 32>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g);
}

static int g_num_cus = 256;

hipError_t launch_gemm(dctk_ctx ctx, hipStream_t s, int in_dtype, int out_acc, int M, int N, int K,
                       const void* A, int64_t lda, int64_t sA, int ta,
                       const void* B, int64_t ldb, int64_t sB, int tb,
                       void* C, int64_t ldc, int64_t sC, int batch, Gate g, int tile) {
  // out_acc = 1: output in the accumulator type; 0: output in the input type
  switch (in_dtype) {
    case DCTK_F64:
      return launch_gemm_vec<double>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g, g_num_cus, tile);
    case DCTK_F32:
      return launch_gemm_vec<float>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g, g_num_cus, tile);
    case DCTK_BF16:
      if (out_acc)
        return launch_gemm_t<bf16_t, float>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g, g_num_cus, tile);
      return launch_gemm_t<bf16_t, bf16_t>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g, g_num_cus, tile);
    case DCTK_F16:
      if (out_acc)
        return launch_gemm_t<f16_t, float>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g, g_num_cus, tile);
      return launch_gemm_t<f16_t, f16_t>(ctx, s, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, C, ldc, sC, batch, g, g_num_cus, tile);
    default:
      return hipErrorInvalidValue;
  }
}

// ---- the c-product and its adjoint on an operator's workspaces ---------------
static size_t dtype_size(int dt) { return dt == DCTK_F64 ? 8 : (dt == DCTK_F32 ? 4 : 2); }

bool fused_eligible(dctk_op op) {
  const int64_t nmax = op->n1 > op->n2 ? op->n1 : op->n2;
  const bool small_offsets = op->p * op->n1 * op->n2 < (int64_t(1) << 31) && op->p * nmax * op->s < (int64_t(1) << 31);
  return !op->two_sided && op->p <= kFusedMaxP && small_offsets;
}

// Without a tuned choice: the fused product while the problem is small enough to
// be latency-bound (fewer 32 x 32 output tiles than CUs) and its transforms stay
// cheap next to the slice GEMMs (p <= 4, or small slices); else transform, GEMM,
// transform.
bool use_fused(dctk_op op, int adjoint) {
  const int path = op->tune[adjoint ? 1 : 0][0];
  if (path >= 0) return path == 1;
  const int64_t M = adjoint ? op->n2 : op->n1, K = adjoint ? op->n1 : op->n2, N = op->s;
  const int64_t t32 = ((M + 31) / 32) * ((N + 31) / 32);
  return t32 < g_num_cus && (op->p <= 4 || M * N * K <= (int64_t)192 * 192 * 192);
}

// The GEMM's gate under a product's control block: it runs unless the process
// stopped at an earlier step.
static Gate gemm_gate(const Ctl& ctl) {
  Gate g{nullptr, 0, 0};
  if (ctl.kind != CTL_PLAIN) {
    g.st = ctl.st;
    g.j = ctl.kind == CTL_ARN_FWD ? ctl.j - 1 : ctl.j;
    const bool fwd = ctl.kind == CTL_GKB_FWD || ctl.kind == CTL_GKB_FWDU;
    g.mode = fwd ? 0 : 1;
    if (fwd) g.j = ctl.j;
  }
  return g;
}

// Step 2 of a three-kernel product: the slice products of X~ (op->xh) into op->ch.
static hipError_t slice_gemms(dctk_op op, hipStream_t s, int adjoint, const Gate& g) {
  dctk_ctx ctx = op->ctx;
  const int tile = op->tune[adjoint ? 1 : 0][1];
  const int64_t p = op->p, n1 = op->n1, n2 = op->n2, sc = op->s;
  const int gdt = op->gemm_dtype;
  const int64_t rin = adjoint ? n1 : n2;
  const int64_t rout = adjoint ? n2 : n1;
  const int64_t sAh = n1 * n2;
  hipError_t e;
  prof_begin(ctx, PROF_GEMM);
  // the left operand: A~ (n1 x n2), or for the adjoint A~^T (n2 x n1) -- read
  // from the transposed copy when the operator keeps one (16-bit types)
  const bool tcopy = adjoint && op->AhT != nullptr;
  const void* Aop = tcopy ? op->AhT : op->Ah;
  const int64_t ldA = tcopy ? n1 : n2;
  const int tA = adjoint && !tcopy ? 1 : 0;
  if (!op->two_sided) {
    // forward: (n1 x n2)(n2 x s);  adjoint: (n2 x n1 := A~^T)(n1 x s)
    e = launch_gemm(ctx, s, gdt, 1, (int)rout, (int)sc, (int)rin, Aop, ldA, sAh, tA,
                    op->xh, sc, rin * sc, 0, op->ch, sc, rout * sc, (int)p, g, tile);
  } else {
    e = launch_gemm(ctx, s, gdt, 0, (int)rout, (int)sc, (int)rin, Aop, ldA, sAh, tA,
                    op->xh, sc, rin * sc, 0, op->th, sc, rout * sc, (int)p, g, tile);
    // right factor: forward (rout x s)(s x s) with B~; adjoint with B~^T
    if (e == hipSuccess)
      e = launch_gemm(ctx, s, gdt, 1, (int)rout, (int)sc, (int)sc, op->th, sc, rout * sc, 0,
                      op->Bh, sc, sc * sc, adjoint ? 1 : 0, op->ch, sc, rout * sc, (int)p, g, tile);
  }
  prof_end(ctx, PROF_GEMM);
  return e;
}

bool pair_eligible(dctk_op op) {
  return !op->fast && tube_pair_ok(op->p, op->vec_dtype) &&
         !(fused_eligible(op) && (use_fused(op, 0) || use_fused(op, 1)));
}

hipError_t pair_first(dctk_op op, hipStream_t s, int adjoint, const void* X, const Ctl& ctl) {
  dctk_ctx ctx = op->ctx;
  const int64_t pp = op->p * op->p;
  const int64_t rin = adjoint ? op->n1 : op->n2;
  const int gi = adjoint ? 2 : 0;
  prof_begin(ctx, PROF_TUBE_FWD);
  hipError_t e = launch_tube(ctx, s, op->vec_dtype, op->gemm_dtype, op->p, rin * op->s, X, op->xh, op->Gd + gi * pp,
                             op->Gf + gi * pp, nullptr, nullptr, ctl, true, false, nullptr);
  prof_end(ctx, PROF_TUBE_FWD);
  if (e != hipSuccess) return e;
  return slice_gemms(op, s, adjoint, gemm_gate(ctl));
}

hipError_t pair_gemm(dctk_op op, hipStream_t s, int adjoint, const Ctl& ctl) {
  return slice_gemms(op, s, adjoint, gemm_gate(ctl));
}

hipError_t pair_transforms(dctk_op op, hipStream_t s, int adjoint, const void* src, void* Y, const Ctl& ctl,
                           int* nblocks_out) {
  dctk_ctx ctx = op->ctx;
  const int64_t pp = op->p * op->p;
  const int64_t rout = adjoint ? op->n2 : op->n1;
  // this product's inverse (L^{-1}, or L^T for the adjoint); its transpose is the
  // next product's forward transform (L^{-T} for the adjoint after a forward
  // product, L after an adjoint)
  const int g1 = adjoint ? 3 : 1;
  prof_begin(ctx, PROF_TUBE_PAIR);
  hipError_t e = launch_tube_pair(ctx, s, op->gemm_dtype, op->p, rout * op->s, (const float*)op->ch,
                                  (const float*)src, (float*)Y, op->xh, op->Gf + g1 * pp, ctl, nblocks_out);
  prof_end(ctx, PROF_TUBE_PAIR);
  return e;
}

hipError_t apply_op(dctk_op op, hipStream_t s, int adjoint, const void* X, void* Y, const void* src,
                    void* xnorm, const Ctl& ctl, int* nblocks_out) {
  dctk_ctx ctx = op->ctx;
  if (fused_eligible(op) && use_fused(op, adjoint)) return launch_fused(op, s, adjoint, X, Y, src, xnorm, ctl, nblocks_out);
  const int64_t p = op->p, n1 = op->n1, n2 = op->n2, sc = op->s;
  const int gdt = op->gemm_dtype, vdt = op->vec_dtype;
  const double* Gd = op->Gd;
  const float* Gf = op->Gf;
  const int64_t pp = p * p;
  hipError_t e;
  // rows of the input / output vectors
  const int64_t rin = adjoint ? n1 : n2;
  const int64_t rout = adjoint ? n2 : n1;
  // step 1: transform the input tubes (L, or L^{-T} for the adjoint) into the GEMM type;
  // this kernel evaluates the control block (input scale, recorded scalars)
  const int gi = adjoint ? 2 : 0;
  prof_begin(ctx, PROF_TUBE_FWD);
  if (op->fast)  // tubes longer than kMaxTube: the O(p log p) transform
    e = launch_tube_fast_ctl(ctx, s, op->tube, adjoint ? DCTK_MAT_LINVT : DCTK_MAT_L, vdt, gdt, p, rin * sc, X,
                             op->xh, nullptr, xnorm, ctl, true, false, nullptr);
  else
    e = launch_tube(ctx, s, vdt, gdt, p, rin * sc, X, op->xh, Gd + gi * pp, Gf + gi * pp, nullptr, xnorm, ctl, true,
                    false, nullptr);
  prof_end(ctx, PROF_TUBE_FWD);
  if (e != hipSuccess) return e;
  // later kernels read the recorded scalars from the state
  Ctl later = ctl;
  later.from_state = 1;
  // step 2: slice products
  e = slice_gemms(op, s, adjoint, gemm_gate(ctl));
  if (e != hipSuccess) return e;
  // step 3: inverse transform (L^{-1}, or L^T for the adjoint) with the epilogue
  const int go = adjoint ? 3 : 1;
  prof_begin(ctx, PROF_TUBE_INV);
  if (op->fast)
    e = launch_tube_fast_ctl(ctx, s, op->tube, adjoint ? DCTK_MAT_LT : DCTK_MAT_LINV, vdt, vdt, p, rout * sc, op->ch,
                             Y, src, nullptr, later, false, true, nblocks_out);
  else
    e = launch_tube(ctx, s, vdt, vdt, p, rout * sc, op->ch, Y, Gd + go * pp, Gf + go * pp, src, nullptr, later, false,
                    true, nblocks_out);
  prof_end(ctx, PROF_TUBE_INV);
  return e;
}

void set_num_cus(int n) { if (n > 0) g_num_cus = n; }
int num_cus() { return g_num_cus; }
size_t elem_size(int dt) { return dtype_size(dt); }

}  // namespace dctk
