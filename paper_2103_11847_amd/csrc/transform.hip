// Tube transforms along mode 3 (Algorithm 1 steps 1 and 3; Remark 2.1).
//
// A tube transform is out = in x_3 G with G a small p x p matrix: for every
// position e of a frontal slice, out[k][e] = sum_t G[k][t] in[t][e].  With the
// slice-major layout the p inputs of a tube are p slices apart, so a thread
// streams VEC consecutive positions of every slice (coalesced 16-byte loads
// along the slice) and keeps KB outputs in registers per pass; G sits in LDS.
// The work is HBM-bound for the p of colour images and video (2p flops per
// 2 elements moved).
#include <cmath>
#include <vector>

#include "mfma.h"

namespace dctk {

// ---- host: the transform matrices, FP64 closed forms -----------------------
// C_n of eq. (dft1), 0-based: C[i][j] = sqrt((2 - [i == 0]) / n) cos(i (2j + 1) pi / (2n)).
static void dct_matrix(int64_t n, std::vector<double>& C) {
  C.assign((size_t)(n * n), 0.0);
  const double pi = 3.14159265358979323846264338327950288;
  for (int64_t i = 0; i < n; ++i) {
    double sc = std::sqrt((i == 0 ? 1.0 : 2.0) / (double)n);
    for (int64_t j = 0; j < n; ++j)
      C[(size_t)(i * n + j)] = sc * std::cos((double)i * (double)(2 * j + 1) * pi / (2.0 * (double)n));
  }
}

int build_tube_matrix(int tube, int which, int64_t p, double* out) {
  if (p <= 0) return DCTK_ESHAPE;
  if (out == nullptr) return DCTK_EINVAL;
  if (which < DCTK_MAT_L || which > DCTK_MAT_LT) return DCTK_EINVAL;
  std::vector<double> C, L((size_t)(p * p)), Li((size_t)(p * p));
  dct_matrix(p, C);
  if (tube == DCTK_TUBE_DCT2) {
    for (int64_t i = 0; i < p; ++i)
      for (int64_t j = 0; j < p; ++j) {
        L[(size_t)(i * p + j)] = C[(size_t)(i * p + j)];
        Li[(size_t)(i * p + j)] = C[(size_t)(j * p + i)];  // C^{-1} = C^T
      }
  } else if (tube == DCTK_TUBE_TH) {
    // M = W^{-1} C (I + Z): row i of C (I + Z) is C[i][j] + C[i][j-1], scaled by 1 / C[i][0].
    for (int64_t i = 0; i < p; ++i)
      for (int64_t j = 0; j < p; ++j) {
        double v = C[(size_t)(i * p + j)] + (j > 0 ? C[(size_t)(i * p + j - 1)] : 0.0);
        L[(size_t)(i * p + j)] = v / C[(size_t)(i * p)];
      }
    // M^{-1} = (I + Z)^{-1} C^T W with (I + Z)^{-1}[i][l] = (-1)^{l - i} for l >= i:
    // M^{-1}[i][j] = C[j][0] * sum_{l >= i} (-1)^{l - i} C[j][l].
    for (int64_t i = 0; i < p; ++i)
      for (int64_t j = 0; j < p; ++j) {
        double acc = 0.0, sg = 1.0;
        for (int64_t l = i; l < p; ++l, sg = -sg) acc += sg * C[(size_t)(j * p + l)];
        Li[(size_t)(i * p + j)] = acc * C[(size_t)(j * p)];
      }
  } else {
    return DCTK_EINVAL;
  }
  for (int64_t i = 0; i < p; ++i)
    for (int64_t j = 0; j < p; ++j) {
      double v;
      switch (which) {
        case DCTK_MAT_L: v = L[(size_t)(i * p + j)]; break;
        case DCTK_MAT_LINV: v = Li[(size_t)(i * p + j)]; break;
        case DCTK_MAT_LINVT: v = Li[(size_t)(j * p + i)]; break;
        default: v = L[(size_t)(j * p + i)]; break;
      }
      out[i * p + j] = v;
    }
  return DCTK_OK;
}

// ---- device: the streaming transform ----------------------------------------
template <typename T> struct Vec4Load;
template <> struct Vec4Load<float> {
  __device__ static void load(const float* p, float* v) {
    float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
};
template <> struct Vec4Load<double> {
  __device__ static void load(const double* p, double* v) {
    double2 a = *reinterpret_cast<const double2*>(p);
    double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};

template <typename T> struct Vec4Store {
  __device__ static void store(T* p, const T* v) {
    for (int i = 0; i < 4; ++i) p[i] = v[i];
  }
};
template <> struct Vec4Store<float> {
  __device__ static void store(float* p, const float* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
};
template <> struct Vec4Store<double> {
  __device__ static void store(double* p, const double* v) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
  }
};

// TIN: float or double; TOUT: float, double, bf16_t or f16_t; TC: compute type.
// SCALE: apply the control block's input scale (and write xnorm); EPI: apply
// its a/b/src epilogue and write per-block partials of out^2.
struct TubeArgs {
  int gx, gy, gz;
  int p;
  int64_t count;       // tube positions (elements per slice)
  const void* in;      // p x count, TIN
  void* out;           // p x count, TOUT
  const void* G;       // p x p, TC
  const void* src;     // p x count, TOUT, or null
  void* xnorm;         // p x count, TIN, or null
  Ctl ctl;
};

template <typename TIN, typename TOUT, typename TC, int KB, bool VEC, bool SCALE, bool EPI>
__device__ __forceinline__ void tube_kernel_body(const TubeArgs& ta, const VBlock vb, const bool grouped) {
  __shared__ double sh[kShCtl];
  const int p = ta.p;
  const int64_t count = ta.count;
  const TIN* __restrict__ in = (const TIN*)ta.in;
  TOUT* out = (TOUT*)ta.out;
  const TC* __restrict__ G = (const TC*)ta.G;
  const TOUT* src = (const TOUT*)ta.src;
  TIN* xnorm = (TIN*)ta.xnorm;
  const Ctl& ctl = ta.ctl;
  double a_d, b_d, s_d;
  if (!ctl_begin(ctl, a_d, b_d, s_d, sh, vb)) return;
  if (!SCALE) s_d = 1.0;
  if (!EPI) { a_d = 1.0; b_d = 0.0; }
  const TC a = (TC)a_d, b = (TC)b_d, sc = (TC)s_d;
  extern __shared__ char smem_raw[];
  TC* sG = reinterpret_cast<TC*>(smem_raw);
  for (int i = threadIdx.x; i < p * p; i += blockDim.x) sG[i] = G[i];
  __syncthreads();
  double sq = 0.0;
  const int64_t stride = (int64_t)ta.gx * blockDim.x * 4;
  if (p <= KB) {
    // all p tubes of a 4-position group at once: every input (and src) load
    // of the group is issued before the first use, from clamped addresses
    const bool use_src = EPI && src != nullptr && b != (TC)0;
    const TOUT* srcl = use_src ? src : out;
    for (int64_t e0 = ((int64_t)vb.x * blockDim.x + threadIdx.x) * 4; e0 < count; e0 += stride) {
      const int nv = (count - e0) < 4 ? (int)(count - e0) : 4;
      TIN xv[KB][4];
      if (VEC && nv == 4) {
#pragma unroll
        for (int t = 0; t < KB; ++t) {
          Vec4Load<TIN>::load(in + (int64_t)(t < p ? t : 0) * count + e0, xv[t]);
          if (t >= p) {
#pragma unroll
            for (int v = 0; v < 4; ++v) xv[t][v] = (TIN)0;
          }
        }
      } else {
#pragma unroll
        for (int t = 0; t < KB; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool ok = t < p && v < nv;
            const TIN x = in[ok ? (int64_t)t * count + e0 + v : 0];
            xv[t][v] = ok ? x : (TIN)0;
          }
      }
      TC sv[KB][4];
#pragma unroll
      for (int k = 0; k < KB; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) sv[k][v] = (TC)0;
      if (use_src) {
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool ok = k < p && v < nv;
            const TOUT x = srcl[ok ? (int64_t)k * count + e0 + v : 0];
            sv[k][v] = ok ? (TC)x : (TC)0;
          }
      }
      if (SCALE) {
#pragma unroll
        for (int t = 0; t < KB; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) xv[t][v] = (TIN)(sc * (TC)xv[t][v]);
        if (xnorm != nullptr) {
#pragma unroll
          for (int t = 0; t < KB; ++t) {
            if (t < p) {
              TIN* xp = xnorm + (int64_t)t * count + e0;
              if (VEC && nv == 4) Vec4Store<TIN>::store(xp, xv[t]);
              else for (int v = 0; v < nv; ++v) xp[v] = xv[t][v];
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        if (k >= p) break;
        TC acc[4] = {(TC)0, (TC)0, (TC)0, (TC)0};
#pragma unroll
        for (int t = 0; t < KB; ++t) {
          const TC gk = t < p ? sG[k * p + t] : (TC)0;
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[v] += gk * (TC)xv[t][v];
        }
        TOUT ov[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          TC r = a * acc[v];
          if (EPI) r += b * sv[k][v];
          ov[v] = cvt<TOUT, TC>(r);
          if (EPI && v < nv) {
            const double rv = (double)r;
            sq += rv * rv;
          }
        }
        TOUT* op = out + (int64_t)k * count + e0;
        if (VEC && nv == 4) Vec4Store<TOUT>::store(op, ov);
        else for (int v = 0; v < nv; ++v) op[v] = ov[v];
      }
    }
    if (EPI && ctl.part_out != nullptr) {
      const double tot = block_sum_all(sq, sh);
      if (threadIdx.x == 0) ctl.part_out[vb.x] = tot;
    }
    return;
  }
  for (int64_t e0 = ((int64_t)vb.x * blockDim.x + threadIdx.x) * 4; e0 < count; e0 += stride) {
    const int nv = (count - e0) < 4 ? (int)(count - e0) : 4;
    for (int k0 = 0; k0 < p; k0 += KB) {
      TC acc[KB][4];
#pragma unroll
      for (int kk = 0; kk < KB; ++kk)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[kk][v] = (TC)0;
      for (int t = 0; t < p; ++t) {
        TIN xv[4];
        const TIN* ip = in + (int64_t)t * count + e0;
        if (VEC && nv == 4) {
          Vec4Load<TIN>::load(ip, xv);
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) xv[v] = v < nv ? ip[v] : (TIN)0;
        }
        if (SCALE) {
#pragma unroll
          for (int v = 0; v < 4; ++v) xv[v] = (TIN)(sc * (TC)xv[v]);
          if (xnorm != nullptr && k0 == 0) {
            TIN* xp = xnorm + (int64_t)t * count + e0;
            if (VEC && nv == 4) Vec4Store<TIN>::store(xp, xv);
            else for (int v = 0; v < nv; ++v) xp[v] = xv[v];
          }
        }
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
          const TC gk = (k0 + kk < p) ? sG[(k0 + kk) * p + t] : (TC)0;
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[kk][v] += gk * (TC)xv[v];
        }
      }
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const int k = k0 + kk;
        if (k >= p) break;
        TOUT* op = out + (int64_t)k * count + e0;
        TOUT ov[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          TC r = a * acc[kk][v];
          if (EPI && b != (TC)0 && v < nv) r += b * (TC)src[(int64_t)k * count + e0 + v];
          ov[v] = cvt<TOUT, TC>(r);
          if (EPI && v < nv) {
            const double rv = (double)r;
            sq += rv * rv;
          }
        }
        if (VEC && nv == 4) {
          Vec4Store<TOUT>::store(op, ov);
        } else {
          for (int v = 0; v < nv; ++v) op[v] = ov[v];
        }
      }
    }
  }
  if (EPI && ctl.part_out != nullptr) {
    const double tot = block_sum_all(sq, sh);
    if (threadIdx.x == 0) ctl.part_out[vb.x] = tot;
  }
}

template <typename TIN, typename TOUT, typename TC, int KB, bool VEC, bool SCALE, bool EPI, bool GROUPED>
__global__ __launch_bounds__(kThreads) void tube_kernel(TubeArgs ta_, const TubeArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    tube_kernel_body<TIN, TOUT, TC, KB, VEC, SCALE, EPI>(ta_, hw_block(), false);
  } else {
    VBlock vb;
    const TubeArgs g = group_args(grp, bmap, vb);
    tube_kernel_body<TIN, TOUT, TC, KB, VEC, SCALE, EPI>(g, vb, true);
  }
}

// the epilogue's src in FP32 (bf16_t is the bit pattern of a bfloat16)
template <typename T> __device__ inline float to_f32(T v) { return (float)v; }
template <> __device__ inline float to_f32<bf16_t>(bf16_t v) { return bf16_to_float(v); }

// Long tubes (p >= 16): the transform out = G x in is a (p x p)(p x count)
// contraction, so it runs on the matrix cores.  A workgroup stages G (p x p,
// FP32, rows padded to 16) in LDS once and then walks its 64-position tiles
// (grid stride).  Every global access of a tile is a row of 64 consecutive
// positions of one slice, moved as 16-byte vectors: the input (from clamped
// addresses, all issued together, scaled by the control block's s and
// written to xnorm on the way) and the epilogue's src are loaded before the
// tile is multiplied; wave w computes the 16 positions of column block w for
// every 16-row band of outputs with 16x16x4 FP32 MFMAs; the products return
// to LDS, and the epilogue reads them back as rows, applies a, b and src,
// stores the rows and accumulates the workgroup's partial sum of out^2.
// Without an epilogue (fewer registers live) the control block's loads, G
// and the first tile are in flight together, and the next tile's rows load
// while the current one is multiplied.
// VEC: count a multiple of 4 and 16-byte aligned in / src / xnorm / out.
template <typename T> struct RowStore;
template <> struct RowStore<float> {
  __device__ static void st(float* p, const float (&v)[4]) {
    *reinterpret_cast<f32x4*>(p) = f32x4{v[0], v[1], v[2], v[3]};
  }
};
template <> struct RowStore<bf16_t> {
  __device__ static void st(bf16_t* p, const float (&v)[4]) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const unsigned lo = (unsigned)float_to_bf16(v[0]) | ((unsigned)float_to_bf16(v[1]) << 16);
    const unsigned hi = (unsigned)float_to_bf16(v[2]) | ((unsigned)float_to_bf16(v[3]) << 16);
    *reinterpret_cast<u32x2*>(p) = u32x2{lo, hi};
  }
};
template <> struct RowStore<f16_t> {
  __device__ static void st(f16_t* p, const float (&v)[4]) {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    *reinterpret_cast<h4*>(p) = h4{(f16_t)v[0], (f16_t)v[1], (f16_t)v[2], (f16_t)v[3]};
  }
};

template <typename TOUT, int PM, bool SCALE, bool EPI, bool VEC>
__device__ __forceinline__ void tube_mfma_kernel_body(const TubeArgs& ta, const VBlock vb, const bool grouped) {
  typedef Mfma<float> MF;
  constexpr int NB = 64;            // positions per tile
  constexpr int LDG = PM + 4;       // G as [k][t], t contiguous (+16 bytes)
  constexpr int LDX = NB + 4;       // input / products as [row][e], e contiguous (+16 bytes)
  constexpr int FR = PM / 16;       // row bands
  constexpr int XU = PM * (NB / 4) / 256;  // 4-position units of a tile per thread
  constexpr int GU = PM * PM / 256;        // G entries per thread
  static_assert(XU * 256 == PM * (NB / 4) && GU * 256 == PM * PM, "tile");
  __shared__ __attribute__((aligned(16))) float sG[PM * LDG];
  __shared__ __attribute__((aligned(16))) float sX[PM * LDX];
  __shared__ double sh[kShCtl];
  const int p = ta.p;
  const int64_t count = ta.count;
  const float* in = (const float*)ta.in;
  TOUT* out = (TOUT*)ta.out;
  const float* G = (const float*)ta.G;
  const float* src = (const float*)ta.src;   // FP32 outputs only (launch_tube refuses src otherwise)
  float* xnorm = (float*)ta.xnorm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ntiles = (count + NB - 1) / NB;

  // a tile's input rows and src rows into registers (clamped addresses, selected)
  float rv[XU][4], sv[XU][4];
  auto load_tile = [&](int64_t tile) {
    const int64_t e0 = tile * NB;
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int i = tid + u * 256;
      const int t = i / (NB / 4), c = (i % (NB / 4)) * 4;
      const int64_t e = e0 + c;
      if constexpr (VEC) {
        const bool ok = t < p && e < count;
        const float4 q = *reinterpret_cast<const float4*>(in + (ok ? (int64_t)t * count + e : 0));
        rv[u][0] = ok ? q.x : 0.0f;
        rv[u][1] = ok ? q.y : 0.0f;
        rv[u][2] = ok ? q.z : 0.0f;
        rv[u][3] = ok ? q.w : 0.0f;
        if (EPI) {
          const bool oks = ok && src != nullptr;
          const float4 w = *reinterpret_cast<const float4*>(oks ? src + (int64_t)t * count + e : in);
          sv[u][0] = oks ? w.x : 0.0f;
          sv[u][1] = oks ? w.y : 0.0f;
          sv[u][2] = oks ? w.z : 0.0f;
          sv[u][3] = oks ? w.w : 0.0f;
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool ok = t < p && e + v < count;
          const float x = in[ok ? (int64_t)t * count + e + v : 0];
          rv[u][v] = ok ? x : 0.0f;
          if (EPI) {
            const bool oks = ok && src != nullptr;
            const float y = (src != nullptr ? src : in)[oks ? (int64_t)t * count + e + v : 0];
            sv[u][v] = oks ? y : 0.0f;
          }
        }
      }
    }
  };

  // prologue: the control block's loads, G and the first tile's rows are all in
  // flight before the first of them is used
  const CtlLoad cl = ctl_load(ta.ctl);
  float gv[GU];
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    const int i = tid + u * 256, k = i / PM, t = i % PM;
    const bool ok = k < p && t < p;
    const float v = G[ok ? k * p + t : 0];
    gv[u] = ok ? v : 0.0f;
  }
  int64_t tile = vb.x;
  if (!EPI && tile < ntiles) load_tile(tile);
  double a_d, b_d, s_d;
  if (!ctl_eval(ta.ctl, cl, a_d, b_d, s_d, sh, vb)) return;
  if (!SCALE) s_d = 1.0;
  if (!EPI) { a_d = 1.0; b_d = 0.0; }
  const float a = (float)a_d, b = (float)b_d, sc = (float)s_d;
  const bool use_src = EPI && src != nullptr && b != 0.0f;   // b = 0: src never enters
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    const int i = tid + u * 256, k = i / PM, t = i % PM;
    sG[k * LDG + t] = gv[u];
  }
  const int lr = lane & 15, lk = lane >> 4;
  double sq = 0.0;
  for (; tile < ntiles; tile += ta.gx) {
    const int64_t e0 = tile * NB;
    if (EPI) load_tile(tile);
    __syncthreads();  // the previous tile's products have been read from LDS (and G is staged)
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int i = tid + u * 256;
      const int t = i / (NB / 4), c = (i % (NB / 4)) * 4;
      const int64_t e = e0 + c;
      if (SCALE) {
#pragma unroll
        for (int v = 0; v < 4; ++v) rv[u][v] *= sc;
        if (xnorm != nullptr && t < p) {
          float* xp = xnorm + (int64_t)t * count + e;
          if (VEC) {
            if (e < count) RowStore<float>::st(xp, rv[u]);
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (e + v < count) xp[v] = rv[u][v];
          }
        }
      }
      *reinterpret_cast<float4*>(&sX[t * LDX + c]) = make_float4(rv[u][0], rv[u][1], rv[u][2], rv[u][3]);
    }
    __syncthreads();
    // without an epilogue (fewer registers live) the next tile's rows load while
    // this one is multiplied; with it they load at the top of the next tile
    if (!EPI && tile + ta.gx < ntiles) load_tile(tile + ta.gx);
    typename MF::frag_t acc[FR];
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[f][r] = 0.0f;
#pragma unroll 4
    for (int t0 = 0; t0 < PM; t0 += 4) {
      const float* bp = &sX[(t0 + lk) * LDX + wave * 16 + lr];
#pragma unroll
      for (int f = 0; f < FR; ++f) acc[f] = MF::mac(&sG[(f * 16 + lr) * LDG + t0 + lk], bp, acc[f]);
    }
    // a wave reads and writes only its own 16 columns of sX, and a wave's LDS
    // accesses complete in order: no block barrier before its products go back
    __builtin_amdgcn_wave_barrier();
    // products back to LDS as [k][e]: lane holds rows 4 (lane / 16) + r of column lane % 16
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) sX[(f * 16 + lk * 4 + r) * LDX + wave * 16 + lr] = acc[f][r];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int i = tid + u * 256;
      const int k = i / (NB / 4), c = (i % (NB / 4)) * 4;
      const int64_t e = e0 + c;
      if (k >= p) continue;
      const float4 q = *reinterpret_cast<const float4*>(&sX[k * LDX + c]);
      float y[4] = {a * q.x, a * q.y, a * q.z, a * q.w};
      if (EPI) {
#pragma unroll
        for (int v = 0; v < 4; ++v) y[v] += use_src ? b * sv[u][v] : 0.0f;
      }
      TOUT* op = out + (int64_t)k * count + e;
      if (VEC) {
        if (e < count) {
          RowStore<TOUT>::st(op, y);
          if (EPI) {
#pragma unroll
            for (int v = 0; v < 4; ++v) sq += (double)y[v] * (double)y[v];
          }
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (e + v < count) {
            op[v] = cvt<TOUT, float>(y[v]);
            if (EPI) sq += (double)y[v] * (double)y[v];
          }
      }
    }
  }
  if (EPI && ta.ctl.part_out != nullptr) {
    const double tot = block_sum_all(sq, sh);
    if (tid == 0) ta.ctl.part_out[vb.x] = tot;
  }
}

template <typename TOUT, int PM, bool SCALE, bool EPI, bool VEC, bool GROUPED>
__global__ __launch_bounds__(256) void tube_mfma_kernel(TubeArgs ta_, const TubeArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    tube_mfma_kernel_body<TOUT, PM, SCALE, EPI, VEC>(ta_, hw_block(), false);
  } else {
    VBlock vb;
    const TubeArgs g = group_args(grp, bmap, vb);
    tube_mfma_kernel_body<TOUT, PM, SCALE, EPI, VEC>(g, vb, true);
  }
}

template <typename TOUT>
static hipError_t launch_tube_mfma(dctk_ctx ctx, hipStream_t s, int64_t p, int64_t count, const void* in, void* out,
                                   const float* G, const void* src, void* xnorm, const Ctl& ctl, bool scale,
                                   bool epi, int* nblocks_out) {
  // a few workgroups per CU, each walking several 64-position tiles, so G
  // is staged once per workgroup rather than once per tile
  int64_t blocks = (count + 63) / 64;
  const int64_t cap = 4 * (int64_t)num_cus();
  if (blocks > cap) blocks = cap;
  if (nblocks_out) *nblocks_out = (int)blocks;
  if (epi && ctl.part_out != nullptr && blocks > kRedBlocks) return hipErrorInvalidConfiguration;
  const bool vec = (count % 4 == 0) && (((uintptr_t)in) % 16 == 0) && (((uintptr_t)xnorm) % 16 == 0) &&
                   (((uintptr_t)out) % 16 == 0) && (((uintptr_t)src) % 16 == 0);
  TubeArgs ta{};
  ta.p = (int)p;
  ta.count = count;
  ta.in = in;
  ta.out = out;
  ta.G = G;
  ta.src = src;
  ta.xnorm = xnorm;
  ta.ctl = ctl;
  const dim3 grid((unsigned)blocks);
#define DCTK_TMV(PM_, SC_, EP_) \
  do { \
    if (vec) return launch_kernel(ctx, s, tube_mfma_kernel<TOUT, PM_, SC_, EP_, true, false>, tube_mfma_kernel<TOUT, PM_, SC_, EP_, true, true>, grid, 256, 0, ta); \
    return launch_kernel(ctx, s, tube_mfma_kernel<TOUT, PM_, SC_, EP_, false, false>, tube_mfma_kernel<TOUT, PM_, SC_, EP_, false, true>, grid, 256, 0, ta); \
  } while (0)
#define DCTK_TM(PM_) \
  do { \
    if (scale && epi) DCTK_TMV(PM_, true, true); \
    if (scale) DCTK_TMV(PM_, true, false); \
    if (epi) DCTK_TMV(PM_, false, true); \
    DCTK_TMV(PM_, false, false); \
  } while (0)
  if (p <= 16) DCTK_TM(16);
  if (p <= 32) DCTK_TM(32);
  if (p <= 48) DCTK_TM(48);
  DCTK_TM(64);
#undef DCTK_TM
#undef DCTK_TMV
}

// ---- the two transforms between consecutive slice products ---------------------
// Inside a Golub-Kahan step the inverse transform of one product and the
// forward transform of the next act on the same tubes: y = a (G1 c) + b src is
// the new basis vector (Algorithm 4's U~ or V~, kept unnormalised in its slot)
// and x = G1^T y is the next product's transformed input (its normalisation is
// applied by the next product's epilogue, as `a`).  The second matrix is always
// the transpose of the first: after a forward product G1 = L^{-1} and the
// adjoint's forward transform is L^{-T}; after an adjoint product G1 = L^T and
// the forward product's transform is L.  One pass over a 64-position tile does
// both: the slice products' rows and the src rows come in, y goes out (with
// the workgroup's partial sum of y^2), y returns to LDS, the second MFMA pass
// forms x reading the one staged copy of G1 transposed, and x goes out in the
// GEMM type -- y is never read back from memory.  The control block is the one
// of the first transform's product; the scale it returns for that product's
// input (1/alpha or 1/beta, as the input x of that product was stored
// unnormalised) joins `a`.
struct PairArgs {
  int gx, gy, gz;
  int p;
  int64_t count;
  const float* c;    // p x count slice products (FP32)
  const float* src;  // p x count, or null
  float* y;          // p x count, the new basis vector
  void* x;           // p x count, TX: the next product's transformed input
  const float* G1;   // p x p
  Ctl ctl;
};

template <typename TX, int PM, bool VEC>
__device__ __forceinline__ void tube_pair_kernel_body(const PairArgs& pa, const VBlock vb, const bool grouped) {
  typedef Mfma<float> MF;
  constexpr int NB = 64;
  // rows of G1 padded by 8: both the row reads of the first pass and the
  // column reads of the second spread over the banks
  constexpr int LDG = PM + 8;
  constexpr int LDX = NB + 4;
  constexpr int FR = PM / 16;
  constexpr int XU = PM * (NB / 4) / 256;
  constexpr int GU = PM * PM / 256;
  static_assert(XU * 256 == PM * (NB / 4) && GU * 256 == PM * PM, "tile");
  __shared__ __attribute__((aligned(16))) float sG1[PM * LDG];
  __shared__ __attribute__((aligned(16))) float sX[PM * LDX];
  __shared__ double sh[kShCtl];
  const int p = pa.p;
  const int64_t count = pa.count;
  const float* in = pa.c;
  const float* src = pa.src;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ntiles = (count + NB - 1) / NB;

  // a tile's product rows (rv) and src rows (sv) into registers (clamped
  // addresses, selected); loading the next tile's rows during the passes
  // measured slower
  float rv[XU][4], sv[XU][4];
  auto load_tile = [&](int64_t tile) {
    const int64_t e0 = tile * NB;
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int i = tid + u * 256;
      const int t = i / (NB / 4), c = (i % (NB / 4)) * 4;
      const int64_t e = e0 + c;
      if constexpr (VEC) {
        const bool ok = t < p && e < count;
        const float4 q = *reinterpret_cast<const float4*>(in + (ok ? (int64_t)t * count + e : 0));
        rv[u][0] = ok ? q.x : 0.0f;
        rv[u][1] = ok ? q.y : 0.0f;
        rv[u][2] = ok ? q.z : 0.0f;
        rv[u][3] = ok ? q.w : 0.0f;
        const bool oks = ok && src != nullptr;
        const float4 w = *reinterpret_cast<const float4*>(oks ? src + (int64_t)t * count + e : in);
        sv[u][0] = oks ? w.x : 0.0f;
        sv[u][1] = oks ? w.y : 0.0f;
        sv[u][2] = oks ? w.z : 0.0f;
        sv[u][3] = oks ? w.w : 0.0f;
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool ok = t < p && e + v < count;
          const float x = in[ok ? (int64_t)t * count + e + v : 0];
          rv[u][v] = ok ? x : 0.0f;
          const bool oks = ok && src != nullptr;
          const float y = (src != nullptr ? src : in)[oks ? (int64_t)t * count + e + v : 0];
          sv[u][v] = oks ? y : 0.0f;
        }
      }
    }
  };
  // one MFMA pass: the products G x (tile in sX) back into sX as [k][e], with
  // G = G1, or (TR) its transpose read from the same LDS copy
  auto mfma_pass = [&](const float* sG, auto tr) {
    constexpr bool TR = decltype(tr)::value;
    typename MF::frag_t acc[FR];
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[f][r] = 0.0f;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int t0 = 0; t0 < PM; t0 += 4) {
      const float* bp = &sX[(t0 + lk) * LDX + wave * 16 + lr];
#pragma unroll
      for (int f = 0; f < FR; ++f)
        acc[f] = MF::mac(TR ? &sG[(t0 + lk) * LDG + f * 16 + lr] : &sG[(f * 16 + lr) * LDG + t0 + lk], bp, acc[f]);
    }
    // a wave reads and writes only its own 16 columns of sX, and a wave's LDS
    // accesses complete in order: no block barrier between its operand reads
    // and its product writes
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int f = 0; f < FR; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) sX[(f * 16 + lk * 4 + r) * LDX + wave * 16 + lr] = acc[f][r];
    __syncthreads();
  };

  // prologue: the control block's loads and the matrix in flight together
  const CtlLoad cl = ctl_load(pa.ctl);
  float g1[GU];
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    const int i = tid + u * 256, k = i / PM, t = i % PM;
    const bool ok = k < p && t < p;
    const float v1 = pa.G1[ok ? k * p + t : 0];
    g1[u] = ok ? v1 : 0.0f;
  }
  double a_d, b_d, s_d;
  if (!ctl_eval(pa.ctl, cl, a_d, b_d, s_d, sh, vb)) return;
  const float a = (float)(a_d * s_d), b = (float)b_d;
  const bool use_src = src != nullptr && b != 0.0f;   // b = 0: src never enters
#pragma unroll
  for (int u = 0; u < GU; ++u) {
    const int i = tid + u * 256, k = i / PM, t = i % PM;
    sG1[k * LDG + t] = g1[u];
  }
  double sq = 0.0;
  for (int64_t tile = vb.x; tile < ntiles; tile += pa.gx) {
    const int64_t e0 = tile * NB;
    load_tile(tile);
    __syncthreads();  // the previous tile's x rows have been read from sX (and G1 is staged)
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int i = tid + u * 256;
      const int t = i / (NB / 4), c = (i % (NB / 4)) * 4;
      *reinterpret_cast<float4*>(&sX[t * LDX + c]) = make_float4(rv[u][0], rv[u][1], rv[u][2], rv[u][3]);
    }
    __syncthreads();
    mfma_pass(sG1, std::false_type{});
    // y = a (G1 c) + b src: written out, summed, and staged for the second pass
    // (rows k >= p are zero in both passes)
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int i = tid + u * 256;
      const int k = i / (NB / 4), c = (i % (NB / 4)) * 4;
      const int64_t e = e0 + c;
      float4* rowp = reinterpret_cast<float4*>(&sX[k * LDX + c]);
      const float4 q = *rowp;
      float y[4] = {a * q.x, a * q.y, a * q.z, a * q.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) y[v] += use_src ? b * sv[u][v] : 0.0f;
      if (k < p) {
        float* op = pa.y + (int64_t)k * count + e;
        if (VEC) {
          if (e < count) {
            RowStore<float>::st(op, y);
#pragma unroll
            for (int v = 0; v < 4; ++v) sq += (double)y[v] * (double)y[v];
          }
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (e + v < count) {
              op[v] = y[v];
              sq += (double)y[v] * (double)y[v];
            }
        }
      }
      // positions beyond the slice enter the second pass as zeros
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (e + v >= count) y[v] = 0.0f;
      *rowp = make_float4(y[0], y[1], y[2], y[3]);
    }
    __syncthreads();
    mfma_pass(sG1, std::true_type{});
#pragma unroll
    for (int u = 0; u < XU; ++u) {
      const int i = tid + u * 256;
      const int k = i / (NB / 4), c = (i % (NB / 4)) * 4;
      const int64_t e = e0 + c;
      if (k >= p) continue;
      const float4 q = *reinterpret_cast<const float4*>(&sX[k * LDX + c]);
      const float xv[4] = {q.x, q.y, q.z, q.w};
      TX* xp = (TX*)pa.x + (int64_t)k * count + e;
      if (VEC) {
        if (e < count) RowStore<TX>::st(xp, xv);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (e + v < count) xp[v] = cvt<TX, float>(xv[v]);
      }
    }
  }
  if (pa.ctl.part_out != nullptr) {
    const double tot = block_sum_all(sq, sh);
    if (tid == 0) pa.ctl.part_out[vb.x] = tot;
  }
}

template <typename TX, int PM, bool VEC, bool GROUPED>
__global__ __launch_bounds__(256) void tube_pair_kernel(PairArgs pa_, const PairArgs* grp, const int4* bmap) {
  if constexpr (!GROUPED) {
    tube_pair_kernel_body<TX, PM, VEC>(pa_, hw_block(), false);
  } else {
    VBlock vb;
    const PairArgs g = group_args(grp, bmap, vb);
    tube_pair_kernel_body<TX, PM, VEC>(g, vb, true);
  }
}

bool tube_pair_ok(int64_t p, int vec_dtype) { return vec_dtype == DCTK_F32 && p >= 16 && p <= kMaxTube; }

hipError_t launch_tube_pair(dctk_ctx ctx, hipStream_t s, int x_dtype, int64_t p, int64_t count, const float* c,
                            const float* src, float* y, void* x, const float* G1, const Ctl& ctl,
                            int* nblocks_out) {
  if (!tube_pair_ok(p, DCTK_F32)) return hipErrorInvalidValue;
  // four workgroups per CU (36 KB of LDS each), each walking several tiles
  int64_t blocks = (count + 63) / 64;
  const int64_t cap = 4 * (int64_t)num_cus();
  if (blocks > cap) blocks = cap;
  if (nblocks_out) *nblocks_out = (int)blocks;
  if (ctl.part_out != nullptr && blocks > kRedBlocks) return hipErrorInvalidConfiguration;
  const size_t xe = x_dtype == DCTK_F32 ? 4 : 2;
  const bool vec = (count % 4 == 0) && ((uintptr_t)c % 16 == 0) && ((uintptr_t)src % 16 == 0) &&
                   ((uintptr_t)y % 16 == 0) && ((uintptr_t)x % (4 * xe) == 0);
  PairArgs pa{};
  pa.p = (int)p;
  pa.count = count;
  pa.c = c;
  pa.src = src;
  pa.y = y;
  pa.x = x;
  pa.G1 = G1;
  pa.ctl = ctl;
  const dim3 grid((unsigned)blocks);
#define DCTK_PAIR_V(TX, PM_)                                                                                     \
  do {                                                                                                         \
    if (vec) return launch_kernel(ctx, s, tube_pair_kernel<TX, PM_, true, false>, tube_pair_kernel<TX, PM_, true, true>, grid, 256, 0, pa); \
    return launch_kernel(ctx, s, tube_pair_kernel<TX, PM_, false, false>, tube_pair_kernel<TX, PM_, false, true>, grid, 256, 0, pa); \
  } while (0)
#define DCTK_PAIR_P(TX)            \
  do {                             \
    if (p <= 16) DCTK_PAIR_V(TX, 16); \
    if (p <= 32) DCTK_PAIR_V(TX, 32); \
    if (p <= 48) DCTK_PAIR_V(TX, 48); \
    DCTK_PAIR_V(TX, 64);           \
  } while (0)
  switch (x_dtype) {
    case DCTK_F32: DCTK_PAIR_P(float);
    case DCTK_BF16: DCTK_PAIR_P(bf16_t);
    case DCTK_F16: DCTK_PAIR_P(f16_t);
    default: return hipErrorInvalidValue;
  }
#undef DCTK_PAIR_P
#undef DCTK_PAIR_V
}

template <typename TIN, typename TOUT, typename TC>
static hipError_t launch_tube_t(dctk_ctx ctx, hipStream_t s, int64_t p, int64_t count, const void* in, void* out,
                                const TC* G, const void* src, void* xnorm, const Ctl& ctl, bool scale, bool epi,
                                int* nblocks_out) {
  int64_t nthreads = (count + 3) / 4;
  int64_t blocks = (nthreads + kThreads - 1) / kThreads;
  if (blocks > kRedBlocks) blocks = kRedBlocks;
  if (blocks < 1) blocks = 1;
  if (nblocks_out) *nblocks_out = (int)blocks;
  size_t shmem = (size_t)(p * p) * sizeof(TC);
  bool vec = (count % 4 == 0) && (((uintptr_t)in) % 32 == 0) && (((uintptr_t)out) % 32 == 0) &&
             (src == nullptr || ((uintptr_t)src) % 32 == 0) && (xnorm == nullptr || ((uintptr_t)xnorm) % 32 == 0);
  TubeArgs ta{};
  ta.p = (int)p;
  ta.count = count;
  ta.in = in;
  ta.out = out;
  ta.G = G;
  ta.src = src;
  ta.xnorm = xnorm;
  ta.ctl = ctl;
  const dim3 grid((unsigned)blocks);
#define DCTK_TUBE_LAUNCH(KB, V, S, E) \
  return launch_kernel(ctx, s, tube_kernel<TIN, TOUT, TC, KB, V, S, E, false>, tube_kernel<TIN, TOUT, TC, KB, V, S, E, true>, grid, kThreads, (unsigned)shmem, ta)
#define DCTK_TUBE_SE(KB, V)                                  \
  do {                                                       \
    if (scale && epi) DCTK_TUBE_LAUNCH(KB, V, true, true);    \
    else if (scale) DCTK_TUBE_LAUNCH(KB, V, true, false);     \
    else if (epi) DCTK_TUBE_LAUNCH(KB, V, false, true);       \
    else DCTK_TUBE_LAUNCH(KB, V, false, false);               \
  } while (0)
  if (p <= 4) {
    if (vec) DCTK_TUBE_SE(4, true); else DCTK_TUBE_SE(4, false);
  } else {
    if (vec) DCTK_TUBE_SE(8, true); else DCTK_TUBE_SE(8, false);
  }
#undef DCTK_TUBE_SE
#undef DCTK_TUBE_LAUNCH
}

// in_dtype: element type of `in` (F64/F32); out_dtype: of `out` (F64, F32, BF16, F16).
// A transform whose output is a GEMM operand applies the input side of the
// control block (scale); one whose input is a GEMM result applies the epilogue
// side (epi).
hipError_t launch_tube(dctk_ctx ctx, hipStream_t s, int in_dtype, int out_dtype, int64_t p, int64_t count,
                       const void* in, void* out, const double* Gd, const float* Gf,
                       const void* src, void* xnorm, const Ctl& ctl, bool scale, bool epi, int* nblocks_out) {
  if (in_dtype == DCTK_F64) {
    if (out_dtype != DCTK_F64) return hipErrorInvalidValue;
    return launch_tube_t<double, double, double>(ctx, s, p, count, in, out, Gd, src, xnorm, ctl, scale, epi, nblocks_out);
  }
  // long tubes on the matrix cores (unless the 64-position blocks would exceed the partial-sum slots)
  const bool mfma = p >= 16 && p <= kMaxTube && !(epi && ctl.part_out != nullptr && (count + 63) / 64 > kRedBlocks);
  switch (out_dtype) {
    case DCTK_F32:
      if (mfma) return launch_tube_mfma<float>(ctx, s, p, count, in, out, Gf, src, xnorm, ctl, scale, epi, nblocks_out);
      return launch_tube_t<float, float, float>(ctx, s, p, count, in, out, Gf, src, xnorm, ctl, scale, epi, nblocks_out);
    case DCTK_BF16:
      if (src) return hipErrorInvalidValue;
      if (mfma)
        return launch_tube_mfma<bf16_t>(ctx, s, p, count, in, out, Gf, nullptr, xnorm, ctl, scale, false, nblocks_out);
      return launch_tube_t<float, bf16_t, float>(ctx, s, p, count, in, out, Gf, nullptr, xnorm, ctl, scale, false,
                                                 nblocks_out);
    case DCTK_F16:
      if (src) return hipErrorInvalidValue;
      if (mfma)
        return launch_tube_mfma<f16_t>(ctx, s, p, count, in, out, Gf, nullptr, xnorm, ctl, scale, false, nblocks_out);
      return launch_tube_t<float, f16_t, float>(ctx, s, p, count, in, out, Gf, nullptr, xnorm, ctl, scale, false,
                                                nblocks_out);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace dctk
