// Tube transforms in O(p log p) operations per tube for power-of-two tube
// lengths (the fast DCT that Sec. 1 and Sec. 2.1 credit the method with).
//
// Every matrix of the transform family factors into one DCT-II core and
// O(p) steps around it.  With F the unnormalised DCT-II,
// (F y)_k = sum_t cos(pi k (2t+1) / (2p)) y_t, D = diag(cos(pi k / (2p))),
// N = diag(p, p/2, ..., p/2) (the row norms of F squared, F F^T = N) and
// S = diag(sqrt((2 - [k = 0]) / p)), eq. (dft1) reads C_n = S F, the first
// column of C_n is S D, and Remark 2.1 gives
//   M      = W^{-1} C_n (I + Z) = D^{-1} F (I + Z)
//   M^{-1} = (I + Z)^{-1} F^{-1} D
//   M^{T}  = (I + Z^T) F^{-1} N D^{-1}        (F^T = F^{-1} N)
//   M^{-T} = D N^{-1} F (I + Z^T)^{-1}
//   C_n = C_n^{-T} = S F,  C_n^{-1} = C_n^T = F^{-1} S^{-1}.
// F is one complex FFT of length p of the tube reordered even entries first,
// odd entries reversed after them, followed by a quarter-wave rotation of
// each output (Makhoul's algorithm); F^{-1} runs the same steps backwards
// with the inverse FFT.  (I + Z)^{-1} and (I + Z^T)^{-1} are alternating
// suffix and prefix sums.
//
// A workgroup owns NB = E / p neighbouring tubes (E = 4096 FP32 or 2048 FP64
// elements): it loads the p x NB block row by row (NB consecutive positions
// of each slice), runs every step in LDS and writes the block back, so each
// element crosses HBM once each way.  Workgroups stay resident and loop over
// blocks of tubes, loading the next block into registers while the current
// one is transformed; the row constants (rotations, diagonals) and the FFT
// twiddles are computed once per workgroup.  The work is HBM-bound: about
// 5 p log2 p flops per tube against 2 p elements moved.
#include <algorithm>
#include <cmath>

#include "fastdct.h"

namespace dctk {

namespace {

constexpr int kFastThreads = 512;
constexpr int kFastLds = 16384;  // bytes of each of the three E-element buffers

template <typename T>
struct FastCfg {
  static constexpr int E = kFastLds / (int)sizeof(T);  // elements per workgroup
};

struct FastArgs {
  int gx, gy, gz;  // the instance's grid (recorded by launch_kernel)
  int p, logp, nb, lognb;
  int group;  // blocks of tubes sharing 128-byte lines, taken by one workgroup back to back
  int inv;    // 0: F core, 1: F^{-1} core (the kernel's INV)
  int pre;    // before F: 0 none, 1 (I + Z), 2 (I + Z^T)^{-1}
  int post;   // after F^{-1}: 0 none, 1 (I + Z^T), 2 (I + Z)^{-1}
  int scale;  // diagonal: 0 D^{-1}, 1 D N^{-1}, 2 S (after F); 3 D, 4 N D^{-1}, 5 S^{-1} (before F^{-1})
  int pad_;
  int64_t count;  // positions per slice
  const void* in;
  void* out;
  // inside a c-product: the input side of the control block (SCALE: the
  // input is multiplied by its scale s, and s * in written to xnorm when
  // given) or its output side (EPI: out = a * (in x_3 G) + b * src, with
  // per-workgroup partial sums of out^2 in ctl.part_out)
  const void* src;  // p x count, or null
  void* xnorm;      // p x count, or null
  Ctl ctl;
};

__device__ inline void sc_pi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ inline void sc_pi(double x, double* s, double* c) { sincospi(x, s, c); }

// diagonal entry k of the scaling `code`; d = cos(pi k / (2p))
template <typename T>
__device__ inline T fast_scale(int code, int k, int p, T d) {
  const T n = k ? (T)p * (T)0.5 : (T)p;
  const T sq = sqrt((k ? (T)2 : (T)1) / (T)p);
  switch (code) {
    case 0: return (T)1 / d;
    case 1: return d / n;
    case 2: return sq;
    case 3: return d;
    case 4: return n / d;
    default: return (T)1 / sq;
  }
}

// Index of element i of the FFT buffers: bits 4-5 are XORed with bits 6-7,
// a bijection on every 256 elements, so that the four operands of a
// radix-4 group (16 tubes apart in a block of 16) fall in different banks.
__device__ inline int sw(int i) { return i ^ (((i >> 6) & 3) << 4); }

__device__ inline int bit_reverse(int n, int bits) { return (int)(__brev((unsigned)n) >> (32 - bits)); }

// In place over each of the NB columns of buf (p x NB, column j holds a
// tube): x_t = sum over i <= t (prefix) or i >= t (suffix) of (-1)^(t-i) y_i,
// i.e. the solution of (I + Z^T) x = y or (I + Z) x = y.  Thread (c, j) scans
// chunk c of column j; the chunk sums meet in `part`.
template <typename T, bool SUFFIX>
__device__ void alt_scan(T* buf, T* part, int p, int nb, int lognb) {
  const int tid = threadIdx.x;
  const int j = tid & (nb - 1), c = tid >> lognb;
  const int nc = kFastThreads >> lognb;  // chunks per column
  const int len = p / nc;
  T sum = 0;
  for (int u = 0; u < len; ++u) {
    const int t = c * len + u;
    const T v = buf[t * nb + j];
    sum += (t & 1) ? -v : v;
  }
  part[tid] = sum;
  __syncthreads();
  T run = 0;
  if (!SUFFIX) {
    for (int q = 0; q < c; ++q) run += part[q * nb + j];
    for (int u = 0; u < len; ++u) {
      const int t = c * len + u;
      const T v = buf[t * nb + j];
      run += (t & 1) ? -v : v;
      buf[t * nb + j] = (t & 1) ? -run : run;
    }
  } else {
    for (int q = c + 1; q < nc; ++q) run += part[q * nb + j];
    for (int u = len - 1; u >= 0; --u) {
      const int t = c * len + u;
      const T v = buf[t * nb + j];
      run += (t & 1) ? -v : v;
      buf[t * nb + j] = (t & 1) ? -run : run;
    }
  }
}

// T: the arithmetic and input type; TO: the output type (T, or a 16-bit GEMM
// operand type for a forward transform feeding the slice products).
template <typename T, typename TO, bool INV, bool PAIR, bool SCALE, bool EPI>
__device__ __forceinline__ void tube_fast_body(const FastArgs& a, const VBlock vb) {
  static_assert(!(SCALE && INV) && !(EPI && !INV), "the input side precedes F, the output side follows F^{-1}");
  constexpr int E = FastCfg<T>::E;
  // With two or more tubes per block (PAIR), tubes j and j + nb/2 share one
  // complex FFT as its real and imaginary parts: the forward input and the
  // inverse output are real, so each FFT serves two tubes.
  constexpr int NQ4 = PAIR ? E / 8 : E / 4;  // radix-4 groups per pass
  constexpr int NQ2 = PAIR ? E / 4 : E / 2;  // radix-2 butterflies of a last stage
  constexpr int U = E / kFastThreads;  // elements per thread and block of tubes
  __shared__ T rb[E];              // the tubes as real values
  __shared__ T re[E], im[E];       // complex FFT buffer, position-major
  __shared__ T twr[E / 2], twi[E / 2];  // exp(-2 pi i m / p), m < p/2
  __shared__ T part[kFastThreads];
  __shared__ double shc[2 * (kFastThreads / 64 + 1)];  // the control block's reductions
  const T* in = (const T*)a.in;
  TO* out = (TO*)a.out;
  const int tid = threadIdx.x;
  // the control block's loads first, so they are in flight with the first block's
  CtlLoad cl{};
  if constexpr (SCALE || EPI) cl = ctl_load(a.ctl);
  const int p = a.p, nb = a.nb, lognb = a.lognb, logp = a.logp;
  const int64_t count = a.count;
  const int64_t ntiles = (count + nb - 1) / nb;
  const T two_p = (T)(2 * p);

  // Once per workgroup (it stays resident over many blocks of tubes): the FFT
  // twiddles, and for the rows k this thread touches the rotation
  // exp(-i pi k / (2p)) and the diagonal entries at k (and at p - k).
  for (int m = tid; m < p / 2; m += kFastThreads) {
    T s, c;
    sc_pi((T)(2 * m) / (T)p, &s, &c);
    twr[m] = c;
    twi[m] = -s;
  }
  // A thread keeps one position j of the block (nb divides the thread count)
  // and rows t0, t0 + RU, t0 + 2 RU, ...
  const int jt = tid & (nb - 1), t0 = tid >> lognb, ru = kFastThreads >> lognb;
  const int64_t rstride = (int64_t)ru * count;
  const int nbc = PAIR ? nb >> 1 : nb, lognbc = PAIR ? lognb - 1 : lognb;  // complex columns
  const int jc = jt & (nbc - 1);                  // this thread's complex column
  const bool hi = PAIR && jt >= nbc;              // imaginary part of it
  T rc[U], rs[U], rq[U], rq2[INV ? U : 1];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = t0 + u * ru;
    sc_pi((T)k / two_p, &rs[u], &rc[u]);
    rq[u] = fast_scale<T>(a.scale, k, p, rc[u]);
    if (INV) {
      T s2, c2;
      sc_pi((T)(p - k) / two_p, &s2, &c2);
      rq2[INV ? u : 0] = k ? fast_scale<T>(a.scale, p - k, p, c2) : (T)0;
    }
  }
  // row t of a block holds positions e0 .. e0 + nb - 1 of slice t; clamped
  // addresses keep every load in bounds, the tail is zeroed when staged
  T pf[U];
  auto fetch = [&](int64_t tile) {
    const int64_t e = tile * nb + jt;
    const T* src = in + (int64_t)t0 * count + (e < count ? e : count - 1);
#pragma unroll
    for (int u = 0; u < U; ++u) pf[u] = src[u * rstride];
  };
  // Workgroup w takes groups w, w + G, w + 2G, ... (G = gridDim.x) of `group`
  // consecutive blocks of tubes; a group spans whole 128-byte lines of every
  // slice, so a line's second part is read from the CU's own L2.  The grid
  // never exceeds the number of groups, so the first block exists.
  const int grp = a.group;
  auto tile_of = [&](int64_t n) { return ((int64_t)vb.x + n / grp * a.gx) * grp + n % grp; };
  int64_t n = 0, tile = tile_of(0);
  fetch(tile);
  T sc = (T)1, ea = (T)1, eb = (T)0;
  bool use_src = false;
  if constexpr (SCALE || EPI) {
    double ad, bd, sd;
    if (!ctl_eval(a.ctl, cl, ad, bd, sd, shc, vb)) return;
    if (SCALE) sc = (T)sd;
    if (EPI) {
      ea = (T)ad;
      eb = (T)bd;
      use_src = a.src != nullptr && bd != 0.0;  // b = 0: src never enters
    }
  }
  T* xn = (T*)a.xnorm;
  // without src the epilogue reads this block's own input rows again (from
  // the cache) instead of a branch around its loads
  const T* sp = use_src ? (const T*)a.src : in;
  double sq = 0.0;
  T sv[EPI ? U : 1];
  for (; tile < ntiles; tile = tile_of(++n)) {
    const int64_t e0 = tile * nb;
    const bool live = e0 + jt < count;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T v = live ? (SCALE ? sc * pf[u] : pf[u]) : (T)0;
      rb[tid + u * kFastThreads] = v;
      if (SCALE && xn != nullptr && live) xn[(int64_t)t0 * count + e0 + jt + u * rstride] = v;
    }
    __syncthreads();
    // the next block of tubes is in flight while this one is transformed
    const int64_t next = tile_of(n + 1);
    fetch(next < ntiles ? next : tile);
    if (a.pre == 2) {
      alt_scan<T, false>(rb, part, p, nb, lognb);
      __syncthreads();
    }
    // FFT input at bit-reversed positions
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = tid + u * kFastThreads;
      const int t = i >> lognb, j = i & (nb - 1);
      if (!INV) {
        T y = rb[i];
        if (a.pre == 1 && t + 1 < p) y += rb[i + nb];
        const int n = (t & 1) ? p - 1 - (t >> 1) : (t >> 1);  // even entries, then odd ones reversed
        if (!PAIR) {
          const int d = bit_reverse(n, logp) * nb + j;
          re[sw(d)] = y;
          im[sw(d)] = 0;
        } else {
          const int d = sw(bit_reverse(n, logp) * nbc + jc);
          if (hi) im[d] = y;
          else re[d] = y;
        }
      } else if (PAIR) {
        // Z_k = V_k(tube jc) + i V_k(tube jc + nbc), formed by the low half of the threads
        if (!hi) {
          const int k = t;
          const T xk = rb[i] * rq[u], yk = rb[i + nbc] * rq[u];
          const int ip = (p - k) * nb + j;
          const T xpk = k ? rb[ip] * rq2[INV ? u : 0] : (T)0;
          const T ypk = k ? rb[ip + nbc] * rq2[INV ? u : 0] : (T)0;
          const T var = rc[u] * xk + rs[u] * xpk, vai = rs[u] * xk - rc[u] * xpk;
          const T vbr = rc[u] * yk + rs[u] * ypk, vbi = rs[u] * yk - rc[u] * ypk;
          const int d = sw(bit_reverse(k, logp) * nbc + jc);
          re[d] = var - vbi;
          im[d] = vai + vbr;
        }
      } else {
        // V_k = exp(i pi k / (2p)) (X_k - i X_{p-k}), X_p = 0, with X = R x
        const int k = t;
        const T xk = rb[i] * rq[u];
        const T xpk = k ? rb[(p - k) * nb + j] * rq2[INV ? u : 0] : (T)0;
        const int d = bit_reverse(k, logp) * nb + j;
        re[sw(d)] = rc[u] * xk + rs[u] * xpk;
        im[sw(d)] = rs[u] * xk - rc[u] * xpk;
      }
    }
    __syncthreads();
    // Decimation in time, in place, two radix-2 stages (half sizes h and 2h)
    // per pass in registers; a last radix-2 stage when log2 p is odd.  The
    // twiddle exp(-+2 pi i m / (2H)) of a stage with half size H is
    // tw[m * p / (2H)].
    int h = 1, sh = logp - 1;
    for (; 2 * h < p; h <<= 2, sh -= 2) {
#pragma unroll 2
      for (int q = tid; q < NQ4; q += kFastThreads) {
        const int b = q >> lognbc, j = q & (nbc - 1);
        const int pos = b & (h - 1);
        const int i0 = (((b - pos) << 2) + pos) * nbc + j, hs = h * nbc;
        const int k1 = pos << sh, k2 = pos << (sh - 1), k3 = (pos + h) << (sh - 1);
        const T w1r = twr[k1], w1i = INV ? -twi[k1] : twi[k1];
        const T w2r = twr[k2], w2i = INV ? -twi[k2] : twi[k2];
        const T w3r = twr[k3], w3i = INV ? -twi[k3] : twi[k3];
        const int x0 = sw(i0), x1 = sw(i0 + hs), x2 = sw(i0 + 2 * hs), x3 = sw(i0 + 3 * hs);
        const T a0r = re[x0], a0i = im[x0], a1r = re[x1], a1i = im[x1];
        const T a2r = re[x2], a2i = im[x2], a3r = re[x3], a3i = im[x3];
        // stage h: (a0, a1) and (a2, a3) with w1
        T tr = w1r * a1r - w1i * a1i, ti = w1r * a1i + w1i * a1r;
        const T b0r = a0r + tr, b0i = a0i + ti, b1r = a0r - tr, b1i = a0i - ti;
        tr = w1r * a3r - w1i * a3i;
        ti = w1r * a3i + w1i * a3r;
        const T b2r = a2r + tr, b2i = a2i + ti, b3r = a2r - tr, b3i = a2i - ti;
        // stage 2h: (b0, b2) with w2, (b1, b3) with w3
        tr = w2r * b2r - w2i * b2i;
        ti = w2r * b2i + w2i * b2r;
        re[x0] = b0r + tr;
        im[x0] = b0i + ti;
        re[x2] = b0r - tr;
        im[x2] = b0i - ti;
        tr = w3r * b3r - w3i * b3i;
        ti = w3r * b3i + w3i * b3r;
        re[x1] = b1r + tr;
        im[x1] = b1i + ti;
        re[x3] = b1r - tr;
        im[x3] = b1i - ti;
      }
      __syncthreads();
    }
    if (h < p) {  // h == p / 2: the last radix-2 stage, twiddle index pos (sh == 0)
#pragma unroll 2
      for (int q = tid; q < NQ2; q += kFastThreads) {
        const int pos = q >> lognbc, j = q & (nbc - 1);
        const int i0 = sw(pos * nbc + j), i1 = sw(pos * nbc + j + h * nbc);
        const T wr = twr[pos], wi = INV ? -twi[pos] : twi[pos];
        const T br = re[i1], bi = im[i1];
        const T tr = wr * br - wi * bi, ti = wr * bi + wi * br;
        const T ar = re[i0], ai = im[i0];
        re[i0] = ar + tr;
        im[i0] = ai + ti;
        re[i1] = ar - tr;
        im[i1] = ai - ti;
      }
      __syncthreads();
    }
    TO* dst = out + (int64_t)t0 * count + e0 + jt;
    if (!INV) {
      // F_k = Re(exp(-i pi k / (2p)) V_k), then the diagonal
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = tid + u * kFastThreads;
        T f;
        if (!PAIR) {
          f = re[sw(i)] * rc[u] + im[sw(i)] * rs[u];
        } else {
          // this tube's spectrum from Z_k and Z_{p-k} of the shared FFT
          const int k = t0 + u * ru;
          const int zk = sw(k * nbc + jc), zp = sw(((p - k) & (p - 1)) * nbc + jc);
          const T zr = re[zk], zi = im[zk], wr = re[zp], wi = im[zp];
          const T vr = hi ? zi + wi : zr + wr, vi = hi ? wr - zr : zi - wi;
          f = (T)0.5 * (vr * rc[u] + vi * rs[u]);
        }
        if (live) dst[u * rstride] = cvt<TO, T>(f * rq[u]);
      }
    } else {
      // the epilogue's src rows, in flight while the output is reordered (and
      // scanned): loaded here rather than with the input, where they would
      // hold registers through the FFT
      if constexpr (EPI) {
        const T* s0 = sp + (int64_t)t0 * count + (live ? e0 + jt : count - 1);
#pragma unroll
        for (int u = 0; u < U; ++u) sv[u] = s0[u * rstride];
      }
      // y_t = v_n / p with n the reordered index of t
      const T inv_p = (T)1 / (T)p;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = tid + u * kFastThreads;
        const int t = i >> lognb, j = i & (nb - 1);
        const int n = (t & 1) ? p - 1 - (t >> 1) : (t >> 1);
        if (!PAIR) rb[i] = re[sw(n * nb + j)] * inv_p;
        else rb[i] = (hi ? im : re)[sw(n * nbc + jc)] * inv_p;
      }
      __syncthreads();
      if (a.post == 2) {
        alt_scan<T, true>(rb, part, p, nb, lognb);
        __syncthreads();
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = tid + u * kFastThreads;
        T y = rb[i];
        if (a.post == 1 && t0 + u * ru > 0) y += rb[i - nb];
        if constexpr (EPI) {
          y = ea * y + (use_src ? eb * sv[u] : (T)0);
          if (live) sq += (double)y * (double)y;
        }
        if (live) dst[u * rstride] = cvt<TO, T>(y);
      }
    }
    __syncthreads();  // the buffers are rewritten by the next block of tubes
  }
  if constexpr (EPI) {
    if (a.ctl.part_out != nullptr) {
      const double tot = block_sum_all(sq, shc);
      if (tid == 0) a.ctl.part_out[vb.x] = tot;
    }
  }
}

template <typename T, typename TO, bool INV, bool PAIR, bool SCALE, bool EPI, bool GROUPED>
__global__ __launch_bounds__(kFastThreads, 4) void tube_fast_kernel(FastArgs a_, const FastArgs* grp,
                                                                    const int4* bmap) {
  if constexpr (!GROUPED) {
    tube_fast_body<T, TO, INV, PAIR, SCALE, EPI>(a_, hw_block());
  } else {
    VBlock vb;
    const FastArgs g = group_args(grp, bmap, vb);
    tube_fast_body<T, TO, INV, PAIR, SCALE, EPI>(g, vb);
  }
}

int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t)1 << l < v) ++l;
  return l;
}

}  // namespace

int tube_fast_max(int dtype) { return dtype == DCTK_F64 ? FastCfg<double>::E : FastCfg<float>::E; }

bool tube_fast_shape_ok(int dtype, int64_t p) {
  return p >= kFastMinTube && p <= tube_fast_max(dtype) && (p & (p - 1)) == 0;
}

// The arguments of transform `which` of family `tube` on p x count elements
// of type `dtype`, and the number of resident workgroups.
static hipError_t fast_setup(int tube, int which, int dtype, int64_t p, int64_t count, FastArgs& a, int64_t& blocks) {
  if ((dtype != DCTK_F64 && dtype != DCTK_F32) || !tube_fast_shape_ok(dtype, p) || count <= 0)
    return hipErrorInvalidValue;
  a = FastArgs{};
  a.count = count;
  a.p = (int)p;
  a.logp = ilog2(p);
  const int E = tube_fast_max(dtype);
  a.nb = E / (int)p;
  a.lognb = ilog2(a.nb);
  const bool th = tube == DCTK_TUBE_TH;
  switch (which) {
    case DCTK_MAT_L: a.inv = 0; a.pre = th ? 1 : 0; a.scale = th ? 0 : 2; break;
    case DCTK_MAT_LINVT: a.inv = 0; a.pre = th ? 2 : 0; a.scale = th ? 1 : 2; break;
    case DCTK_MAT_LINV: a.inv = 1; a.post = th ? 2 : 0; a.scale = th ? 3 : 5; break;
    case DCTK_MAT_LT: a.inv = 1; a.post = th ? 1 : 0; a.scale = th ? 4 : 5; break;
    default: return hipErrorInvalidValue;
  }
  const int64_t tiles = (count + a.nb - 1) / a.nb;
  // Blocks of tubes narrower than a 128-byte line go to one workgroup in
  // groups, while a group's lines (p of them) still fit the L2 share of the
  // workgroups resident on an XCD (p <= 512).
  const int seg = a.nb * (dtype == DCTK_F64 ? 8 : 4);
  a.group = (p <= 512 && seg < 128) ? 128 / seg : 1;
  const int64_t groups = (tiles + a.group - 1) / a.group;
  // resident workgroups (two fit a CU's LDS, 16 waves), each looping over groups
  blocks = std::min<int64_t>(groups, 2 * (int64_t)num_cus());
  return hipSuccess;
}

hipError_t launch_tube_fast(dctk_ctx ctx, hipStream_t s, int tube, int which, int dtype, int64_t p, int64_t count,
                            const void* in, void* out) {
  if (recording(ctx)) return hipErrorNotSupported;
  FastArgs a;
  int64_t blocks = 0;
  hipError_t e = fast_setup(tube, which, dtype, p, count, a, blocks);
  if (e != hipSuccess) return e;
  a.in = in;
  a.out = out;
  a.ctl.kind = CTL_PLAIN;
  const dim3 g((unsigned)blocks);
  const bool pair = a.nb >= 2;
#define DCTK_FAST_PLAIN(T, I, P) \
  return launch_kernel(ctx, s, tube_fast_kernel<T, T, I, P, false, false, false>, \
                       tube_fast_kernel<T, T, I, P, false, false, false>, g, kFastThreads, 0, a)
#define DCTK_FAST_T(T)                                              \
  do {                                                              \
    if (a.inv) {                                                    \
      if (pair) DCTK_FAST_PLAIN(T, true, true);                     \
      DCTK_FAST_PLAIN(T, true, false);                              \
    }                                                               \
    if (pair) DCTK_FAST_PLAIN(T, false, true);                      \
    DCTK_FAST_PLAIN(T, false, false);                               \
  } while (0)
  if (dtype == DCTK_F64) DCTK_FAST_T(double);
  DCTK_FAST_T(float);
#undef DCTK_FAST_T
#undef DCTK_FAST_PLAIN
}

hipError_t launch_tube_fast_ctl(dctk_ctx ctx, hipStream_t s, int tube, int which, int in_dtype, int out_dtype,
                                int64_t p, int64_t count, const void* in, void* out, const void* src, void* xnorm,
                                const Ctl& ctl, bool scale, bool epi, int* nblocks_out) {
  FastArgs a;
  int64_t blocks = 0;
  hipError_t e = fast_setup(tube, which, in_dtype, p, count, a, blocks);
  if (e != hipSuccess) return e;
  // the input side belongs to F (the transforms L, L^{-T}), the output side to F^{-1} (L^{-1}, L^T)
  if (scale == epi || (scale && a.inv) || (epi && !a.inv)) return hipErrorInvalidValue;
  if (epi && out_dtype != in_dtype) return hipErrorInvalidValue;
  if (in_dtype == DCTK_F64 && out_dtype != DCTK_F64) return hipErrorInvalidValue;
  if (epi && ctl.part_out != nullptr && blocks > kRedBlocks) return hipErrorInvalidConfiguration;
  if (nblocks_out) *nblocks_out = (int)blocks;
  a.in = in;
  a.out = out;
  a.src = epi ? src : nullptr;
  a.xnorm = scale ? xnorm : nullptr;
  a.ctl = ctl;
  const dim3 g((unsigned)blocks);
  const bool pair = a.nb >= 2;
#define DCTK_FAST_CTL(T, TO, I, P, S, E_)                                                         \
  return launch_kernel(ctx, s, tube_fast_kernel<T, TO, I, P, S, E_, false>,                       \
                       tube_fast_kernel<T, TO, I, P, S, E_, true>, g, kFastThreads, 0, a)
#define DCTK_FAST_FWD(T, TO)                                  \
  do {                                                        \
    if (pair) DCTK_FAST_CTL(T, TO, false, true, true, false); \
    DCTK_FAST_CTL(T, TO, false, false, true, false);          \
  } while (0)
#define DCTK_FAST_INV(T)                                      \
  do {                                                        \
    if (pair) DCTK_FAST_CTL(T, T, true, true, false, true);   \
    DCTK_FAST_CTL(T, T, true, false, false, true);            \
  } while (0)
  if (in_dtype == DCTK_F64) {
    if (scale) DCTK_FAST_FWD(double, double);
    DCTK_FAST_INV(double);
  }
  if (epi) DCTK_FAST_INV(float);
  switch (out_dtype) {
    case DCTK_F32: DCTK_FAST_FWD(float, float);
    case DCTK_BF16: DCTK_FAST_FWD(float, bf16_t);
    case DCTK_F16: DCTK_FAST_FWD(float, f16_t);
    default: return hipErrorInvalidValue;
  }
#undef DCTK_FAST_INV
#undef DCTK_FAST_FWD
#undef DCTK_FAST_CTL
}

}  // namespace dctk
