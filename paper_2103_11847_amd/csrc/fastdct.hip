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
// element crosses HBM once each way.  The work is HBM-bound: about
// 5 p log2 p flops per tube against 2 p elements moved.
#include <cmath>

#include "fastdct.h"

namespace dctk {

namespace {

constexpr int kFastThreads = 256;
constexpr int kFastLds = 16384;  // bytes of each of the three E-element buffers

template <typename T>
struct FastCfg {
  static constexpr int E = kFastLds / (int)sizeof(T);  // elements per workgroup
};

struct FastArgs {
  const void* in;
  void* out;
  int64_t count;  // positions per slice
  int p, logp, nb, lognb;
  int inv;    // 0: F core, 1: F^{-1} core
  int pre;    // before F: 0 none, 1 (I + Z), 2 (I + Z^T)^{-1}
  int post;   // after F^{-1}: 0 none, 1 (I + Z^T), 2 (I + Z)^{-1}
  int scale;  // diagonal: 0 D^{-1}, 1 D N^{-1}, 2 S (after F); 3 D, 4 N D^{-1}, 5 S^{-1} (before F^{-1})
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

template <typename T>
__global__ __launch_bounds__(kFastThreads) void tube_fast_kernel(FastArgs a) {
  constexpr int E = FastCfg<T>::E;
  __shared__ T rb[E];              // the tubes as real values
  __shared__ T re[E], im[E];       // complex FFT buffer, position-major
  __shared__ T twr[E / 2], twi[E / 2];  // exp(-2 pi i m / p), m < p/2
  __shared__ T part[kFastThreads];
  const T* in = (const T*)a.in;
  T* out = (T*)a.out;
  const int tid = threadIdx.x;
  const int p = a.p, nb = a.nb, lognb = a.lognb, logp = a.logp;
  const int64_t count = a.count;
  const int64_t e0 = (int64_t)blockIdx.x * nb;

  for (int m = tid; m < p / 2; m += kFastThreads) {
    T s, c;
    sc_pi((T)(2 * m) / (T)p, &s, &c);
    twr[m] = c;
    twi[m] = -s;
  }
  // load the block: row t holds positions e0 .. e0 + nb - 1 of slice t
  for (int i = tid; i < E; i += kFastThreads) {
    const int t = i >> lognb, j = i & (nb - 1);
    const int64_t e = e0 + j;
    const int64_t ec = e < count ? e : count - 1;
    const T v = in[(int64_t)t * count + ec];
    rb[i] = e < count ? v : (T)0;
  }
  __syncthreads();
  if (a.pre == 2) {
    alt_scan<T, false>(rb, part, p, nb, lognb);
    __syncthreads();
  }
  const T two_p = (T)(2 * p);
  // FFT input at bit-reversed positions
  for (int i = tid; i < E; i += kFastThreads) {
    const int t = i >> lognb, j = i & (nb - 1);
    if (!a.inv) {
      T y = rb[i];
      if (a.pre == 1 && t + 1 < p) y += rb[i + nb];
      const int n = (t & 1) ? p - 1 - (t >> 1) : (t >> 1);  // even entries, then odd ones reversed
      const int d = bit_reverse(n, logp) * nb + j;
      re[d] = y;
      im[d] = 0;
    } else {
      // V_k = exp(i pi k / (2p)) (X_k - i X_{p-k}), X_p = 0, with X = R x
      const int k = t;
      T s, c;
      sc_pi((T)k / two_p, &s, &c);
      const T xk = rb[i] * fast_scale<T>(a.scale, k, p, c);
      T xpk = 0;
      if (k) {
        T s2, c2;
        sc_pi((T)(p - k) / two_p, &s2, &c2);
        xpk = rb[(p - k) * nb + j] * fast_scale<T>(a.scale, p - k, p, c2);
      }
      const int d = bit_reverse(k, logp) * nb + j;
      re[d] = c * xk + s * xpk;
      im[d] = s * xk - c * xpk;
    }
  }
  __syncthreads();
  // radix-2 decimation in time, in place; twiddle exp(-+2 pi i pos / (2h)) = tw[pos * p / (2h)]
  for (int h = 1, sh = logp - 1; h < p; h <<= 1, --sh) {
    for (int q = tid; q < E / 2; q += kFastThreads) {
      const int b = q >> lognb, j = q & (nb - 1);
      const int pos = b & (h - 1);
      const int i0 = (((b - pos) << 1) + pos) * nb + j, i1 = i0 + h * nb;
      const T wr = twr[pos << sh], wi = a.inv ? -twi[pos << sh] : twi[pos << sh];
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
  if (!a.inv) {
    // F_k = Re(exp(-i pi k / (2p)) V_k), then the diagonal
    for (int i = tid; i < E; i += kFastThreads) {
      const int k = i >> lognb, j = i & (nb - 1);
      T s, c;
      sc_pi((T)k / two_p, &s, &c);
      const T f = re[i] * c + im[i] * s;
      const int64_t e = e0 + j;
      if (e < count) out[(int64_t)k * count + e] = f * fast_scale<T>(a.scale, k, p, c);
    }
    return;
  }
  // y_t = v_n / p with n the reordered index of t
  const T inv_p = (T)1 / (T)p;
  for (int i = tid; i < E; i += kFastThreads) {
    const int t = i >> lognb, j = i & (nb - 1);
    const int n = (t & 1) ? p - 1 - (t >> 1) : (t >> 1);
    rb[i] = re[n * nb + j] * inv_p;
  }
  __syncthreads();
  if (a.post == 2) {
    alt_scan<T, true>(rb, part, p, nb, lognb);
    __syncthreads();
  }
  for (int i = tid; i < E; i += kFastThreads) {
    const int t = i >> lognb, j = i & (nb - 1);
    T y = rb[i];
    if (a.post == 1 && t > 0) y += rb[i - nb];
    const int64_t e = e0 + j;
    if (e < count) out[(int64_t)t * count + e] = y;
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

hipError_t launch_tube_fast(dctk_ctx ctx, hipStream_t s, int tube, int which, int dtype, int64_t p, int64_t count,
                            const void* in, void* out) {
  if (recording(ctx)) return hipErrorNotSupported;
  if ((dtype != DCTK_F64 && dtype != DCTK_F32) || !tube_fast_shape_ok(dtype, p) || count <= 0)
    return hipErrorInvalidValue;
  FastArgs a{};
  a.in = in;
  a.out = out;
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
  const int64_t blocks = (count + a.nb - 1) / a.nb;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (dtype == DCTK_F64)
    tube_fast_kernel<double><<<dim3((unsigned)blocks), dim3(kFastThreads), 0, s>>>(a);
  else
    tube_fast_kernel<float><<<dim3((unsigned)blocks), dim3(kFastThreads), 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace dctk
