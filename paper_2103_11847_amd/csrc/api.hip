// The C-ABI of libdctkrylov: contexts, operators, tube transforms, c-products,
// Krylov workspaces and the DC-LSQR / DC-GK / DC-GMRES solvers.
//
// Everything after argument validation is enqueued on the context's stream;
// Krylov scalars (alpha, beta, h, the LSQR rotations, lambda, y) live in a
// device-resident state so a solve synchronises once, at the end.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"
#include "projected.h"
#include "fastdct.h"

static_assert(dctk::PROF_KINDS == DCTK_PROF_KINDS, "profiler kinds");

using namespace dctk;

namespace dctk {

int hip_fail(dctk_ctx ctx, hipError_t e) {
  if (ctx) ctx->last_hip_error = (int)e;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return DCTK_ENOMEM;
  return DCTK_EHIP;
}

static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + nb && pb < pa + na;
}

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Profiler {
  struct Rec { hipEvent_t a, b; int kind; };
  std::vector<Rec> recs;
  hipEvent_t open = nullptr;
};

void prof_begin(dctk_ctx ctx, int kind) {
  (void)kind;
  if (!ctx || !ctx->prof || ctx->rec) return;
  Profiler* P = (Profiler*)ctx->prof;
  hipEvent_t ev;
  if (hipEventCreate(&ev) != hipSuccess) return;
  (void)hipEventRecord(ev, ctx->stream);
  P->open = ev;
}

void prof_kernel(dctk_ctx ctx, int kind, hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (!ctx || !ctx->prof) return;
  Profiler* P = (Profiler*)ctx->prof;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return;
  }
  P->recs.push_back({a, b, kind});
  *start = a;
  *stop = b;
}

void prof_end(dctk_ctx ctx, int kind) {
  if (!ctx || !ctx->prof || ctx->rec) return;
  Profiler* P = (Profiler*)ctx->prof;
  if (!P->open) return;
  hipEvent_t ev;
  if (hipEventCreate(&ev) != hipSuccess) return;
  (void)hipEventRecord(ev, ctx->stream);
  P->recs.push_back({P->open, ev, kind});
  P->open = nullptr;
}

// ---- staging without allocation ----------------------------------------------
// dctk_tube_apply_noalloc builds its p x p transform matrix in this file-scope
// array instead of a buffer allocated per call.  Every GPU the library runs on
// holds one copy (32 KB) until the process ends; all calls on that GPU share it.
// Host code never passes the array's name to a kernel (on the host it only
// stands in for the symbol): it uses the device address that
// hipGetSymbolAddress returns, taken once per device with that device current.
constexpr int kMaxScratchDevices = 256;
static __device__ __align__(256) double scratch[kMaxTube * kMaxTube];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices];

static hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (ptr == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// The matrix G (row-major p x p) of one of the four transforms, built on the
// device from the closed forms the host builder uses: C_n of eq. (dft1), and
// for the T+H transform M = W^{-1} C_n (I + Z), M^{-1} = (I + Z)^{-1} C_n^T W
// (Remark 2.1); the plain DCT's inverse is C_n^T.  One workgroup; C_n in LDS.
__global__ __launch_bounds__(256) void k_tube_matrix(int tube, int which, int p, int out_f64, void* out) {
  __shared__ double C[kMaxTube * kMaxTube];
  const int pp = p * p;
  for (int e = threadIdx.x; e < pp; e += blockDim.x) {
    const int i = e / p, j = e % p;
    const double sc = sqrt((i == 0 ? 1.0 : 2.0) / (double)p);
    C[e] = sc * cospi((double)(i * (2 * j + 1)) / (2.0 * (double)p));
  }
  __syncthreads();
  for (int e = threadIdx.x; e < pp; e += blockDim.x) {
    const int r = e / p, c = e % p;
    // G[r][c] is L[i][j] or L^{-1}[i][j] with (i, j) = (r, c) or (c, r)
    const bool inv = which == DCTK_MAT_LINV || which == DCTK_MAT_LINVT;
    const bool tr = which == DCTK_MAT_LINVT || which == DCTK_MAT_LT;
    const int i = tr ? c : r, j = tr ? r : c;
    double v;
    if (tube == DCTK_TUBE_DCT2) {
      v = inv ? C[j * p + i] : C[i * p + j];
    } else if (!inv) {
      v = (C[i * p + j] + (j > 0 ? C[i * p + j - 1] : 0.0)) / C[i * p];
    } else {
      double acc = 0.0, sg = 1.0;
      for (int l = i; l < p; ++l, sg = -sg) acc += sg * C[j * p + l];
      v = acc * C[j * p];
    }
    if (out_f64)
      static_cast<double*>(out)[e] = v;
    else
      static_cast<float*>(out)[e] = (float)v;
  }
}

}  // namespace dctk

extern "C" {

const char* dctk_status_string(int status) {
  switch (status) {
    case DCTK_OK: return "ok";
    case DCTK_BREAKDOWN: return "Krylov breakdown (result valid)";
    case DCTK_EINVAL: return "invalid argument";
    case DCTK_ESHAPE: return "inconsistent or non-positive dimensions";
    case DCTK_EDTYPE: return "unsupported element type";
    case DCTK_ENOMEM: return "out of memory";
    case DCTK_EHIP: return "HIP runtime error";
    case DCTK_ENONFINITE: return "non-finite value";
    case DCTK_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

int dctk_version(void) { return 100; }

int dctk_tube_matrix(int tube, int which, int64_t p, double* out) { return build_tube_matrix(tube, which, p, out); }

// ---- context -----------------------------------------------------------------
int dctk_create(dctk_ctx* out, int device, void* hip_stream) {
  if (out == nullptr) return DCTK_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DCTK_EINVAL;
  dctk_ctx c = new (std::nothrow) dctk_ctx_s();
  if (!c) return DCTK_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->last_hip_error = 0;
  c->prof = nullptr;
  c->rec = nullptr;
  c->scratch = nullptr;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = scratch_address(device, &c->scratch);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e == hipSuccess) e = hipMalloc((void**)&c->red_partials, sizeof(double) * kRedBlocks * kRedVals);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    int st = hip_fail(c, e);
    if (c->red_partials) (void)hipFree(c->red_partials);
    delete c;
    return st;
  }
  set_num_cus(c->num_cus);
  *out = c;
  return DCTK_OK;
}

int dctk_destroy(dctk_ctx ctx) {
  if (!ctx) return DCTK_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(ctx->red_partials);
  delete ctx;
  return DCTK_OK;
}

int dctk_set_stream(dctk_ctx ctx, void* hip_stream) {
  if (!ctx) return DCTK_EINVAL;
  ctx->stream = (hipStream_t)hip_stream;
  return DCTK_OK;
}

int dctk_synchronize(dctk_ctx ctx) {
  if (!ctx) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return DCTK_OK;
}

int dctk_last_hip_error(dctk_ctx ctx) { return ctx ? ctx->last_hip_error : 0; }

int dctk_profile_begin(dctk_ctx ctx) {
  if (!ctx) return DCTK_EINVAL;
  if (ctx->prof) return DCTK_ESTATE;
  Profiler* P = new (std::nothrow) Profiler();
  if (!P) return DCTK_ENOMEM;
  ctx->prof = P;
  return DCTK_OK;
}

int dctk_profile_end(dctk_ctx ctx, double* ms, int* count) {
  if (!ctx) return DCTK_EINVAL;
  if (!ctx->prof) return DCTK_ESTATE;
  Profiler* P = (Profiler*)ctx->prof;
  ctx->prof = nullptr;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  double acc[PROF_KINDS] = {};
  int cnt[PROF_KINDS] = {};
  for (auto& r : P->recs) {
    float t = 0.0f;
    if (e == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      acc[r.kind] += t;
      cnt[r.kind] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (P->open) (void)hipEventDestroy(P->open);
  delete P;
  if (e != hipSuccess) return hip_fail(ctx, e);
  for (int k = 0; k < PROF_KINDS; ++k) {
    if (ms) ms[k] = acc[k];
    if (count) count[k] = cnt[k];
  }
  return DCTK_OK;
}

// ---- tube transforms -----------------------------------------------------------
static int tube_fast_impl(dctk_ctx ctx, int tube, int which, int dtype, int64_t p, int64_t count, const void* in,
                          void* out) {
  if (!ctx || !in || !out) return DCTK_EINVAL;
  if (tube != DCTK_TUBE_TH && tube != DCTK_TUBE_DCT2) return DCTK_EINVAL;
  if (which < DCTK_MAT_L || which > DCTK_MAT_LT) return DCTK_EINVAL;
  if (dtype != DCTK_F64 && dtype != DCTK_F32) return DCTK_EDTYPE;
  if (count <= 0 || !tube_fast_shape_ok(dtype, p) || (count + (tube_fast_max(dtype) / p) - 1) / (tube_fast_max(dtype) / p) > 0x7fffffff)
    return DCTK_ESHAPE;
  const size_t bytes = (size_t)(p * count) * (dtype == DCTK_F64 ? 8 : 4);
  if (ranges_overlap(in, bytes, out, bytes)) return DCTK_EINVAL;
  if (ctx->rec) return DCTK_ESTATE;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  DCTK_HIP(ctx, launch_tube_fast(ctx, ctx->stream, tube, which, dtype, p, count, in, out));
  return DCTK_OK;
}

int dctk_tube_fast(dctk_ctx ctx, int tube, int which, int dtype, int64_t p, int64_t count, const void* in,
                   void* out) {
  return tube_fast_impl(ctx, tube, which, dtype, p, count, in, out);
}

static int tube_common(dctk_ctx ctx, int tube, int which, int dtype, int64_t p, int64_t count, const void* in,
                       void* out) {
  if (!ctx || !in || !out) return DCTK_EINVAL;
  if (tube != DCTK_TUBE_TH && tube != DCTK_TUBE_DCT2) return DCTK_EINVAL;
  if (dtype != DCTK_F64 && dtype != DCTK_F32) return DCTK_EDTYPE;
  // tubes beyond the dense transform's LDS matrix take the O(p log p) transform
  if (p > kMaxTube && tube_fast_shape_ok(dtype, p)) return tube_fast_impl(ctx, tube, which, dtype, p, count, in, out);
  if (p <= 0 || count <= 0 || p > kMaxTube) return DCTK_ESHAPE;
  const size_t bytes = (size_t)(p * count) * (dtype == DCTK_F64 ? 8 : 4);
  if (ranges_overlap(in, bytes, out, bytes)) return DCTK_EINVAL;
  std::vector<double> G((size_t)(p * p));
  build_tube_matrix(tube, which, p, G.data());
  std::vector<float> Gf((size_t)(p * p));
  for (size_t i = 0; i < G.size(); ++i) Gf[i] = (float)G[i];
  // the matrix travels in a small device buffer owned by this call
  void* dG = nullptr;
  const size_t gbytes = G.size() * (dtype == DCTK_F64 ? 8 : 4);
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  DCTK_HIP(ctx, hipMalloc(&dG, gbytes));
  hipError_t e = hipMemcpyAsync(dG, dtype == DCTK_F64 ? (const void*)G.data() : (const void*)Gf.data(), gbytes,
                                hipMemcpyHostToDevice, ctx->stream);
  Ctl plain{};
  plain.kind = CTL_PLAIN;
  plain.a = 1.0;
  plain.s = 1.0;
  if (e == hipSuccess)
    e = launch_tube(ctx, ctx->stream, dtype, dtype, p, count, in, out, (const double*)dG, (const float*)dG, nullptr,
                    nullptr, plain, false, true, nullptr);
  // the host copies of G must outlive the async copy; the device copy is freed after the work
  hipError_t e3 = hipStreamSynchronize(ctx->stream);
  hipError_t e2 = hipFree(dG);
  if (e != hipSuccess) return hip_fail(ctx, e);
  if (e2 != hipSuccess) return hip_fail(ctx, e2);
  if (e3 != hipSuccess) return hip_fail(ctx, e3);
  return DCTK_OK;
}

int dctk_tube_fwd(dctk_ctx ctx, int tube, int adjoint_pair, int dtype, int64_t p, int64_t count, const void* in,
                  void* out) {
  return tube_common(ctx, tube, adjoint_pair ? DCTK_MAT_LINVT : DCTK_MAT_L, dtype, p, count, in, out);
}
int dctk_tube_inv(dctk_ctx ctx, int tube, int adjoint_pair, int dtype, int64_t p, int64_t count, const void* in,
                  void* out) {
  return tube_common(ctx, tube, adjoint_pair ? DCTK_MAT_LT : DCTK_MAT_LINV, dtype, p, count, in, out);
}

int dctk_tube_apply_noalloc(dctk_ctx ctx, int tube, int which, int dtype, int64_t p, int64_t count, const void* in,
                            void* out) {
  if (!ctx || !in || !out) return DCTK_EINVAL;
  if (tube != DCTK_TUBE_TH && tube != DCTK_TUBE_DCT2) return DCTK_EINVAL;
  if (which < DCTK_MAT_L || which > DCTK_MAT_LT) return DCTK_EINVAL;
  if (dtype != DCTK_F64 && dtype != DCTK_F32) return DCTK_EDTYPE;
  // long tubes: the O(p log p) transform, which uses no staging memory
  if (p > kMaxTube && tube_fast_shape_ok(dtype, p)) return tube_fast_impl(ctx, tube, which, dtype, p, count, in, out);
  if (p <= 0 || count <= 0 || p > kMaxTube) return DCTK_ESHAPE;
  const size_t bytes = (size_t)(p * count) * (dtype == DCTK_F64 ? 8 : 4);
  if (ranges_overlap(in, bytes, out, bytes)) return DCTK_EINVAL;
  if (ctx->rec) return DCTK_ESTATE;
  if (!ctx->scratch) return DCTK_ESTATE;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_tube_matrix, dim3(1), dim3(256), 0, ctx->stream, tube, which, (int)p,
                     dtype == DCTK_F64 ? 1 : 0, ctx->scratch);
  DCTK_HIP(ctx, hipGetLastError());
  Ctl plain{};
  plain.kind = CTL_PLAIN;
  plain.a = 1.0;
  plain.s = 1.0;
  DCTK_HIP(ctx, launch_tube(ctx, ctx->stream, dtype, dtype, p, count, in, out, (const double*)ctx->scratch,
                            (const float*)ctx->scratch, nullptr, nullptr, plain, false, true, nullptr));
  return DCTK_OK;
}

// ---- operators -------------------------------------------------------------------
static void op_free(dctk_op op) {
  if (!op) return;
  void* ptrs[] = {op->Ah, op->AhT, op->Bh, op->Gd, op->Gf, op->xh, op->th, op->ch};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete op;
}

// The transform matrices of an operator on tensors with tube modes
// dims[0] = n3, ..., dims[nd-1] = nN (flattened tube index q = k3 + n3 (k4 +
// n4 (...)), mode N most significant): transforming every tube mode is one
// product with G = G_N (x) ... (x) G_3 on q, and the four matrices of that
// Kronecker product are the Kronecker products of each mode's four
// (inverses and transposes factor mode by mode).  One mode: the p x p matrices.
static void build_op_matrices(int tube, int nd, const int64_t* dims, int64_t P, std::vector<double>& Gd) {
  const int64_t pp = P * P;
  Gd.assign((size_t)(4 * pp), 0.0);
  std::vector<std::vector<double>> mode((size_t)nd);
  for (int w = 0; w < 4; ++w) {
    for (int m = 0; m < nd; ++m) {
      mode[m].assign((size_t)(dims[m] * dims[m]), 0.0);
      build_tube_matrix(tube, w, dims[m], mode[m].data());
    }
    double* G = Gd.data() + w * pp;
    for (int64_t r = 0; r < P; ++r)
      for (int64_t c = 0; c < P; ++c) {
        double v = 1.0;
        int64_t rr = r, cc = c;
        for (int m = 0; m < nd; ++m) {
          const int64_t n = dims[m];
          v *= mode[m][(size_t)((rr % n) * n + (cc % n))];
          rr /= n;
          cc /= n;
        }
        G[r * P + c] = v;
      }
  }
}

static int op_create_impl(dctk_ctx ctx, int tube, int gemm_dtype, int nd, const int64_t* dims, int64_t n1,
                          int64_t n2, const void* A, int64_t s, const void* B, dctk_op* out) {
  if (!ctx || !A || !out || !dims) return DCTK_EINVAL;
  *out = nullptr;
  if (tube != DCTK_TUBE_TH && tube != DCTK_TUBE_DCT2) return DCTK_EINVAL;
  if (gemm_dtype < DCTK_F64 || gemm_dtype > DCTK_F16) return DCTK_EDTYPE;
  if (nd < 1 || nd > kMaxTubeModes) return DCTK_ESHAPE;
  int64_t p = 1;
  // one tube mode longer than kMaxTube: a power of two up to kFastOpMaxP,
  // transformed by the O(p log p) kernels instead of a p x p matrix
  const bool fast = nd == 1 && dims[0] > kMaxTube;
  if (fast && (dims[0] > kFastOpMaxP || !tube_fast_shape_ok(DCTK_F64, dims[0]))) return DCTK_ESHAPE;
  for (int m = 0; m < nd && !fast; ++m) {
    if (dims[m] <= 0 || dims[m] > kMaxTube) return DCTK_ESHAPE;
    p *= dims[m];
    if (p > kMaxTube) return DCTK_ESHAPE;
  }
  if (fast) p = dims[0];
  if (n1 <= 0 || n2 <= 0 || s <= 0) return DCTK_ESHAPE;
  if (n1 > (1 << 30) || n2 > (1 << 30) || s > (1 << 30)) return DCTK_ESHAPE;
  dctk_op op = new (std::nothrow) dctk_op_s();
  if (!op) return DCTK_ENOMEM;
  op->ctx = ctx;
  op->tube = tube;
  op->gemm_dtype = gemm_dtype;
  op->vec_dtype = gemm_dtype == DCTK_F64 ? DCTK_F64 : DCTK_F32;
  op->p = p; op->n1 = n1; op->n2 = n2; op->s = s;
  op->two_sided = B != nullptr;
  op->fast = fast ? 1 : 0;
  for (int d = 0; d < 2; ++d) {
    op->tune[d][0] = -1;
    op->tune[d][1] = 0;
  }
  const size_t ge = elem_size(gemm_dtype);
  const size_t ae = gemm_dtype == DCTK_F64 ? 8 : 4;
  const int64_t nmax = n1 > n2 ? n1 : n2;
  const int64_t pp = p * p;
  std::vector<double> Gd;
  if (!fast) build_op_matrices(tube, nd, dims, p, Gd);
  std::vector<float> Gf(Gd.size());
  for (size_t i = 0; i < Gd.size(); ++i) Gf[i] = (float)Gd[i];
  double* tmp = nullptr;
  hipError_t e = hipSetDevice(ctx->device);
#define DCTK_TRY(call) do { if (e == hipSuccess) e = (call); } while (0)
  if (!fast) {
    DCTK_TRY(hipMalloc((void**)&op->Gd, sizeof(double) * 4 * pp));
    DCTK_TRY(hipMalloc((void**)&op->Gf, sizeof(float) * 4 * pp));
    DCTK_TRY(hipMemcpy(op->Gd, Gd.data(), sizeof(double) * 4 * pp, hipMemcpyHostToDevice));
    DCTK_TRY(hipMemcpy(op->Gf, Gf.data(), sizeof(float) * 4 * pp, hipMemcpyHostToDevice));
  }
  DCTK_TRY(hipMalloc(&op->Ah, ge * (size_t)(p * n1 * n2)));
  // 16-bit products read A~ with the contraction index contiguous in both
  // directions (16-byte rows straight into LDS): keep the transposed slices
  // for the adjoint; the FP32 slice GEMMs of the three-kernel path also read
  // them (the untransposed operand order of the forward product is the faster
  // one), while the fused FP32 products stage A~ itself
  if (gemm_dtype == DCTK_BF16 || gemm_dtype == DCTK_F16 || gemm_dtype == DCTK_F32)
    DCTK_TRY(hipMalloc(&op->AhT, ge * (size_t)(p * n1 * n2)));
  if (op->two_sided) DCTK_TRY(hipMalloc(&op->Bh, ge * (size_t)(p * s * s)));
  DCTK_TRY(hipMalloc(&op->xh, ge * (size_t)(p * nmax * s)));
  if (op->two_sided) DCTK_TRY(hipMalloc(&op->th, ge * (size_t)(p * nmax * s)));
  DCTK_TRY(hipMalloc(&op->ch, ae * (size_t)(p * nmax * s)));
  // A~ = A x_3 L and B~ = B x_3 L in FP64, then cast to the GEMM type
  const int64_t tmpn = (n1 * n2 > s * s || !op->two_sided) ? n1 * n2 : s * s;
  if (gemm_dtype != DCTK_F64) DCTK_TRY(hipMalloc((void**)&tmp, sizeof(double) * (size_t)(p * tmpn)));
  Ctl none{};
  none.kind = CTL_PLAIN;
  none.a = 1.0;
  none.s = 1.0;
#define DCTK_TUBE_F64(SRC, DST, CNT)                                                                   \
  (fast ? launch_tube_fast(ctx, ctx->stream, tube, DCTK_MAT_L, DCTK_F64, p, (CNT), (SRC), (DST))         \
        : launch_tube(ctx, ctx->stream, DCTK_F64, DCTK_F64, p, (CNT), (SRC), (DST), op->Gd, op->Gf, nullptr, \
                      nullptr, none, false, true, nullptr))
  if (gemm_dtype == DCTK_F64) {
    DCTK_TRY(DCTK_TUBE_F64(A, op->Ah, n1 * n2));
    if (op->two_sided) DCTK_TRY(DCTK_TUBE_F64(B, op->Bh, s * s));
  } else {
    DCTK_TRY(DCTK_TUBE_F64(A, tmp, n1 * n2));
    DCTK_TRY(launch_cast(ctx, p * n1 * n2, tmp, gemm_dtype, op->Ah));
    if (op->AhT) DCTK_TRY(launch_cast_t(ctx, p, n1, n2, tmp, gemm_dtype, op->AhT));
    if (op->two_sided) {
      DCTK_TRY(DCTK_TUBE_F64(B, tmp, s * s));
      DCTK_TRY(launch_cast(ctx, p * s * s, tmp, gemm_dtype, op->Bh));
    }
  }
#undef DCTK_TUBE_F64
  DCTK_TRY(hipStreamSynchronize(ctx->stream));
#undef DCTK_TRY
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) {
    int st = hip_fail(ctx, e);
    op_free(op);
    return st;
  }
  *out = op;
  return DCTK_OK;
}

int dctk_op_create(dctk_ctx ctx, int tube, int gemm_dtype, int64_t p, int64_t n1, int64_t n2, const void* A,
                   int64_t s, const void* B, dctk_op* out) {
  return op_create_impl(ctx, tube, gemm_dtype, 1, &p, n1, n2, A, s, B, out);
}

int dctk_op_create_nd(dctk_ctx ctx, int tube, int gemm_dtype, int ntube, const int64_t* tube_dims, int64_t n1,
                      int64_t n2, const void* A, int64_t s, const void* B, dctk_op* out) {
  return op_create_impl(ctx, tube, gemm_dtype, ntube, tube_dims, n1, n2, A, s, B, out);
}

int dctk_op_destroy(dctk_op op) {
  if (!op) return DCTK_EINVAL;
  (void)hipSetDevice(op->ctx->device);
  (void)hipStreamSynchronize(op->ctx->stream);
  op_free(op);
  return DCTK_OK;
}

int dctk_op_autotune(dctk_ctx ctx, dctk_op op, int reps, int* choice) {
  if (!ctx || !op || reps < 1 || reps > 1000) return DCTK_EINVAL;
  if (op->ctx->device != ctx->device || ctx->rec) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  const size_t ve = op->vec_dtype == DCTK_F64 ? 8 : 4;
  const int64_t nmax = op->n1 > op->n2 ? op->n1 : op->n2;
  const size_t bytes = (size_t)(op->p * nmax * op->s) * ve;
  void* X = nullptr;
  void* Y = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&X, bytes);
  if (e == hipSuccess) e = hipMalloc(&Y, bytes);
  if (e == hipSuccess) e = hipMemsetAsync(X, 0, bytes, ctx->stream);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  Ctl c{};
  c.kind = CTL_PLAIN;
  c.a = 1.0;
  c.s = 1.0;
  for (int adj = 0; adj < 2 && e == hipSuccess; ++adj) {
    int cand[7][2];
    int nc = 0;
    if (fused_eligible(op)) {
      cand[nc][0] = 1; cand[nc++][1] = 16;
      cand[nc][0] = 1; cand[nc++][1] = 32;
      if (op->p <= 4 && op->gemm_dtype != DCTK_F64) { cand[nc][0] = 1; cand[nc++][1] = 64; }
    }
    cand[nc][0] = 0; cand[nc++][1] = 32;
    cand[nc][0] = 0; cand[nc++][1] = 64;
    if (op->gemm_dtype != DCTK_F64) { cand[nc][0] = 0; cand[nc++][1] = 128; }
    if (op->gemm_dtype == DCTK_BF16 || op->gemm_dtype == DCTK_F16) { cand[nc][0] = 0; cand[nc++][1] = 256; }
    float best = 1e30f;
    int bi = -1;
    for (int i = 0; i < nc && e == hipSuccess; ++i) {
      op->tune[adj][0] = cand[i][0];
      op->tune[adj][1] = cand[i][1];
      hipError_t el = hipSuccess;
      for (int r = 0; r < 2 && el == hipSuccess; ++r) el = apply_op(op, ctx->stream, adj, X, Y, nullptr, nullptr, c, nullptr);
      if (el != hipSuccess) continue;  // a variant the shape cannot take: skip it
      e = hipEventRecord(e0, ctx->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = apply_op(op, ctx->stream, adj, X, Y, nullptr, nullptr, c, nullptr);
      if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms < best) {
        best = ms;
        bi = i;
      }
    }
    op->tune[adj][0] = bi >= 0 ? cand[bi][0] : -1;
    op->tune[adj][1] = bi >= 0 ? cand[bi][1] : 0;
    if (choice) {
      choice[2 * adj] = op->tune[adj][0];
      choice[2 * adj + 1] = op->tune[adj][1];
    }
  }
  (void)hipStreamSynchronize(ctx->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (X) (void)hipFree(X);
  if (Y) (void)hipFree(Y);
  if (e != hipSuccess) {
    for (int d = 0; d < 2; ++d) {
      op->tune[d][0] = -1;
      op->tune[d][1] = 0;
    }
    return hip_fail(ctx, e);
  }
  return DCTK_OK;
}

int dctk_op_set_path(dctk_op op, int adjoint, int path, int tile) {
  if (!op || (adjoint != 0 && adjoint != 1) || path < -1 || path > 1) return DCTK_EINVAL;
  if (tile != 0 && tile != 16 && tile != 32 && tile != 64 && tile != 128 && tile != 256) return DCTK_EINVAL;
  if (path == 1 && (!fused_eligible(op) || tile >= 128)) return DCTK_EINVAL;
  if (tile == 256 && op->gemm_dtype != DCTK_BF16 && op->gemm_dtype != DCTK_F16) return DCTK_EINVAL;
  if (path == 0 && tile == 16) return DCTK_EINVAL;
  op->tune[adjoint][0] = path;
  op->tune[adjoint][1] = tile;
  return DCTK_OK;
}

int dctk_op_info(dctk_op op, int64_t* dims) {
  if (!op || !dims) return DCTK_EINVAL;
  dims[0] = op->p; dims[1] = op->n1; dims[2] = op->n2; dims[3] = op->s;
  dims[4] = op->two_sided; dims[5] = op->gemm_dtype; dims[6] = op->vec_dtype; dims[7] = op->tube;
  return DCTK_OK;
}

static int cprod_common(dctk_ctx ctx, dctk_op op, int adjoint, double a, const void* in, double b, void* out) {
  if (!ctx || !op || !in || !out) return DCTK_EINVAL;
  if (op->ctx != ctx && op->ctx->device != ctx->device) return DCTK_EINVAL;
  if (!std::isfinite(a) || !std::isfinite(b)) return DCTK_EINVAL;
  const size_t ve = op->vec_dtype == DCTK_F64 ? 8 : 4;
  const size_t nin = (size_t)(op->p * (adjoint ? op->n1 : op->n2) * op->s) * ve;
  const size_t nout = (size_t)(op->p * (adjoint ? op->n2 : op->n1) * op->s) * ve;
  if (ranges_overlap(in, nin, out, nout)) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  Ctl c{};
  c.kind = CTL_PLAIN;
  c.a = a;
  c.b = b;
  c.s = 1.0;
  DCTK_HIP(ctx, apply_op(op, ctx->stream, adjoint, in, out, b != 0.0 ? out : nullptr, nullptr, c, nullptr));
  return DCTK_OK;
}

int dctk_cprod(dctk_ctx ctx, dctk_op op, double a, const void* X, double b, void* Y) {
  return cprod_common(ctx, op, 0, a, X, b, Y);
}
int dctk_cprod_T(dctk_ctx ctx, dctk_op op, double a, const void* Y, double b, void* X) {
  return cprod_common(ctx, op, 1, a, Y, b, X);
}

// ---- Krylov workspaces -----------------------------------------------------------
int dctk_krylov_create(dctk_ctx ctx, dctk_op op, int kind, int k_max, int ortho, dctk_krylov* out) {
  if (!ctx || !op || !out) return DCTK_EINVAL;
  *out = nullptr;
  if (kind != DCTK_KRYLOV_GKB && kind != DCTK_KRYLOV_ARNOLDI) return DCTK_EINVAL;
  if (k_max < 1 || k_max > kMaxK) return DCTK_EINVAL;
  if (ortho != DCTK_ORTHO_MGS && ortho != DCTK_ORTHO_CGS2) return DCTK_EINVAL;
  if (kind == DCTK_KRYLOV_ARNOLDI && (op->n1 != op->n2)) return DCTK_ESHAPE;
  dctk_krylov ws = new (std::nothrow) dctk_krylov_s();
  if (!ws) return DCTK_ENOMEM;
  ws->op = op;
  ws->kind = kind;
  ws->k_max = k_max;
  ws->ortho = ortho;
  const int64_t nmax = op->n1 > op->n2 ? op->n1 : op->n2;
  ws->nvec = round_up(op->p * nmax * op->s, 64);  // slot stride in elements (256-byte aligned slots)
  const size_t ve = op->vec_dtype == DCTK_F64 ? 8 : 4;
  ws->vbytes = (size_t)ws->nvec * ve;
  hipError_t e = hipSetDevice(ctx->device);
  const size_t nslots = (size_t)(k_max + 1);
  if (e == hipSuccess) e = hipMalloc(&ws->U, ws->vbytes * nslots);
  if (e == hipSuccess && kind == DCTK_KRYLOV_GKB) e = hipMalloc(&ws->V, ws->vbytes * nslots);
  if (e == hipSuccess) e = hipMalloc(&ws->X, ws->vbytes);
  if (e == hipSuccess) e = hipMalloc(&ws->W, ws->vbytes);
  if (e == hipSuccess) e = hipMalloc(&ws->T, 2 * ws->vbytes);
  if (e == hipSuccess) e = hipMalloc(&ws->R, ws->vbytes);
  if (e == hipSuccess) e = hipMalloc((void**)&ws->partA, sizeof(double) * kNormParts);
  if (e == hipSuccess) e = hipMalloc((void**)&ws->partB, sizeof(double) * kNormParts);
  if (e == hipSuccess) e = hipMalloc((void**)&ws->partM, sizeof(double) * kRedBlocks * kRedVals);
  if (e == hipSuccess) e = hipMalloc((void**)&ws->st, sizeof(KState));
  if (e == hipSuccess) e = hipMemset(ws->st, 0, sizeof(KState));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    int st = hip_fail(ctx, e);
    void* ptrs[] = {ws->U, ws->V, ws->X, ws->W, ws->T, ws->R, ws->partA, ws->partB, ws->partM, ws->st};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
    delete ws;
    return st;
  }
  *out = ws;
  return DCTK_OK;
}

int dctk_krylov_destroy(dctk_krylov ws) {
  if (!ws) return DCTK_EINVAL;
  (void)hipSetDevice(ws->op->ctx->device);
  (void)hipStreamSynchronize(ws->op->ctx->stream);
  void* ptrs[] = {ws->U, ws->V, ws->X, ws->W, ws->T, ws->R, ws->partA, ws->partB, ws->partM, ws->st};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete ws;
  return DCTK_OK;
}

}  // extern "C"

namespace dctk {

static inline char* slot(void* base, const dctk_krylov ws, int i) { return (char*)base + (size_t)i * ws->vbytes; }

static Ctl make_ctl(int kind, int j, KState* st, const double* part_in, int npart_in, double* part_out) {
  Ctl c{};
  c.kind = kind;
  c.j = j;
  c.st = st;
  c.part_in = part_in;
  c.npart_in = npart_in;
  c.part_out = part_out;
  c.a = 1.0;
  c.s = 1.0;
  return c;
}

// Slots [lo, hi) of the basis bit mask.
static unsigned long long slot_bits(int lo, int hi) {
  unsigned long long m = 0;
  for (int i = lo; i < hi && i < 64; ++i) m |= 1ull << i;
  return m;
}

// Classical Gram-Schmidt applied twice: w -= B (B^T w), with B the first nb slots of `basis`.
// When hcol is given the coefficients are also added to it (Arnoldi column).
static hipError_t cgs2(dctk_ctx ctx, dctk_krylov ws, void* basis, int nb, void* w, int64_t n, Gate g,
                       double* hcol) {
  hipError_t e;
  KState* st = ws->st;
  for (int pass = 0; pass < 2; ++pass) {
    int nbk = 0;
    if ((e = launch_multidot(ctx, ws->op->vec_dtype, n, basis, ws->nvec, nb, w, ws->partM, &nbk, g)) != hipSuccess)
      return e;
    if ((e = launch_coef_finalize(ctx, ws->partM, nbk, nb, st->coef, hcol, kMaxK, g)) != hipSuccess) return e;
    if ((e = launch_subtract(ctx, ws->op->vec_dtype, n, w, basis, ws->nvec, nb, st->coef, g)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// Algorithm 4 step 2 and Algorithm 6 step 2, writing the LSQR iterate into X:
//   partials of ||C||^2;  [beta_1, U_1 = C/beta_1, V~ = M*(U_1), partials of ||V~||^2];
//   [alpha_1, V_1 = V~/alpha_1, W_1 = V_1, X_0 = 0]
static hipError_t gkb_init_impl(dctk_ctx ctx, dctk_krylov ws, const void* C, void* X, double tol) {
  dctk_op op = ws->op;
  KState* st = ws->st;
  const int vdt = op->vec_dtype;
  const int64_t nU = op->p * op->n1 * op->s, nV = op->p * op->n2 * op->s;
  hipError_t e;
  ws->vmask = 0;
  rec_phase(ctx);
  if ((e = launch_state_reset(ctx, st, 1, tol)) != hipSuccess) return e;
  int npA = 0, npB = 0;
  rec_phase(ctx);
  if ((e = launch_sumsq(ctx, vdt, nU, C, nullptr, ws->partA, &npA, Gate{nullptr, 0, 0})) != hipSuccess) return e;
  const Ctl c = make_ctl(CTL_GKB_INIT, 0, st, ws->partA, npA, ws->partB);
  rec_phase(ctx);
  if ((e = apply_op(op, ctx->stream, 1, C, slot(ws->V, ws, 0), nullptr, slot(ws->U, ws, 0), c, &npB)) != hipSuccess)
    return e;
  rec_phase(ctx);
  return launch_gkb_start(ctx, vdt, nV, X, X ? ws->W : nullptr, slot(ws->V, ws, 0), ws->partB, npB, st);
}

// Algorithm 4 step 3 (a)-(f) with the LSQR update of Algorithm 6 (c)-(g), step j:
//   K1: T = M(V_j) - alpha_j U_j, partials of ||T||^2             (one product)
//   K2: beta_{j+1}; U_{j+1} = T/beta_{j+1}; V~ = M*(U_{j+1}) - beta_{j+1} V_j,
//       partials of ||V~||^2                                         (one product)
//   K3: alpha_{j+1}; rotation; V_{j+1} = V~/alpha_{j+1}; X and W updates
// With reorthogonalisation, CGS2 passes run on T (before K2) and on V~ (before K3).
static hipError_t gkb_step_impl(dctk_ctx ctx, dctk_krylov ws, int j, void* X) {
  dctk_op op = ws->op;
  KState* st = ws->st;
  const int vdt = op->vec_dtype;
  const int64_t nU = op->p * op->n1 * op->s, nV = op->p * op->n2 * op->s;
  void* Uj = slot(ws->U, ws, j - 1);
  void* Un = slot(ws->U, ws, j);
  void* Vj = slot(ws->V, ws, j - 1);
  void* Vn = slot(ws->V, ws, j);
  void* T = ws->T;
  hipError_t e;
  int npA = 0, npB = 0;
  ws->vmask &= ~slot_bits(j, j + 1);  // this step writes U_{j+1} and V_{j+1} normalised
  const bool ru = ws->reorth == DCTK_REORTH_FULL;
  const bool rv = ws->reorth != DCTK_REORTH_NONE;
  const Ctl c1 = make_ctl(CTL_GKB_FWD, j, st, nullptr, 0, ru ? nullptr : ws->partA);
  rec_phase(ctx);
  if ((e = apply_op(op, ctx->stream, 0, Vj, T, Uj, nullptr, c1, &npA)) != hipSuccess) return e;
  if (ru) {
    const Gate g{st, j, 0};
    if ((e = cgs2(ctx, ws, ws->U, j, T, nU, g, nullptr)) != hipSuccess) return e;
    if ((e = launch_sumsq(ctx, vdt, nU, T, nullptr, ws->partA, &npA, g)) != hipSuccess) return e;
  }
  const Ctl c2 = make_ctl(CTL_GKB_ADJ, j, st, ws->partA, npA, rv ? nullptr : ws->partB);
  rec_phase(ctx);
  if ((e = apply_op(op, ctx->stream, 1, T, Vn, Vj, Un, c2, &npB)) != hipSuccess) return e;
  if (rv) {
    const Gate g{st, j, 1};
    if ((e = cgs2(ctx, ws, ws->V, j, Vn, nV, g, nullptr)) != hipSuccess) return e;
    if ((e = launch_sumsq(ctx, vdt, nV, Vn, nullptr, ws->partB, &npB, g)) != hipSuccess) return e;
  }
  rec_phase(ctx);
  return launch_gkb_update(ctx, vdt, nV, X, X ? ws->W : nullptr, nullptr, Vn, ws->partB, npB, st, j);
}

// Whether a solve without the LSQR iterate can fold each LSQR update into the
// next forward product (its first kernel, fused or the forward transform):
// no reorthogonalisation.
static bool merged_steps(dctk_krylov ws) { return ws->reorth == DCTK_REORTH_NONE; }

// Step j of a Tikhonov solve (no LSQR iterate) with the update folded in.  The
// new basis vectors stay in their slots unnormalised, as the products leave
// them (U slot j: beta_{j+1} U_{j+1}, V slot j: alpha_{j+1} V_{j+1}): the
// product that reads one scales it as it is staged, the epilogue that uses one
// as src divides its coefficient by the normaliser, and the combine divides
// y_j -- so no normalised copy is written.  The first step of a run (pending =
// false) reads the slots the initialisation or the previous run's flush
// normalised.
//   K1: unless pending = false, alpha_j and the rotation of step j-1 from the
//       partials of alpha_j V_j; T = M(V_j) - alpha_j U_j into U slot j, with
//       its partials
//   K2: beta_{j+1}; V~ = M*(U_{j+1}) - beta_{j+1} V_j into V slot j, with its
//       partials.
// The update of the last step is flushed by gkb_flush_update.
static hipError_t gkb_step_merged(dctk_ctx ctx, dctk_krylov ws, int j, bool pending) {
  dctk_op op = ws->op;
  KState* st = ws->st;
  void* Uj = slot(ws->U, ws, j - 1);
  void* Un = slot(ws->U, ws, j);
  void* Vj = slot(ws->V, ws, j - 1);
  void* Vn = slot(ws->V, ws, j);
  hipError_t e;
  int npA = 0, npB = 0;
  Ctl c1 = pending ? make_ctl(CTL_GKB_FWDU, j, st, ws->partB, ws->last_npart, ws->partA)
                   : make_ctl(CTL_GKB_FWD, j, st, nullptr, 0, ws->partA);
  c1.src_div = pending ? 1 : 0;
  Ctl c2 = make_ctl(CTL_GKB_ADJ, j, st, ws->partA, 0, ws->partB);
  c2.src_div = pending ? 1 : 0;
  if (pair_eligible(op)) {
    // Three-kernel products with paired transforms: each product's inverse
    // transform also forms the next product's transformed input (from the
    // unnormalised vector it has just written), so only the first step of a
    // run has a forward transform of its own.  A pending update is evaluated
    // by the first paired kernel of the step, after the forward GEMM (the
    // GEMM's input is alpha_j V_j transformed; 1/alpha_j joins the epilogue).
    // (one schedule point per product, as on the other paths, so batches of
    // mixed paths stay aligned step by step)
    rec_phase(ctx);
    if ((e = pending ? pair_gemm(op, ctx->stream, 0, c1) : pair_first(op, ctx->stream, 0, Vj, c1)) != hipSuccess)
      return e;
    if ((e = pair_transforms(op, ctx->stream, 0, Uj, Un, c1, &npA)) != hipSuccess) return e;
    c2.npart_in = npA;
    rec_phase(ctx);
    if ((e = pair_gemm(op, ctx->stream, 1, c2)) != hipSuccess) return e;
    if ((e = pair_transforms(op, ctx->stream, 1, Vj, Vn, c2, &npB)) != hipSuccess) return e;
    ws->last_npart = npB;
    return hipSuccess;
  }
  rec_phase(ctx);
  if ((e = apply_op(op, ctx->stream, 0, Vj, Un, Uj, nullptr, c1, &npA)) != hipSuccess) return e;
  c2.npart_in = npA;
  rec_phase(ctx);
  if ((e = apply_op(op, ctx->stream, 1, Un, Vn, Vj, nullptr, c2, &npB)) != hipSuccess) return e;
  ws->last_npart = npB;
  return hipSuccess;
}

// The LSQR update of step j left pending by gkb_step_merged: alpha_{j+1}, the
// rotation, V_{j+1} and U_{j+1} normalised in their slots.
static hipError_t gkb_flush_update(dctk_ctx ctx, dctk_krylov ws, int j) {
  dctk_op op = ws->op;
  rec_phase(ctx);
  return launch_gkb_update(ctx, op->vec_dtype, op->p * op->n2 * op->s, nullptr, nullptr, nullptr,
                           slot(ws->V, ws, j), ws->partB, ws->last_npart, ws->st, j, slot(ws->U, ws, j));
}

// Steps from..to of a Tikhonov solve, with the update of step to flushed.
static hipError_t gkb_steps_tik(dctk_ctx ctx, dctk_krylov ws, int from, int to) {
  hipError_t e;
  if (merged_steps(ws)) {
    for (int j = from; j <= to; ++j)
      if ((e = gkb_step_merged(ctx, ws, j, j > from)) != hipSuccess) return e;
    if (to < from) return hipSuccess;
    // slots from..to-1 keep their vectors unnormalised; the flush normalises slot to
    ws->vmask = (ws->vmask | slot_bits(from, to)) & ~slot_bits(to, to + 1);
    return gkb_flush_update(ctx, ws, to);
  }
  for (int j = from; j <= to; ++j)
    if ((e = gkb_step_impl(ctx, ws, j, nullptr)) != hipSuccess) return e;
  return hipSuccess;
}

// Everything dctk_lsqr_tik_solve enqueues (Algorithms 4-6, then Algorithm 5's
// projected solve and X = V_k (*) y when lambda != 0).  Also used, with the
// context recording, to plan batches.
hipError_t lsqr_enqueue(dctk_ctx ctx, dctk_krylov ws, const void* C, void* X, const dctk_solve_opts* opts) {
  dctk_op op = ws->op;
  hipError_t e;
  ws->reorth = opts->reorth;
  const bool tik = opts->lambda != 0.0;
  // the LSQR iterate (Algorithm 6) is formed only when it is the answer
  if ((e = gkb_init_impl(ctx, ws, C, tik ? nullptr : X, opts->tol)) != hipSuccess) return e;
  if (tik) {
    if ((e = gkb_steps_tik(ctx, ws, 1, opts->k_max)) != hipSuccess) return e;
  } else {
    for (int j = 1; j <= opts->k_max; ++j)
      if ((e = gkb_step_impl(ctx, ws, j, X)) != hipSuccess) return e;
  }
  ws->host_steps = opts->k_max;
  ws->initialised = 1;
  if (tik) {
    // Algorithm 5: lambda (GCV, the discrepancy principle or fixed), y, X = V_k (*) y
    rec_phase(ctx);
    e = (opts->gcv_mode == 2 && opts->lambda < 0.0)
            ? launch_projected_disc(ctx, ws->st, opts->target)
            : launch_projected(ctx, ws->st, 1, opts->gcv_mode, opts->lambda < 0.0 ? -1.0 : opts->lambda);
    if (e != hipSuccess) return e;
    rec_phase(ctx);
    if ((e = launch_combine(ctx, op->vec_dtype, op->p * op->n2 * op->s, X, nullptr, ws->V, ws->nvec, opts->k_max,
                            &ws->st->steps, ws->st->y, Gate{nullptr, 0, 0}, ws->vmask, ws->st->alpha)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// Algorithm 2 step 2 on R with the partials of ||R||^2 already in `part`: V_1 = R / ||R||.
static hipError_t arnoldi_start_impl(dctk_ctx ctx, dctk_krylov ws, const void* R, const double* part, int npart) {
  dctk_op op = ws->op;
  const int64_t n = op->p * op->n1 * op->s;
  return launch_arn_start(ctx, op->vec_dtype, n, slot(ws->U, ws, 0), R, part, npart, ws->st);
}

// Algorithm 2 step 3 (a)-(e), step j: W = M(V_j) (with V_j = W_{j-1}/h_{j,j-1}
// formed and recorded by the same kernel), the Gram-Schmidt passes, and the
// partials of ||W||^2 in partA (h_{j+1,j} is recorded by the next product or
// by launch_arn_finish).
static hipError_t arnoldi_step_impl(dctk_ctx ctx, dctk_krylov ws, int j) {
  dctk_op op = ws->op;
  KState* st = ws->st;
  const int vdt = op->vec_dtype;
  const int64_t n = op->p * op->n1 * op->s;
  void* Win = (j == 1) ? slot(ws->U, ws, 0) : slot(ws->T, ws, (j - 1) & 1);
  void* xnorm = (j == 1) ? nullptr : slot(ws->U, ws, j - 1);
  void* W = slot(ws->T, ws, j & 1);
  hipError_t e;
  const Ctl c = make_ctl(CTL_ARN_FWD, j, st, ws->partA, ws->last_npart, nullptr);
  if ((e = apply_op(op, ctx->stream, 0, Win, W, nullptr, xnorm, c, nullptr)) != hipSuccess) return e;
  double* Hcol = &st->H[j - 1];  // H[i][j-1] at Hcol[i * kMaxK]
  int np = 0;
  if (ws->ortho == DCTK_ORTHO_MGS) {
    // h_{i,j} = <V_i, W>; W -= h_{i,j} V_i, as: record and subtract the previous term, then dot with V_i
    const double* pin = nullptr;
    int npin = 0;
    for (int i = 0; i <= j; ++i) {
      double* pout = (i == j) ? ws->partA : ((i & 1) ? ws->partM : ws->partB);
      const void* vprev = i > 0 ? slot(ws->U, ws, i - 1) : nullptr;
      const void* vi = i < j ? slot(ws->U, ws, i) : nullptr;
      double* hdst = i > 0 ? &Hcol[(i - 1) * kMaxK] : nullptr;
      if ((e = launch_mgs(ctx, vdt, n, W, vprev, vi, pin, npin, hdst, pout, &np, st, j)) != hipSuccess) return e;
      pin = pout;
      npin = np;
    }
  } else {
    const Gate g{st, j - 1, 1};
    if ((e = cgs2(ctx, ws, ws->U, j, W, n, g, Hcol)) != hipSuccess) return e;
    if ((e = launch_sumsq(ctx, vdt, n, W, nullptr, ws->partA, &np, g)) != hipSuccess) return e;
  }
  ws->last_npart = np;
  return hipSuccess;
}

struct HostState {
  int steps, stop_step, stop_kind, status, converged, cycles, halt, total_steps;
  double tol, beta0, lambda, gcv, resnorm;
};

static int read_state(dctk_ctx ctx, dctk_krylov ws, HostState* hs) {
  static_assert(sizeof(HostState) <= sizeof(KState), "state prefix");
  DCTK_HIP(ctx, hipMemcpyAsync(hs, ws->st, sizeof(HostState), hipMemcpyDeviceToHost, ctx->stream));
  DCTK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return DCTK_OK;
}

// The state up to and including the LSQR scalars (phibar), in one copy and one
// synchronisation.
static int read_state_lsqr(dctk_ctx ctx, dctk_krylov ws, KState* hk) {
  DCTK_HIP(ctx, hipMemcpyAsync(hk, ws->st, offsetof(KState, H), hipMemcpyDeviceToHost, ctx->stream));
  DCTK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return DCTK_OK;
}

hipError_t learned_enqueue(dctk_ctx ctx, dctk_krylov ws, dctk_mlp m, const void* C, void* X,
                           const dctk_solve_opts* opts, double gate) {
  const int kf = 8;
  dctk_op op = ws->op;
  hipError_t e;
  ws->reorth = opts->reorth;
  if ((e = gkb_init_impl(ctx, ws, C, nullptr, opts->tol)) != hipSuccess) return e;
  if ((e = gkb_steps_tik(ctx, ws, 1, kf)) != hipSuccess) return e;
  rec_phase(ctx);
  if ((e = launch_mlp_stop(ctx, m, ws->st, kf, opts->k_max)) != hipSuccess) return e;
  // steps beyond the predicted stop exit at once (their gate reads st->k_limit)
  if ((e = gkb_steps_tik(ctx, ws, kf + 1, opts->k_max)) != hipSuccess) return e;
  ws->host_steps = opts->k_max;
  ws->initialised = 1;
  rec_phase(ctx);
  if ((e = launch_projected(ctx, ws->st, 1, opts->gcv_mode, -1.0, 0, -1.0, gate, 1)) != hipSuccess) return e;
  rec_phase(ctx);
  return launch_combine(ctx, op->vec_dtype, op->p * op->n2 * op->s, X, nullptr, ws->V, ws->nvec, opts->k_max,
                        &ws->st->steps, ws->st->y, Gate{nullptr, 0, 0}, ws->vmask, ws->st->alpha);
}

// alpha_1.. and beta_1.. of the recorded process into the caller's host arrays
// (info->alpha / beta, at most info->cap entries, steps + 1 at most)
static void copy_gk_scalars(const KState& hk, int steps, dctk_solve_info* info) {
  if (!info || info->cap <= 0) return;
  const int n = std::min(info->cap, std::max(0, steps) + 1);
  for (int j = 0; j < n; ++j) {
    if (info->alpha) info->alpha[j] = hk.alpha[j];
    if (info->beta) info->beta[j] = hk.beta[j];
  }
}

int lsqr_info(dctk_ctx ctx, dctk_krylov ws, const dctk_solve_opts* opts, dctk_solve_info* info) {
  static thread_local KState hk;
  int r;
  if ((r = read_state_lsqr(ctx, ws, &hk))) return r;
  const bool tik = opts->lambda != 0.0;
  const int steps = hk.steps < 0 ? 0 : (hk.steps > kMaxK ? kMaxK : hk.steps);
  if (info) {
    info->iters = hk.steps;
    info->status = hk.status;
    info->converged = hk.converged;
    info->cycles = 0;
    info->lambda = tik ? hk.lambda : 0.0;
    info->resnorm = std::fabs(hk.phibar[steps]);
    info->gcv = (tik && opts->lambda < 0.0) ? hk.gcv : NAN;
    copy_gk_scalars(hk, steps, info);
  }
  return hk.status;
}

}  // namespace dctk

extern "C" {

static int ws_check(dctk_ctx ctx, dctk_krylov ws, int kind) {
  if (!ctx || !ws) return DCTK_EINVAL;
  if (ws->kind != kind) return DCTK_EINVAL;
  if (ws->op->ctx->device != ctx->device) return DCTK_EINVAL;
  return DCTK_OK;
}

int dctk_gkb_init(dctk_ctx ctx, dctk_krylov ws, const void* C, int reorth, double tol) {
  int r = ws_check(ctx, ws, DCTK_KRYLOV_GKB);
  if (r) return r;
  if (!C) return DCTK_EINVAL;
  if (reorth < DCTK_REORTH_NONE || reorth > DCTK_REORTH_FULL) return DCTK_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return DCTK_EINVAL;
  ws->reorth = reorth;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  DCTK_HIP(ctx, gkb_init_impl(ctx, ws, C, ws->X, tol));
  ws->host_steps = 0;
  ws->initialised = 1;
  return DCTK_OK;
}

int dctk_gkb_step(dctk_ctx ctx, dctk_krylov ws) {
  int r = ws_check(ctx, ws, DCTK_KRYLOV_GKB);
  if (r) return r;
  if (!ws->initialised || ws->host_steps >= ws->k_max) return DCTK_ESTATE;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  const int j = ws->host_steps + 1;
  DCTK_HIP(ctx, gkb_step_impl(ctx, ws, j, ws->X));
  ws->host_steps = j;
  return DCTK_OK;
}

int dctk_arnoldi_init(dctk_ctx ctx, dctk_krylov ws, const void* V) {
  int r = ws_check(ctx, ws, DCTK_KRYLOV_ARNOLDI);
  if (r) return r;
  if (!V) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  DCTK_HIP(ctx, launch_state_reset(ctx, ws->st, 1, 0.0));
  int np = 0;
  DCTK_HIP(ctx, launch_sumsq(ctx, ws->op->vec_dtype, ws->op->p * ws->op->n1 * ws->op->s, V, nullptr, ws->partB, &np,
                             Gate{nullptr, 0, 0}));
  DCTK_HIP(ctx, arnoldi_start_impl(ctx, ws, V, ws->partB, np));
  ws->host_steps = 0;
  ws->initialised = 1;
  return DCTK_OK;
}

int dctk_arnoldi_step(dctk_ctx ctx, dctk_krylov ws) {
  int r = ws_check(ctx, ws, DCTK_KRYLOV_ARNOLDI);
  if (r) return r;
  if (!ws->initialised || ws->host_steps >= ws->k_max) return DCTK_ESTATE;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  const int j = ws->host_steps + 1;
  DCTK_HIP(ctx, arnoldi_step_impl(ctx, ws, j));
  // record h_{j+1,j} now (the next step's product records the same value again)
  DCTK_HIP(ctx, launch_arn_finish(ctx, ws->partA, ws->last_npart, ws->st, j + 1));
  ws->host_steps = j;
  return DCTK_OK;
}

int dctk_krylov_read(dctk_ctx ctx, dctk_krylov ws, double* alpha, double* beta_or_H, int* info4) {
  if (!ctx || !ws) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  KState* h = new (std::nothrow) KState();
  if (!h) return DCTK_ENOMEM;
  hipError_t e = hipMemcpyAsync(h, ws->st, sizeof(KState), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(ctx, e);
  }
  const int K = ws->k_max;
  if (ws->kind == DCTK_KRYLOV_GKB) {
    if (alpha) for (int i = 0; i <= K; ++i) alpha[i] = h->alpha[i];
    if (beta_or_H) for (int i = 0; i <= K; ++i) beta_or_H[i] = h->beta[i];
  } else {
    if (beta_or_H)
      for (int i = 0; i <= K; ++i)
        for (int j = 0; j < K; ++j) beta_or_H[i * K + j] = h->H[i * kMaxK + j];
    if (alpha) alpha[0] = h->beta0;
  }
  if (info4) {
    info4[0] = h->steps;
    info4[1] = h->status;
    info4[2] = h->converged;
    info4[3] = K;
    info4[4] = (int)h->sweeps;
    info4[5] = h->cycles;
  }
  delete h;
  return DCTK_OK;
}

int dctk_krylov_basis(dctk_krylov ws, int which, int j, void** ptr) {
  if (!ws || !ptr) return DCTK_EINVAL;
  if (which == 2) { *ptr = ws->X; return DCTK_OK; }
  if (which == 3) { *ptr = ws->W; return DCTK_OK; }
  if (j < 0 || j > ws->k_max) return DCTK_EINVAL;
  if (which == 0) { *ptr = slot(ws->U, ws, j); return DCTK_OK; }
  if (which == 1 && ws->V) { *ptr = slot(ws->V, ws, j); return DCTK_OK; }
  return DCTK_EINVAL;
}

int dctk_krylov_copy(dctk_ctx ctx, dctk_krylov ws, int which, int j, void* dst) {
  if (!ctx || !ws || !dst) return DCTK_EINVAL;
  void* src = nullptr;
  int r = dctk_krylov_basis(ws, which, j, &src);
  if (r) return r;
  dctk_op op = ws->op;
  const bool u_side = (ws->kind == DCTK_KRYLOV_GKB && which == 0);
  const int64_t n = op->p * (u_side ? op->n1 : op->n2) * op->s;
  const size_t bytes = (size_t)n * (op->vec_dtype == DCTK_F64 ? 8 : 4);
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  DCTK_HIP(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  return DCTK_OK;
}

}  // extern "C"

int dctk::check_solve_opts(const dctk_solve_opts* o, const dctk_krylov ws) {
  if (!o) return DCTK_EINVAL;
  if (o->k_max < 1 || o->k_max > ws->k_max) return DCTK_EINVAL;
  if (o->reorth < DCTK_REORTH_NONE || o->reorth > DCTK_REORTH_FULL) return DCTK_EINVAL;
  if (o->gcv_mode < 0 || o->gcv_mode > 2) return DCTK_EINVAL;
  if (o->gcv_mode == 2 && o->lambda < 0.0 && !(o->target > 0.0 && std::isfinite(o->target))) return DCTK_EINVAL;
  if (std::isnan(o->lambda) || std::isinf(o->lambda)) return DCTK_EINVAL;
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return DCTK_EINVAL;
  return DCTK_OK;
}

extern "C" {

int dctk_lsqr_tik_solve(dctk_ctx ctx, dctk_krylov ws, const void* C, void* X, const dctk_solve_opts* opts,
                        dctk_solve_info* info) {
  int r = ws_check(ctx, ws, DCTK_KRYLOV_GKB);
  if (r) return r;
  if (!C || !X) return DCTK_EINVAL;
  if ((r = check_solve_opts(opts, ws))) return r;
  dctk_op op = ws->op;
  const size_t ve = op->vec_dtype == DCTK_F64 ? 8 : 4;
  if (ranges_overlap(C, (size_t)(op->p * op->n1 * op->s) * ve, X, (size_t)(op->p * op->n2 * op->s) * ve))
    return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  DCTK_HIP(ctx, lsqr_enqueue(ctx, ws, C, X, opts));
  if (info == nullptr) return DCTK_OK;  // enqueued only: no read-back, no synchronisation
  return lsqr_info(ctx, ws, opts, info);
}

int dctk_lsqr_lcurve_solve(dctk_ctx ctx, dctk_krylov ws, const void* C, void* X, const dctk_solve_opts* opts,
                           dctk_solve_info* info, int* k_opt) {
  int r = ws_check(ctx, ws, DCTK_KRYLOV_GKB);
  if (r) return r;
  if (!C || !X) return DCTK_EINVAL;
  if ((r = check_solve_opts(opts, ws))) return r;
  dctk_op op = ws->op;
  const size_t ve = op->vec_dtype == DCTK_F64 ? 8 : 4;
  if (ranges_overlap(C, (size_t)(op->p * op->n1 * op->s) * ve, X, (size_t)(op->p * op->n2 * op->s) * ve))
    return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  ws->reorth = opts->reorth;
  DCTK_HIP(ctx, gkb_init_impl(ctx, ws, C, nullptr, opts->tol));
  DCTK_HIP(ctx, gkb_steps_tik(ctx, ws, 1, opts->k_max));
  ws->host_steps = opts->k_max;
  ws->initialised = 1;
  DCTK_HIP(ctx, launch_lcurve(ctx, ws->st));
  DCTK_HIP(ctx, launch_combine(ctx, op->vec_dtype, op->p * op->n2 * op->s, X, nullptr, ws->V, ws->nvec, opts->k_max,
                               &ws->st->steps, ws->st->y, Gate{nullptr, 0, 0}, ws->vmask, ws->st->alpha));
  static thread_local KState hk;
  if ((r = read_state_lsqr(ctx, ws, &hk))) return r;
  if (info) {
    info->iters = hk.steps;
    info->status = hk.status;
    info->converged = hk.converged;
    info->cycles = 0;
    info->lambda = 0.0;
    info->resnorm = hk.resnorm;
    info->gcv = NAN;
    copy_gk_scalars(hk, hk.steps, info);
  }
  if (k_opt) *k_opt = hk.steps > 0 ? (int)hk.sweeps : 0;
  return hk.status;
}

int dctk_krylov_project(dctk_ctx ctx, dctk_krylov ws, int k, const dctk_solve_opts* opts, void* X,
                        dctk_solve_info* info) {
  int r = ws_check(ctx, ws, DCTK_KRYLOV_GKB);
  if (r) return r;
  if (!X || !opts) return DCTK_EINVAL;
  if (!ws->initialised || k < 1 || k > ws->host_steps) return DCTK_EINVAL;
  if (opts->gcv_mode < 0 || opts->gcv_mode > 2) return DCTK_EINVAL;
  if (opts->gcv_mode == 2 && opts->lambda < 0.0 && !(opts->target > 0.0 && std::isfinite(opts->target)))
    return DCTK_EINVAL;
  if (std::isnan(opts->lambda) || std::isinf(opts->lambda) || opts->lambda == 0.0) return DCTK_EINVAL;
  dctk_op op = ws->op;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  if (opts->gcv_mode == 2 && opts->lambda < 0.0)
    DCTK_HIP(ctx, launch_projected_disc(ctx, ws->st, opts->target, k));
  else
    DCTK_HIP(ctx, launch_projected(ctx, ws->st, 1, opts->gcv_mode, opts->lambda < 0.0 ? -1.0 : opts->lambda, k));
  // the basis vectors beyond a breakdown are never formed: combine min(k, steps) of them
  DCTK_HIP(ctx, launch_combine(ctx, op->vec_dtype, op->p * op->n2 * op->s, X, nullptr, ws->V, ws->nvec, k,
                               &ws->st->steps, ws->st->y, Gate{nullptr, 0, 0}, ws->vmask, ws->st->alpha));
  static thread_local KState hk;
  if ((r = read_state_lsqr(ctx, ws, &hk))) return r;
  if (info) {
    info->iters = hk.steps < k ? hk.steps : k;
    info->status = hk.status;
    info->converged = hk.converged;
    info->cycles = 0;
    info->lambda = hk.lambda;
    info->resnorm = std::fabs(hk.phibar[info->iters < 0 ? 0 : info->iters]);
    info->gcv = opts->lambda < 0.0 ? hk.gcv : NAN;
    copy_gk_scalars(hk, info->iters, info);
  }
  return hk.status;
}

int dctk_lsqr_learned_solve(dctk_ctx ctx, dctk_krylov ws, dctk_mlp mlp, const void* C, void* X,
                            const dctk_solve_opts* opts, double gate, dctk_solve_info* info, int* pred_k,
                            int* accepted) {
  int r = ws_check(ctx, ws, DCTK_KRYLOV_GKB);
  if (r) return r;
  if (!C || !X || !mlp) return DCTK_EINVAL;
  if ((r = check_solve_opts(opts, ws))) return r;
  if (opts->lambda >= 0.0 || opts->gcv_mode == 2 || !(gate >= 1.0) || !std::isfinite(gate)) return DCTK_EINVAL;
  const int kf = 8;  // steps whose scalars feed the network
  if (opts->k_max < kf) return DCTK_EINVAL;
  dctk_op op = ws->op;
  const size_t ve = op->vec_dtype == DCTK_F64 ? 8 : 4;
  if (ranges_overlap(C, (size_t)(op->p * op->n1 * op->s) * ve, X, (size_t)(op->p * op->n2 * op->s) * ve))
    return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  ws->reorth = opts->reorth;
  DCTK_HIP(ctx, gkb_init_impl(ctx, ws, C, nullptr, opts->tol));
  DCTK_HIP(ctx, gkb_steps_tik(ctx, ws, 1, kf));
  float pred[5];
  DCTK_HIP(ctx, mlp_predict(ctx, mlp, ws->st, kf, opts->k_max, pred));
  const bool valid = pred[4] > 0.5f;
  const int kstop = valid ? (int)pred[3] : opts->k_max;
  DCTK_HIP(ctx, gkb_steps_tik(ctx, ws, kf + 1, kstop));
  ws->host_steps = kstop;
  ws->initialised = 1;
  DCTK_HIP(ctx, launch_projected(ctx, ws->st, 1, opts->gcv_mode, -1.0, 0, valid ? (double)pred[2] : -1.0, gate));
  DCTK_HIP(ctx, launch_combine(ctx, op->vec_dtype, op->p * op->n2 * op->s, X, nullptr, ws->V, ws->nvec, kstop,
                               &ws->st->steps, ws->st->y, Gate{nullptr, 0, 0}, ws->vmask, ws->st->alpha));
  double gate_ok = 0.0;
  DCTK_HIP(ctx, hipMemcpyAsync(&gate_ok, &ws->st->gate_ok, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (pred_k) *pred_k = valid ? kstop : -1;
  if (accepted) *accepted = gate_ok > 0.5 ? 1 : 0;
  return lsqr_info(ctx, ws, opts, info);
}

int dctk_gmres_tik_solve(dctk_ctx ctx, dctk_krylov ws, const void* C, void* X, int cycles,
                         const dctk_solve_opts* opts, dctk_solve_info* info) {
  int r = ws_check(ctx, ws, DCTK_KRYLOV_ARNOLDI);
  if (r) return r;
  if (!C || !X) return DCTK_EINVAL;
  if (cycles < 1) return DCTK_EINVAL;
  if ((r = check_solve_opts(opts, ws))) return r;
  if (opts->gcv_mode == 2) return DCTK_EINVAL;  // the discrepancy principle: DC-GK only
  dctk_op op = ws->op;
  const size_t ve = op->vec_dtype == DCTK_F64 ? 8 : 4;
  const int64_t n = op->p * op->n1 * op->s;
  if (ranges_overlap(C, (size_t)n * ve, X, (size_t)n * ve)) return DCTK_EINVAL;
  DCTK_HIP(ctx, hipSetDevice(ctx->device));
  KState* st = ws->st;
  const Gate g0{st, 0, 0};  // open unless the solve halted
  const int m = opts->k_max;
  DCTK_HIP(ctx, launch_state_reset(ctx, st, 1, opts->tol));
  // R_0 = C - M(X_0) with the partials of ||R_0||^2
  Ctl cr{};
  cr.kind = CTL_PLAIN;
  cr.a = -1.0;
  cr.b = 1.0;
  cr.s = 1.0;
  cr.st = st;
  cr.part_out = ws->partB;
  double* partR = ws->partB;
  int npR = 0;
  // the residual partials live in partB only until the cycle start consumes them
  DCTK_HIP(ctx, apply_op(op, ctx->stream, 0, X, ws->R, C, nullptr, cr, &npR));
  for (int c = 0; c < cycles; ++c) {
    DCTK_HIP(ctx, launch_state_reset(ctx, st, 0, 0.0));
    DCTK_HIP(ctx, arnoldi_start_impl(ctx, ws, ws->R, partR, npR));
    for (int j2 = 1; j2 <= m; ++j2) DCTK_HIP(ctx, arnoldi_step_impl(ctx, ws, j2));
    DCTK_HIP(ctx, launch_arn_finish(ctx, ws->partA, ws->last_npart, st, m + 1));
    DCTK_HIP(ctx, launch_projected(ctx, st, 0, opts->gcv_mode, opts->lambda < 0.0 ? -1.0 : opts->lambda));
    DCTK_HIP(ctx, launch_combine(ctx, op->vec_dtype, n, X, X, ws->U, ws->nvec, m, &st->steps, st->y, g0));
    DCTK_HIP(ctx, apply_op(op, ctx->stream, 0, X, ws->R, C, nullptr, cr, &npR));
    DCTK_HIP(ctx, launch_gmres_res(ctx, partR, npR, st));
  }
  ws->host_steps = 0;
  ws->initialised = 0;
  HostState hs;
  if ((r = read_state(ctx, ws, &hs))) return r;
  if (info) {
    info->iters = hs.total_steps;
    info->status = hs.status;
    info->converged = hs.converged;
    info->cycles = hs.cycles;
    info->lambda = hs.lambda;
    info->resnorm = hs.resnorm;
    info->gcv = opts->lambda < 0.0 ? hs.gcv : NAN;
  }
  return hs.status;
}

}  // extern "C"
