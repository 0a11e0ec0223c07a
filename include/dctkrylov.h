/*
 * libdctkrylov -- discrete cosine tensor Krylov solvers on AMD Instinct MI355X (gfx950).
 *
 * Implements the c-product of El Ichi, El Guide and Jbilou, "Discrete cosine
 * transform LSQR and GMRES methods for multidimensional ill-posed problems"
 * (arXiv:2103.11847), its exact adjoint, and the global Golub-Kahan / LSQR and
 * global Arnoldi / GMRES solvers with projected Tikhonov regularisation and GCV.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Tensors.  A third-order tensor T in R^{n1 x n2 x n3} is a dense buffer of
 *   n3*n1*n2 elements holding frontal slice k (0-based) at offset k*n1*n2,
 *   each slice row-major: element (i, j, k) at [k*n1*n2 + i*n2 + j].  The
 *   paper's p is n3.  "Vectors" of the Krylov methods are tensors
 *   X in R^{n2 x s x p} (buffer length p*n2*s) or R^{n1 x s x p}.
 * Pointers.  Unless a parameter says "host", every tensor pointer is a device
 *   pointer on the context's device, owned by the caller; the library never
 *   frees or reallocates it.  Buffers may not overlap unless stated.
 * Streams.  All GPU work of a call is enqueued on the context's stream.
 *   Kernel-level calls (tube transforms, products, single Krylov steps) are
 *   asynchronous; calls that fill a host struct or host array synchronise
 *   the stream once before returning.
 * Errors.  Every call returns an int status.  Arguments are validated
 *   before anything is enqueued.  DCTK_BREAKDOWN is a positive status: the
 *   partial result is valid.  A failing HIP call maps to DCTK_EHIP and its
 *   hipError_t is available from dctk_last_hip_error.  No C++ exception
 *   crosses this interface.
 * Threads.  A context and the objects made from it are used by one host
 *   thread at a time.
 */
#ifndef DCTKRYLOV_H
#define DCTKRYLOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define DCTK_OK 0
#define DCTK_BREAKDOWN 1      /* Krylov breakdown (Algorithm 2 step 3(d)); result valid */
#define DCTK_EINVAL (-1)      /* NULL pointer, bad enum, non-finite scalar, k out of range */
#define DCTK_ESHAPE (-2)      /* inconsistent or non-positive dimensions */
#define DCTK_EDTYPE (-3)      /* unsupported dtype combination */
#define DCTK_ENOMEM (-4)      /* device or host allocation failed */
#define DCTK_EHIP (-5)        /* a HIP runtime call failed */
#define DCTK_ENONFINITE (-6)  /* the input or a Krylov scalar is NaN/Inf */
#define DCTK_ESTATE (-7)      /* call out of order (e.g. step before init) */

/* ---- element types --------------------------------------------------- */
#define DCTK_F64 0
#define DCTK_F32 1
#define DCTK_BF16 2
#define DCTK_F16 3

/* ---- tube transforms (Sec. 2.2) --------------------------------------- */
/* DCTK_TUBE_TH:   L = M = W^{-1} C_n (I + Z) of Remark 2.1 (W = diag of the
 *                 first column of C_n, Z = ones on the superdiagonal).  With
 *                 this L, Algorithm 1 computes exactly the Definition
 *                 A *c B = ten(mat(A) mat(B)) of Sec. 2.2.  Default.
 * DCTK_TUBE_DCT2: L = C_n, the orthonormal DCT-II of eq. (dft1), i.e. the
 *                 Matlab dct of Algorithm 1 step 1 read literally.          */
#define DCTK_TUBE_TH 0
#define DCTK_TUBE_DCT2 1

/* which matrix of the transform family (dctk_tube_matrix) */
#define DCTK_MAT_L 0          /* L          forward transform                    */
#define DCTK_MAT_LINV 1       /* L^{-1}     inverse transform                    */
#define DCTK_MAT_LINVT 2      /* L^{-T}     forward transform of the adjoint     */
#define DCTK_MAT_LT 3         /* L^{T}      inverse transform of the adjoint     */

typedef struct dctk_ctx_s* dctk_ctx;
typedef struct dctk_op_s* dctk_op;
typedef struct dctk_krylov_s* dctk_krylov;
typedef struct dctk_mlp_s* dctk_mlp;

/* ---- context ---------------------------------------------------------- */
/* Creates a context bound to HIP device `device` and the HIP stream
 * `hip_stream` (a hipStream_t; NULL = the null stream).  The context owns
 * small device scratch for reductions.  Error: DCTK_EINVAL (out NULL),
 * DCTK_EHIP (device cannot be set). */
int dctk_create(dctk_ctx* out, int device, void* hip_stream);
int dctk_destroy(dctk_ctx ctx);
/* Replaces the stream used by later calls (same device). */
int dctk_set_stream(dctk_ctx ctx, void* hip_stream);
/* Waits for all work enqueued by this context. */
int dctk_synchronize(dctk_ctx ctx);
/* Static English text for a status code; never NULL. */
const char* dctk_status_string(int status);
/* The hipError_t of the last failing HIP call made for ctx (0 if none). */
int dctk_last_hip_error(dctk_ctx ctx);
/* Interface version (major*100 + minor). */
int dctk_version(void);

/* Kernel timing.  Between dctk_profile_begin and dctk_profile_end the
 * library times every c-product launch it enqueues for this context with
 * HIP events on the context's stream (a fused product's events are recorded
 * by its own dispatch, so they time the kernel alone; the unfused kinds are
 * bracketed by separate event records).  dctk_profile_end synchronises and
 * writes, per kind, the summed device time in ms to ms[DCTK_PROF_KINDS] and
 * the launch count to count[DCTK_PROF_KINDS] (either may be NULL).  Kinds:
 * 0 forward tube transform, 1 slice GEMMs of one product, 2 inverse tube
 * transform with epilogue (these three make up an unfused product), 3 one
 * fused forward product M(X), 4 one fused adjoint product M*(Y), 5 an
 * inverse transform with its epilogue paired with the next product's forward
 * transform (the Golub-Kahan steps of a Tikhonov solve with three-kernel
 * products, FP32 vectors, 16 <= p <= 64).
 * Error: DCTK_ESTATE if not profiling. */
#define DCTK_PROF_KINDS 6
int dctk_profile_begin(dctk_ctx ctx);
int dctk_profile_end(dctk_ctx ctx, double* ms, int* count);

/* ---- tube transforms (Algorithm 1 steps 1 and 3; Remark 2.1) ----------- */
/* Host helper: writes the p x p matrix `which` (DCTK_MAT_*) of transform
 * `tube`, row-major FP64, into the host array out[p*p].  Built in FP64 from
 * the closed forms of eq. (dft1) and Remark 2.1.  No GPU is touched. */
int dctk_tube_matrix(int tube, int which, int64_t p, double* out);

/* out = in x_3 G along the tubes: out[k][e] = sum_t G[k][t] in[t][e] for
 * e < count, where in/out hold p slices of `count` elements (count = n1*n2
 * of a tensor) and G = L (adjoint_pair = 0) or L^{-T} (adjoint_pair = 1).
 * dtype: DCTK_F64 or DCTK_F32 (both buffers).  in and out must not overlap. */
int dctk_tube_fwd(dctk_ctx ctx, int tube, int adjoint_pair, int dtype, int64_t p, int64_t count,
                  const void* in, void* out);
/* Same with G = L^{-1} (adjoint_pair = 0) or L^{T} (adjoint_pair = 1). */
int dctk_tube_inv(dctk_ctx ctx, int tube, int adjoint_pair, int dtype, int64_t p, int64_t count,
                  const void* in, void* out);
/* Tubes longer than 64: dctk_tube_fwd and dctk_tube_inv accept a power-of-two
 * p up to 4096 (DCTK_F32) or 2048 (DCTK_F64) and hand it to the O(p log p)
 * transform below, enqueued without synchronising.  Other p > 64 give
 * DCTK_ESHAPE. */

/* Fast tube transform (the fast DCT credited to the method in Sec. 1 and
 * Sec. 2.1): out = in x_3 G with G = matrix `which` (DCTK_MAT_*) of `tube`,
 * as the DCT-II of one complex FFT of length p per tube (Makhoul's
 * reordering) wrapped in the O(p) factors of Remark 2.1:
 * M = W^{-1} C_n (I + Z) = D^{-1} F (I + Z) with F the unnormalised DCT-II
 * and D = diag(cos(pi k / (2p))); the inverses of (I + Z) and (I + Z^T) are
 * alternating suffix and prefix sums.  Layout as dctk_tube_fwd: in/out hold p
 * slices of `count` elements, slice-major, DCTK_F64 or DCTK_F32 (both).
 * p: a power of two, 16 <= p <= 4096 (DCTK_F32) or 2048 (DCTK_F64).
 * Enqueued on the context's stream; returns without synchronising and
 * allocates nothing; the caller keeps both buffers alive until the stream
 * has run the work.  Rounding: FP32 results agree with the dense transform
 * to a relative 1e-6 (p = 256) to 4e-6 (p = 1024) in the 2-norm; the row
 * scaling D^{-1} (up to 2p / pi) amplifies the FFT's rounding by up to that
 * factor for the last rows of M and M^{-T}.  Blocks of E / p >= 2 tubes
 * (E = 4096 FP32, 2048 FP64) share complex FFTs in pairs: position e of a
 * block is the real part, e + E / (2p) the imaginary part, so a tube's error
 * is bounded relative to the norm of the pair's outputs (within 4x the
 * whole-array figures above), not its own: a tube next to a partner 1e4
 * times larger gets ~1e4 times its own relative error.
 * Errors: DCTK_EINVAL (NULL, bad tube/which, in and out overlap),
 * DCTK_EDTYPE, DCTK_ESHAPE (p not allowed, count <= 0), DCTK_ESTATE (while a
 * batch plan is being recorded), DCTK_EHIP. */
int dctk_tube_fast(dctk_ctx ctx, int tube, int which, int dtype, int64_t p, int64_t count, const void* in,
                   void* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the transform of
 * dctk_tube_fwd / dctk_tube_inv without allocating.  out = in x_3 G with
 * G = matrix `which` (DCTK_MAT_L, _LINV, _LINVT, _LT) of `tube`; layout, dtype
 * and overlap rules as dctk_tube_fwd.  Where dctk_tube_fwd copies G into a
 * device buffer allocated and freed per call (and synchronises), this call
 * builds G on the device into a fixed staging array of the library
 * (64 x 64 FP64 = 32 KB per GPU, held until the process ends) and only
 * enqueues: no hipMalloc, hipFree or host synchronisation.  p <= 64 uses the
 * staging array; a power-of-two p up to 4096 (DCTK_F32) or 2048 (DCTK_F64)
 * goes to dctk_tube_fast, which stages nothing; any other p gives
 * DCTK_ESHAPE.  All calls on one GPU share the staging array: calls that
 * overlap on one GPU (other streams, other contexts or host threads) race and
 * must be ordered by the caller.  The result equals dctk_tube_fwd /
 * dctk_tube_inv's to rounding (the device builds G from the same closed
 * forms).  Errors: DCTK_EINVAL, DCTK_EDTYPE, DCTK_ESHAPE, DCTK_ESTATE (while a
 * batch plan is being recorded), DCTK_EHIP. */
int dctk_tube_apply_noalloc(dctk_ctx ctx, int tube, int which, int dtype, int64_t p, int64_t count,
                            const void* in, void* out);


/* ---- operators M(X) = A *c X  or  A *c X *c B  (eq. 2) ------------------ */
/* Creates the operator of eq. (2) from A in R^{n1 x n2 x p} (device, FP64,
 * the layout above) and, if B != NULL, B in R^{s x s x p} (device, FP64).
 * The transform-domain slices A~ = A x_3 L (and B~) are computed once in FP64
 * and stored in `gemm_dtype` (DCTK_F64, DCTK_F32, DCTK_BF16 or DCTK_F16),
 * owned by the operator.  The operator acts on vectors X in R^{n2 x s x p}.
 * Vector element type: DCTK_F64 when gemm_dtype is DCTK_F64, else DCTK_F32
 * (BF16/F16 operators cast the transformed vector to the GEMM type and
 * accumulate in FP32).  A and B are only read during this call.
 * Tube length: p <= 64 keeps the four p x p transform matrices and applies
 * them on the matrix cores; a power-of-two p from 128 to 2048 uses the
 * O(p log p) transform of dctk_tube_fast for A~, B~ and both transforms of
 * every product (the fast DCT of Sec. 1 and Sec. 2.1), with the same
 * products, workspaces, solvers and batches.
 * Errors: DCTK_ESHAPE (a dimension <= 0, or p > 64 and not a power of two
 * up to 2048), DCTK_EDTYPE, DCTK_ENOMEM. */
int dctk_op_create(dctk_ctx ctx, int tube, int gemm_dtype, int64_t p, int64_t n1, int64_t n2,
                   const void* A, int64_t s, const void* B, dctk_op* out);
/* Order-N operators (the recursive extension to higher-order tensors that
 * Sec. 1 states): A in R^{n1 x n2 x n3 x ... x nN}, X in R^{n2 x s x n3 x ...
 * x nN}, with ntube = N - 2 tube modes of sizes tube_dims[0] = n3, ...,
 * tube_dims[ntube-1] = nN (host array).  Storage: (nN, ..., n3, rows, cols)
 * row-major, i.e. the order-3 layout with p = n3 * ... * nN frontal slices
 * and flattened slice index q = k3 + n3 (k4 + n4 (...)).  The product is the
 * order-3 Definition applied recursively over the last mode (blocks in the
 * Toeplitz-plus-Hankel pattern, multiplied by the order-(N-1) product); it
 * is computed by the transform of every tube mode, which on q is the single
 * matrix L_{nN} (x) ... (x) L_{n3}, so every product path, Krylov workspace
 * and solver of an order-3 operator applies unchanged.  1 <= ntube <= 6,
 * product of tube_dims <= 64; ntube = 1 is dctk_op_create.
 * Errors as dctk_op_create (DCTK_ESHAPE also for ntube out of range). */
int dctk_op_create_nd(dctk_ctx ctx, int tube, int gemm_dtype, int ntube, const int64_t* tube_dims,
                      int64_t n1, int64_t n2, const void* A, int64_t s, const void* B, dctk_op* out);
int dctk_op_destroy(dctk_op op);

/* Product paths.  A product (and its adjoint) runs either fused -- one
 * kernel doing the tube transform while staging tiles, the p slice GEMMs on
 * the matrix cores and the inverse transform in the epilogue (one-sided
 * operators with p <= 8) -- or as three kernels: tube transform, batched slice
 * GEMMs, inverse transform with epilogue (Algorithm 1 steps 1-3).  The
 * output tile edge of the GEMM part is 16, 32 or 64 (fused) or 32, 64, 128
 * or 256 (three kernels; 128 not for FP64; 256, tiles of 256 x 128, only for
 * BF16 and FP16 GEMMs).  All paths compute the same product;
 * results differ only by the rounding of the contraction order.
 * dctk_op_autotune: times every path and tile the operator can take, `reps`
 * launches each (1..1000) of the forward and of the adjoint product on ctx's
 * stream, and keeps the fastest per direction for all later products of op.
 * choice (host int[4], may be NULL) receives {forward path, forward tile,
 * adjoint path, adjoint tile} with path 1 = fused, 0 = three kernels.
 * Synchronises; allocates and frees two temporary vectors.
 * dctk_op_set_path: sets a direction's path (-1 = chosen by problem size, the
 * default) and tile (0 = by problem size).  Errors: DCTK_EINVAL for a path
 * or tile the operator cannot take. */
int dctk_op_autotune(dctk_ctx ctx, dctk_op op, int reps, int* choice);
int dctk_op_set_path(dctk_op op, int adjoint, int path, int tile);
/* dims[0..7] = p, n1, n2, s, two_sided, gemm_dtype, vec_dtype, tube. */
int dctk_op_info(dctk_op op, int64_t* dims);

/* Y = a * M(X) + b * Y   (Algorithm 1 applied to eq. 2).  X: p x n2 x s,
 * Y: p x n1 x s, both in the operator's vector type.  b == 0 never reads Y.
 * X and Y must not overlap.  Asynchronous. */
int dctk_cprod(dctk_ctx ctx, dctk_op op, double a, const void* X, double b, void* Y);
/* X = a * M*(Y) + b * X, with M* the exact adjoint of M under the inner
 * product <A, B> = sum a_ijk b_ijk of Sec. 2.2 (the paper's A^T *c, which it
 * uses in Algorithms 4 and 6 without defining it).  For DCTK_TUBE_DCT2 this
 * is the slice-transpose product; for DCTK_TUBE_TH it uses L^{-T} and L^T. */
int dctk_cprod_T(dctk_ctx ctx, dctk_op op, double a, const void* Y, double b, void* X);

/* ---- Krylov workspaces and single steps (Algorithms 2 and 4) ------------ */
#define DCTK_KRYLOV_GKB 0       /* Golub-Kahan (Algorithm 4) + LSQR (Algorithm 6) */
#define DCTK_KRYLOV_ARNOLDI 1   /* global Arnoldi (Algorithm 2)                    */

#define DCTK_REORTH_NONE 0      /* paper-literal                                */
#define DCTK_REORTH_V 1         /* GKB: reorthogonalise V_{j+1} against V_1..V_j  */
#define DCTK_REORTH_FULL 2      /* GKB: both U and V (classical Gram-Schmidt x2)  */

#define DCTK_ORTHO_MGS 0        /* Arnoldi: modified Gram-Schmidt (Algorithm 2)   */
#define DCTK_ORTHO_CGS2 1       /* Arnoldi: classical Gram-Schmidt applied twice  */

/* Allocates a device workspace for `kind` on operator op: the bases
 * (k_max + 1 vectors each), the FP64 projected matrix and scalars, and the
 * iterate buffers.  The workspace belongs to op's context and must be
 * destroyed before op.  k_max in [1, 64]. */
int dctk_krylov_create(dctk_ctx ctx, dctk_op op, int kind, int k_max, int ortho, dctk_krylov* out);
int dctk_krylov_destroy(dctk_krylov ws);

/* Algorithm 4 step 2 on C (p x n1 x s): beta_1 = ||C||, U_1 = C/beta_1,
 * alpha_1 = ||M*(U_1)||, V_1 = M*(U_1)/alpha_1, and the LSQR start of
 * Algorithm 6 step 2 (W_1 = V_1, X_0 = 0, rhobar_1 = alpha_1, phibar_1 = beta_1).
 * `reorth` is DCTK_REORTH_*.  Asynchronous. */
int dctk_gkb_init(dctk_ctx ctx, dctk_krylov ws, const void* C, int reorth, double tol);
/* One pass of Algorithm 4 step 3 (a)-(f) together with the LSQR update of
 * Algorithm 6 steps 3(c)-(g).  All scalars stay on the device; after a
 * breakdown or once |phibar_{j+1}| < tol the step is a no-op.  Asynchronous.
 * Error: DCTK_ESTATE if not initialised or k_max steps were taken. */
int dctk_gkb_step(dctk_ctx ctx, dctk_krylov ws);
/* Algorithm 2 step 2 on V (p x n1 x s, n1 == n2): beta = ||V||, V_1 = V/beta. */
int dctk_arnoldi_init(dctk_ctx ctx, dctk_krylov ws, const void* V);
/* One pass of Algorithm 2 step 3 (a)-(e): column j of H~ on the device. */
int dctk_arnoldi_step(dctk_ctx ctx, dctk_krylov ws);

/* Synchronises and copies the workspace scalars to host arrays (any may be
 * NULL):  GKB: alpha[0..k_max] = alpha_1.., beta[0..k_max] = beta_1..;
 * Arnoldi: H[(k_max+1) * k_max] row-major h_{i+1,j+1}, beta[0] = ||V||.
 * info[0..5] = steps taken, status (DCTK_OK / DCTK_BREAKDOWN), converged
 * flag, the capacity k_max, the Jacobi sweeps of the last projected solve
 * (0 when it needed no SVD: DC-GK with the rectangular GCV or a fixed
 * lambda), and the GMRES cycles run. */
int dctk_krylov_read(dctk_ctx ctx, dctk_krylov ws, double* alpha, double* beta_or_H, int* info);
/* Device pointer to basis vector j (0-based) of basis `which`
 * (0 = U for GKB / V for Arnoldi, 1 = V for GKB), or to the LSQR iterate X
 * (which = 2) and search direction W (which = 3) -- formed by dctk_gkb_step
 * and by solves with lambda == 0 only.  Owned by the workspace.  A Tikhonov
 * solve without reorthogonalisation (lambda != 0) writes no normalised copy
 * of its intermediate basis vectors: after k steps, GKB slots 1..k-1 hold
 * beta_{j+1} U_{j+1} and alpha_{j+1} V_{j+1} (the recorded alpha, beta of
 * dctk_krylov_read); slots 0 and k hold the normalised vectors. */
int dctk_krylov_basis(dctk_krylov ws, int which, int j, void** ptr);

/* Enqueues a copy of the vector named by (which, j) as in dctk_krylov_basis
 * into the caller's device buffer dst (p*n1*s or p*n2*s elements of the
 * vector type).  Asynchronous. */
int dctk_krylov_copy(dctk_ctx ctx, dctk_krylov ws, int which, int j, void* dst);

/* ---- solvers ------------------------------------------------------------ */
typedef struct {
  int k_max;        /* GKB steps (LSQR) or Arnoldi steps per cycle (GMRES), <= workspace k_max */
  int reorth;       /* DCTK_REORTH_* (GKB only) */
  int gcv_mode;     /* how lambda < 0 is chosen: 0: GCV of the rectangular projected problem;
                       1: GCV as printed in eq. (gcv2); 2 (DC-GK only): the discrepancy principle
                       (Sec. 2), lambda with ||C - M(X_lambda)|| = target */
  int reserved;
  double lambda;    /* < 0: lambda chosen by gcv_mode; 0: no Tikhonov (LSQR iterate / GMRES LS); > 0: fixed */
  double tol;       /* stop when the residual norm < tol; 0 runs k_max steps / all cycles */
  double target;    /* gcv_mode 2: the residual norm eta * delta (noise norm delta, eta >= 1), > 0 */
} dctk_solve_opts;

typedef struct {
  int iters;        /* GKB steps taken (LSQR) or total Arnoldi steps (GMRES) */
  int status;       /* DCTK_OK or DCTK_BREAKDOWN */
  int converged;    /* 1 when stopped by tol */
  int cycles;       /* GMRES cycles run */
  double lambda;    /* regularisation parameter used (last cycle for GMRES) */
  double resnorm;   /* LSQR: |phibar_{k+1}| = ||C - M(X_LSQR)||;  GMRES: ||C - M(X)|| */
  double gcv;       /* GCV value at lambda (NaN when lambda was not chosen by GCV) */
  /* Optional caller-owned host arrays (the library never allocates or frees
   * them; NULL or cap <= 0: not written).  After a DC-LSQR / DC-GK solve
   * (dctk_lsqr_tik_solve, dctk_lsqr_lcurve_solve, dctk_krylov_project, the
   * batches) they receive the Golub-Kahan scalars of Algorithm 4,
   * alpha[j] = alpha_{j+1} and beta[j] = beta_{j+1} for j < min(cap, iters + 1)
   * (beta_1 = ||C||_F).  DC-GMRES leaves them untouched. */
  double* alpha;
  double* beta;
  int cap;
  int reserved;
} dctk_solve_info;

/* DC-LSQR / DC-GK (Algorithms 4, 5, 6) for min ||M(X) - C||: runs k_max
 * Golub-Kahan steps with the LSQR recurrence (X_0 = 0).  lambda == 0 returns
 * the LSQR iterate of Algorithm 6; otherwise X = V_k (*) y_lambda with y the
 * projected Tikhonov solution of eq. (normeq2) (lambda > 0 fixed, < 0 chosen
 * by GCV), computed in FP64 on the device.  With lambda != 0 the LSQR iterate
 * and search direction (dctk_krylov_basis which = 2, 3) are not formed, and
 * with no reorthogonalisation each step's LSQR update runs inside the next
 * forward product (same recurrence; two launches per step when both products
 * are fused, in the forward transform of the three-kernel product otherwise).  ws must be a DCTK_KRYLOV_GKB workspace of op.
 * C: p x n1 x s, X (output): p x n2 x s.  Synchronises once to fill info
 * and returns the solve's status; with info NULL the solve is only enqueued
 * on ctx's stream (no read-back, no synchronisation, DCTK_OK once enqueued),
 * so solves can follow each other on the device without host round trips. */
int dctk_lsqr_tik_solve(dctk_ctx ctx, dctk_krylov ws, const void* C, void* X,
                        const dctk_solve_opts* opts, dctk_solve_info* info);
/* DC-GMRES(m) with Tikhonov on every cycle (Algorithm 3), m = opts->k_max,
 * `cycles` restart cycles (the paper's itermax), X (p x n2 x s, n1 == n2)
 * holds X_0 on entry and the result on exit.  ws must be a
 * DCTK_KRYLOV_ARNOLDI workspace of op.  Synchronises once to fill info. */
int dctk_gmres_tik_solve(dctk_ctx ctx, dctk_krylov ws, const void* C, void* X, int cycles,
                         const dctk_solve_opts* opts, dctk_solve_info* info);

/* LSQR with the stopping index from the L-curve (Sec. 3.2, after Algorithm
 * 6): runs k_max Golub-Kahan steps (opts->lambda and gcv_mode are ignored;
 * reorth and tol as for dctk_lsqr_tik_solve), evaluates for every k the
 * LSQR iterate's residual ||C - M(X_k)|| = |phibar_{k+1}| and norm ||X_k||
 * from the projected bidiagonal in FP64 on the device, takes as k_opt the
 * corner of the curve (log ||R_k||, log ||X_k||): the interior point of
 * largest curvature of the circle through it and its neighbours, turning the
 * way an L-curve's corner turns (k_opt = steps taken when no point does), and
 * returns X = X_{k_opt}.  info->resnorm is its residual norm, *k_opt (may be
 * NULL) the index.  Synchronises once.  ws must be a DCTK_KRYLOV_GKB
 * workspace of op; C: p x n1 x s, X (output): p x n2 x s. */
int dctk_lsqr_lcurve_solve(dctk_ctx ctx, dctk_krylov ws, const void* C, void* X,
                           const dctk_solve_opts* opts, dctk_solve_info* info, int* k_opt);

/* Algorithm 5 at step count k from the bases a finished (or stepped) GKB
 * workspace holds: the projected Tikhonov solution of the first k steps (k in
 * [1, steps enqueued]; lambda fixed (> 0) or by GCV (< 0); opts->k_max, reorth
 * and tol are ignored) and X = V_k (*) y.  The workspace is left as it was,
 * apart from its recorded lambda / GCV.  Synchronises to fill info. */
int dctk_krylov_project(dctk_ctx ctx, dctk_krylov ws, int k, const dctk_solve_opts* opts, void* X,
                        dctk_solve_info* info);

/* ---- learned stopping index and regularisation parameter ---------------- */
/* A 16-64-64-2 network with GELU activations predicts, from the first 8 GKB
 * steps, log lambda and the stopping index of DC-LSQR / DC-GK (the paper
 * leaves both to the user or to GCV, Sec. 3.1 and Sec. 4).  Inputs: for j =
 * 1..8, log(alpha_j / beta_j) and log(|phibar_{j+1}| / beta_1) (Algorithms 4
 * and 6).  Outputs (t_lambda, t_k) are normalised: lambda = exp(t_lambda sigma
 * + mu), k = round(t_k k_scale + k_offset) (dctk_mlp_set_scaling; defaults 0,
 * 1, 40, 0; k_offset is a calibrated safety margin: stopping late costs steps,
 * stopping early costs restoration error).
 * Parameters: DCTK_MLP_PARAMS FP32 values [W1 (64x16), b1 (64), W2 (64x64),
 * b2 (64), W3 (2x64), b3 (2)], weights row-major (output, input); every pass
 * uses them rounded to bfloat16 and accumulates in FP32.  Training minimises
 * (1/2B) sum_b [w_lambda (out_b0 - T_b0)^2 + w_k (out_b1 - T_b1)^2] with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).  Device arrays: X is B x 16, outputs
 * and targets B x 2, row-major FP32; B in [1, DCTK_MLP_MAX_BATCH].
 * dctk_mlp_create: Xavier-uniform weights from a splitmix64 stream of `seed`,
 *   zero biases.  Owns its parameters, Adam moments and scratch.
 * dctk_mlp_set_params / get_params: host FP32 master values (set also resets
 *   Adam); get may also return the bfloat16 bits (host_bf16, may be NULL).
 * dctk_mlp_forward: out = network(X), async.
 * dctk_mlp_gradient: grad (device, DCTK_MLP_PARAMS) of sum_b <dout_b, out_b>.
 * dctk_mlp_train_step: one Adam step on the loss above; *loss (host, may be
 *   NULL; synchronises when given) receives the loss before the step.
 * dctk_mlp_features: the 16 inputs of a GKB workspace after >= 8 steps into
 *   out16 (device); NaN when unavailable (fewer steps, breakdown).
 * dctk_lsqr_learned_solve: DC-GK with the learned stop: 8 GKB steps, the
 *   network's (lambda, k) (k clamped to [8, opts->k_max]), GKB steps up to k,
 *   then Algorithm 5 at k with lambda = the prediction if GCV(prediction) <=
 *   gate * min GCV (gate >= 1), else the GCV minimiser.  opts->lambda must be
 *   < 0.  *pred_k gets k (-1: no valid prediction; then k_max steps and GCV),
 *   *accepted 1 when the predicted lambda passed the gate.  Synchronises
 *   twice (after the prediction and at the end). */
#define DCTK_MLP_PARAMS 5378
#define DCTK_MLP_MAX_BATCH (1 << 20)
int dctk_mlp_create(dctk_ctx ctx, uint64_t seed, dctk_mlp* out);
int dctk_mlp_destroy(dctk_mlp m);
int dctk_mlp_set_params(dctk_ctx ctx, dctk_mlp m, const float* host);
int dctk_mlp_get_params(dctk_ctx ctx, dctk_mlp m, float* host, uint16_t* host_bf16);
int dctk_mlp_set_scaling(dctk_mlp m, double mu, double sigma, double k_scale, double k_offset);
int dctk_mlp_forward(dctk_ctx ctx, dctk_mlp m, int B, const float* X, float* out);
int dctk_mlp_gradient(dctk_ctx ctx, dctk_mlp m, int B, const float* X, const float* dout, float* grad);
int dctk_mlp_train_step(dctk_ctx ctx, dctk_mlp m, int B, const float* X, const float* T, double w_lambda,
                        double w_k, double lr, double* loss);
int dctk_mlp_features(dctk_ctx ctx, dctk_krylov ws, float* out16);
int dctk_lsqr_learned_solve(dctk_ctx ctx, dctk_krylov ws, dctk_mlp mlp, const void* C, void* X,
                            const dctk_solve_opts* opts, double gate, dctk_solve_info* info, int* pred_k,
                            int* accepted);

/* ---- batches of independent solves ------------------------------------- */
/* Many DC-LSQR / DC-GK solves (Algorithms 4, 5, 6) of independent problems
 * of uneven n1, n2, s and n3, run together.  The plan records, for every
 * instance, the kernel launches dctk_lsqr_tik_solve would enqueue with opts;
 * the launches of one kernel at the same point of the schedule are merged,
 * across instances, into one launch whose workgroups each look up their
 * instance; the resulting schedule (one launch per kernel variant per
 * schedule point) is captured once into a HIP graph.  Every instance computes
 * exactly what its own dctk_lsqr_tik_solve would.
 *
 * dctk_batch_create: count in [1, DCTK_BATCH_MAX]; ws[i] DCTK_KRYLOV_GKB
 *   workspaces of distinct operators on ctx's device (the products of a batch
 *   run concurrently and an operator's transform scratch is not shared);
 *   C[i] (p x n1 x s) and X[i]
 *   (p x n2 x s) device buffers of instance i in its vector type, captured by
 *   the plan (every run reads C[i] and writes X[i]; they must outlive the
 *   batch).  opts applies to all (k_max <= each workspace's).  With mlp !=
 *   NULL every instance uses the learned stop without a host round trip:
 *   after step 8 the network sets, on the device, the instance's step limit
 *   (later steps' kernels exit at once) and its proposed lambda, which the
 *   projected solve keeps when GCV(proposal) <= gate * min GCV (opts->lambda
 *   < 0, k_max >= 8, gate >= 1).  The plan holds mlp's parameters by
 *   reference: later training changes later runs.  use_graph = 0 replays the merged launches from the host
 *   instead of a graph.  The batch owns device copies of the launch arguments
 *   (allocated here, freed by dctk_batch_destroy).  Errors: DCTK_EINVAL on a
 *   bad argument, DCTK_ENOMEM, DCTK_EHIP.
 * dctk_batch_run: enqueues one run of all solves on ctx's stream (async).
 * dctk_batch_info: synchronises and fills infos[0..count) as
 *   dctk_lsqr_tik_solve would; returns DCTK_OK or the first non-OK status.
 * dctk_batch_stats: launches per run of the merged schedule, and of the
 *   same solves run one by one (either may be NULL).
 * dctk_batch_learned: synchronises; per instance the learned step limit (0:
 *   none) and whether the proposed lambda passed the gate (host arrays of
 *   count, either may be NULL).
 * dctk_batch_destroy: synchronises ctx's stream and frees the plan. */
#define DCTK_BATCH_MAX 256
typedef struct dctk_batch_s* dctk_batch;
int dctk_batch_create(dctk_ctx ctx, int count, const dctk_krylov* ws, const void* const* C, void* const* X,
                      const dctk_solve_opts* opts, dctk_mlp mlp, double gate, int use_graph, dctk_batch* out);
int dctk_batch_learned(dctk_ctx ctx, dctk_batch b, int* k_limit, int* accepted);
int dctk_batch_run(dctk_ctx ctx, dctk_batch b);
int dctk_batch_info(dctk_ctx ctx, dctk_batch b, dctk_solve_info* infos);
int dctk_batch_stats(dctk_batch b, int* merged_launches, int* single_launches);
int dctk_batch_destroy(dctk_batch b);
/* One call for a batch solved once: for ops[0..count) (distinct operators on
 * ctx's device) creates a DCTK_KRYLOV_GKB workspace of opts->k_max steps per
 * operator, plans the batch (graph-captured merged launches, no learned
 * stop), runs it once, fills infos[0..count) (alpha / beta as described at
 * dctk_solve_info when the caller set them) and frees the workspaces and the
 * plan.  C[i] / X[i] as for dctk_batch_create.  Synchronises.  Returns
 * DCTK_OK or the first non-OK solve status; errors as dctk_batch_create. */
int dctk_batch_lsqr_tik_solve(dctk_ctx ctx, int count, const dctk_op* ops, const void* const* C, void* const* X,
                              const dctk_solve_opts* opts, dctk_solve_info* infos);

#ifdef __cplusplus
}
#endif

#endif /* DCTKRYLOV_H */
