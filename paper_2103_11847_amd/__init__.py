"""libdctkrylov: discrete cosine tensor Krylov solvers on AMD Instinct MI355X.

Thin Python binding of the C-ABI declared in include/dctkrylov.h.  Every
function here has the name of the C entry point it calls and only marshals
arguments (torch tensors -> device pointers, structs -> ctypes); all
arithmetic runs in the HIP library.  Importing the package does not load
the library; the first call does, and raises if it is missing or cannot be
loaded (there is no fallback).

Tensors are torch tensors on the GPU, contiguous, shaped (p, rows, cols):
frontal slice k is t[k].
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdctkrylov.so")

DCTK_OK, DCTK_BREAKDOWN = 0, 1
DCTK_EINVAL, DCTK_ESHAPE, DCTK_EDTYPE, DCTK_ENOMEM, DCTK_EHIP, DCTK_ENONFINITE, DCTK_ESTATE = -1, -2, -3, -4, -5, -6, -7
DCTK_F64, DCTK_F32, DCTK_BF16, DCTK_F16 = 0, 1, 2, 3
DCTK_TUBE_TH, DCTK_TUBE_DCT2 = 0, 1
DCTK_MAT_L, DCTK_MAT_LINV, DCTK_MAT_LINVT, DCTK_MAT_LT = 0, 1, 2, 3
DCTK_KRYLOV_GKB, DCTK_KRYLOV_ARNOLDI = 0, 1
DCTK_REORTH_NONE, DCTK_REORTH_V, DCTK_REORTH_FULL = 0, 1, 2
DCTK_ORTHO_MGS, DCTK_ORTHO_CGS2 = 0, 1
DCTK_BATCH_MAX = 256
DCTK_MLP_PARAMS = 5378
DCTK_MLP_MAX_BATCH = 1 << 20

TUBES = {"th": DCTK_TUBE_TH, "dct2": DCTK_TUBE_DCT2}
DTYPES = {"f64": DCTK_F64, "f32": DCTK_F32, "bf16": DCTK_BF16, "f16": DCTK_F16}


class DctkError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (where, _status_string(status), status))


class dctk_solve_opts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int), ("reorth", ctypes.c_int), ("gcv_mode", ctypes.c_int),
                ("reserved", ctypes.c_int), ("lam", ctypes.c_double), ("tol", ctypes.c_double),
                ("target", ctypes.c_double)]


class dctk_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("converged", ctypes.c_int),
                ("cycles", ctypes.c_int), ("lam", ctypes.c_double), ("resnorm", ctypes.c_double),
                ("gcv", ctypes.c_double), ("alpha", ctypes.POINTER(ctypes.c_double)),
                ("beta", ctypes.POINTER(ctypes.c_double)), ("cap", ctypes.c_int), ("reserved", ctypes.c_int)]

    def as_dict(self):
        return {"iters": self.iters, "status": self.status, "converged": self.converged,
                "cycles": self.cycles, "lambda": self.lam, "resnorm": self.resnorm, "gcv": self.gcv}


def solve_info_with_scalars(cap):
    """A dctk_solve_info whose alpha / beta point at host arrays of `cap` doubles
    (returned with it: keep them alive while the info is in use)."""
    a = (ctypes.c_double * cap)()
    b = (ctypes.c_double * cap)()
    info = dctk_solve_info()
    info.alpha = ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
    info.beta = ctypes.cast(b, ctypes.POINTER(ctypes.c_double))
    info.cap = cap
    return info, a, b


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_L = ctypes.c_int64
_D = ctypes.c_double
_SIGS = {
    "dctk_create": (_I, [ctypes.POINTER(_P), _I, _P]),
    "dctk_destroy": (_I, [_P]),
    "dctk_set_stream": (_I, [_P, _P]),
    "dctk_synchronize": (_I, [_P]),
    "dctk_status_string": (ctypes.c_char_p, [_I]),
    "dctk_last_hip_error": (_I, [_P]),
    "dctk_version": (_I, []),
    "dctk_profile_begin": (_I, [_P]),
    "dctk_profile_end": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I)]),
    "dctk_tube_matrix": (_I, [_I, _I, _L, ctypes.POINTER(_D)]),
    "dctk_tube_fwd": (_I, [_P, _I, _I, _I, _L, _L, _P, _P]),
    "dctk_tube_inv": (_I, [_P, _I, _I, _I, _L, _L, _P, _P]),
    "dctk_tube_fast": (_I, [_P, _I, _I, _I, _L, _L, _P, _P]),
    "dctk_tube_apply_noalloc": (_I, [_P, _I, _I, _I, _L, _L, _P, _P]),
    "dctk_op_create": (_I, [_P, _I, _I, _L, _L, _L, _P, _L, _P, ctypes.POINTER(_P)]),
    "dctk_op_create_nd": (_I, [_P, _I, _I, _I, ctypes.POINTER(_L), _L, _L, _P, _L, _P, ctypes.POINTER(_P)]),
    "dctk_op_destroy": (_I, [_P]),
    "dctk_op_info": (_I, [_P, ctypes.POINTER(_L)]),
    "dctk_op_autotune": (_I, [_P, _P, _I, ctypes.POINTER(_I)]),
    "dctk_op_set_path": (_I, [_P, _I, _I, _I]),
    "dctk_cprod": (_I, [_P, _P, _D, _P, _D, _P]),
    "dctk_cprod_T": (_I, [_P, _P, _D, _P, _D, _P]),
    "dctk_krylov_create": (_I, [_P, _P, _I, _I, _I, ctypes.POINTER(_P)]),
    "dctk_krylov_destroy": (_I, [_P]),
    "dctk_gkb_init": (_I, [_P, _P, _P, _I, _D]),
    "dctk_gkb_step": (_I, [_P, _P]),
    "dctk_arnoldi_init": (_I, [_P, _P, _P]),
    "dctk_arnoldi_step": (_I, [_P, _P]),
    "dctk_krylov_read": (_I, [_P, _P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_I)]),
    "dctk_krylov_basis": (_I, [_P, _I, _I, ctypes.POINTER(_P)]),
    "dctk_krylov_copy": (_I, [_P, _P, _I, _I, _P]),
    "dctk_lsqr_tik_solve": (_I, [_P, _P, _P, _P, ctypes.POINTER(dctk_solve_opts), ctypes.POINTER(dctk_solve_info)]),
    "dctk_lsqr_lcurve_solve": (_I, [_P, _P, _P, _P, ctypes.POINTER(dctk_solve_opts), ctypes.POINTER(dctk_solve_info),
                                    ctypes.POINTER(_I)]),
    "dctk_gmres_tik_solve": (_I, [_P, _P, _P, _P, _I, ctypes.POINTER(dctk_solve_opts),
                                  ctypes.POINTER(dctk_solve_info)]),
    "dctk_krylov_project": (_I, [_P, _P, _I, ctypes.POINTER(dctk_solve_opts), _P, ctypes.POINTER(dctk_solve_info)]),
    "dctk_mlp_create": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "dctk_mlp_destroy": (_I, [_P]),
    "dctk_mlp_set_params": (_I, [_P, _P, ctypes.POINTER(ctypes.c_float)]),
    "dctk_mlp_get_params": (_I, [_P, _P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_uint16)]),
    "dctk_mlp_set_scaling": (_I, [_P, _D, _D, _D, _D]),
    "dctk_mlp_forward": (_I, [_P, _P, _I, _P, _P]),
    "dctk_mlp_gradient": (_I, [_P, _P, _I, _P, _P, _P]),
    "dctk_mlp_train_step": (_I, [_P, _P, _I, _P, _P, _D, _D, _D, ctypes.POINTER(_D)]),
    "dctk_mlp_features": (_I, [_P, _P, _P]),
    "dctk_lsqr_learned_solve": (_I, [_P, _P, _P, _P, _P, ctypes.POINTER(dctk_solve_opts), _D,
                                     ctypes.POINTER(dctk_solve_info), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "dctk_batch_create": (_I, [_P, _I, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                               ctypes.POINTER(dctk_solve_opts), _P, _D, _I, ctypes.POINTER(_P)]),
    "dctk_batch_learned": (_I, [_P, _P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "dctk_batch_run": (_I, [_P, _P]),
    "dctk_batch_info": (_I, [_P, _P, ctypes.POINTER(dctk_solve_info)]),
    "dctk_batch_stats": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "dctk_batch_destroy": (_I, [_P]),
    "dctk_batch_lsqr_tik_solve": (_I, [_P, _I, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                       ctypes.POINTER(dctk_solve_opts), ctypes.POINTER(dctk_solve_info)]),
}
EXPORTED = tuple(sorted(_SIGS))


def lib():
    """Load libdctkrylov.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdctkrylov.so is not built (%s); run python -m paper_2103_11847_amd.build"
                               % LIB_PATH)
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _status_string(status):
    try:
        return lib().dctk_status_string(status).decode()
    except Exception:  # noqa: BLE001 - message formatting only
        return "status %d" % status


def _check(status, where, allow_breakdown=True):
    if status == DCTK_OK or (allow_breakdown and status == DCTK_BREAKDOWN):
        return status
    raise DctkError(status, where)


def _ptr(t, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("expected %s, got %s" % (dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _torch():
    import torch
    return torch


def _vec_torch_dtype(code):
    torch = _torch()
    return torch.float64 if code == DCTK_F64 else torch.float32


# ---- context -------------------------------------------------------------------
def dctk_version():
    return lib().dctk_version()


def dctk_create(device=0, stream=None):
    """Context on `device` and a HIP stream (a torch stream or raw pointer; default: torch's current)."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    h = ctypes.c_void_p()
    _check(lib().dctk_create(ctypes.byref(h), int(device), ctypes.c_void_p(sp)), "dctk_create")
    return h


def dctk_destroy(ctx):
    return _check(lib().dctk_destroy(ctx), "dctk_destroy")


def dctk_set_stream(ctx, stream):
    sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return _check(lib().dctk_set_stream(ctx, ctypes.c_void_p(sp)), "dctk_set_stream")


def dctk_synchronize(ctx):
    return _check(lib().dctk_synchronize(ctx), "dctk_synchronize")


def dctk_status_string(status):
    return lib().dctk_status_string(int(status)).decode()


def dctk_last_hip_error(ctx):
    return lib().dctk_last_hip_error(ctx)


PROF_KINDS = ("tube_fwd", "gemm", "tube_inv", "fused_fwd", "fused_adj", "tube_pair")


def dctk_profile_begin(ctx):
    return _check(lib().dctk_profile_begin(ctx), "dctk_profile_begin")


def dctk_profile_end(ctx):
    """Returns {kind: (ms_total, launches)} for the kinds in PROF_KINDS."""
    ms = (ctypes.c_double * len(PROF_KINDS))()
    cnt = (ctypes.c_int * len(PROF_KINDS))()
    _check(lib().dctk_profile_end(ctx, ms, cnt), "dctk_profile_end")
    return {k: (ms[i], cnt[i]) for i, k in enumerate(PROF_KINDS)}


# ---- tube transforms ----------------------------------------------------------------
def dctk_tube_matrix(tube, which, p):
    """The p x p transform matrix (host, FP64) as a nested list."""
    buf = (ctypes.c_double * (p * p))()
    _check(lib().dctk_tube_matrix(int(tube), int(which), int(p), buf), "dctk_tube_matrix")
    return [[buf[i * p + j] for j in range(p)] for i in range(p)]


def _tube_call(fn, name, ctx, tube, adjoint_pair, x, out):
    torch = _torch()
    code = DCTK_F64 if x.dtype == torch.float64 else DCTK_F32
    if x.dtype not in (torch.float64, torch.float32) or out.dtype != x.dtype or out.shape != x.shape:
        raise ValueError("tube transform needs matching float32/float64 tensors")
    p = x.shape[0]
    count = x.numel() // p if p else 0
    return _check(fn(ctx, int(tube), int(adjoint_pair), code, p, count, _ptr(x), _ptr(out)), name)


def dctk_tube_fwd(ctx, tube, adjoint_pair, x, out):
    return _tube_call(lib().dctk_tube_fwd, "dctk_tube_fwd", ctx, tube, adjoint_pair, x, out)


def dctk_tube_inv(ctx, tube, adjoint_pair, x, out):
    return _tube_call(lib().dctk_tube_inv, "dctk_tube_inv", ctx, tube, adjoint_pair, x, out)


def dctk_tube_fast(ctx, tube, which, x, out):
    """O(p log p) transform by matrix `which` (DCTK_MAT_*); enqueued, no synchronisation."""
    return _tube_call(lib().dctk_tube_fast, "dctk_tube_fast", ctx, tube, which, x, out)


def dctk_tube_apply_noalloc(ctx, tube, which, x, out):
    """Transform by matrix `which` (DCTK_MAT_*) without allocating; enqueued only."""
    return _tube_call(lib().dctk_tube_apply_noalloc, "dctk_tube_apply_noalloc", ctx, tube, which, x, out)


# ---- operators ----------------------------------------------------------------------
def dctk_op_create(ctx, tube, gemm_dtype, A, s, B=None):
    """A: (p, n1, n2) float64 GPU tensor; B: optional (p, s, s) float64."""
    torch = _torch()
    p, n1, n2 = A.shape
    h = ctypes.c_void_p()
    _check(lib().dctk_op_create(ctx, int(tube), int(gemm_dtype), p, n1, n2, _ptr(A, torch.float64), int(s),
                                _ptr(B, torch.float64), ctypes.byref(h)), "dctk_op_create")
    return h


def dctk_op_create_nd(ctx, tube, gemm_dtype, A, s, B=None):
    """Order-N operator.  A: float64 GPU tensor shaped (nN, ..., n3, n1, n2);
    B: optional (nN, ..., n3, s, s).  Vectors are (nN, ..., n3, rows, s), or
    equivalently the order-3 layout with p = n3 * ... * nN slices."""
    torch = _torch()
    n1, n2 = A.shape[-2], A.shape[-1]
    dims = list(reversed(A.shape[:-2]))
    arr = (ctypes.c_int64 * len(dims))(*dims)
    h = ctypes.c_void_p()
    _check(lib().dctk_op_create_nd(ctx, int(tube), int(gemm_dtype), len(dims), arr, n1, n2, _ptr(A, torch.float64),
                                   int(s), _ptr(B, torch.float64), ctypes.byref(h)), "dctk_op_create_nd")
    return h


def dctk_op_destroy(op):
    return _check(lib().dctk_op_destroy(op), "dctk_op_destroy")


def dctk_op_info(op):
    d = (ctypes.c_int64 * 8)()
    _check(lib().dctk_op_info(op, d), "dctk_op_info")
    keys = ("p", "n1", "n2", "s", "two_sided", "gemm_dtype", "vec_dtype", "tube")
    return dict(zip(keys, list(d)))


def dctk_op_autotune(ctx, op, reps=10):
    """Time the product paths and tiles of op; returns {fwd_path, fwd_tile, adj_path, adj_tile}."""
    ch = (ctypes.c_int * 4)()
    _check(lib().dctk_op_autotune(ctx, op, int(reps), ch), "dctk_op_autotune")
    return {"fwd_path": ch[0], "fwd_tile": ch[1], "adj_path": ch[2], "adj_tile": ch[3]}


def dctk_op_set_path(op, adjoint, path, tile=0):
    return _check(lib().dctk_op_set_path(op, int(adjoint), int(path), int(tile)), "dctk_op_set_path")


def dctk_cprod(ctx, op, a, X, b, Y):
    return _check(lib().dctk_cprod(ctx, op, float(a), _ptr(X), float(b), _ptr(Y)), "dctk_cprod")


def dctk_cprod_T(ctx, op, a, Y, b, X):
    return _check(lib().dctk_cprod_T(ctx, op, float(a), _ptr(Y), float(b), _ptr(X)), "dctk_cprod_T")


# ---- Krylov workspaces ---------------------------------------------------------------
def dctk_krylov_create(ctx, op, kind, k_max, ortho=DCTK_ORTHO_MGS):
    h = ctypes.c_void_p()
    _check(lib().dctk_krylov_create(ctx, op, int(kind), int(k_max), int(ortho), ctypes.byref(h)),
           "dctk_krylov_create")
    return h


def dctk_krylov_destroy(ws):
    return _check(lib().dctk_krylov_destroy(ws), "dctk_krylov_destroy")


def dctk_gkb_init(ctx, ws, C, reorth=DCTK_REORTH_NONE, tol=0.0):
    return _check(lib().dctk_gkb_init(ctx, ws, _ptr(C), int(reorth), float(tol)), "dctk_gkb_init")


def dctk_gkb_step(ctx, ws):
    return _check(lib().dctk_gkb_step(ctx, ws), "dctk_gkb_step")


def dctk_arnoldi_init(ctx, ws, V):
    return _check(lib().dctk_arnoldi_init(ctx, ws, _ptr(V)), "dctk_arnoldi_init")


def dctk_arnoldi_step(ctx, ws):
    return _check(lib().dctk_arnoldi_step(ctx, ws), "dctk_arnoldi_step")


def dctk_krylov_read(ctx, ws, k_max, kind):
    """Returns dict(alpha, beta | H, beta0, steps, status, converged)."""
    info = (ctypes.c_int * 6)()
    if kind == DCTK_KRYLOV_GKB:
        a = (ctypes.c_double * (k_max + 1))()
        b = (ctypes.c_double * (k_max + 1))()
        _check(lib().dctk_krylov_read(ctx, ws, a, b, info), "dctk_krylov_read")
        return {"alpha": list(a), "beta": list(b), "steps": info[0], "status": info[1], "converged": info[2],
                "sweeps": info[4]}
    a = (ctypes.c_double * 1)()
    H = (ctypes.c_double * ((k_max + 1) * k_max))()
    _check(lib().dctk_krylov_read(ctx, ws, a, H, info), "dctk_krylov_read")
    Hm = [[H[i * k_max + j] for j in range(k_max)] for i in range(k_max + 1)]
    return {"H": Hm, "beta0": a[0], "steps": info[0], "status": info[1], "converged": info[2],
            "sweeps": info[4], "cycles": info[5]}


def dctk_krylov_basis(ws, which, j):
    p = ctypes.c_void_p()
    _check(lib().dctk_krylov_basis(ws, int(which), int(j), ctypes.byref(p)), "dctk_krylov_basis")
    return p.value


# ---- solvers ----------------------------------------------------------------------------
def make_opts(k_max, reorth=DCTK_REORTH_NONE, gcv_mode=0, lam=-1.0, tol=0.0, target=0.0):
    return dctk_solve_opts(int(k_max), int(reorth), int(gcv_mode), 0, float(lam), float(tol), float(target))


def dctk_lsqr_tik_solve(ctx, ws, C, X, opts, info=True):
    """info=False: enqueue only (the library gets a NULL info; nothing is read back).
    info may also be a dctk_solve_info to fill (e.g. from solve_info_with_scalars)."""
    if isinstance(info, dctk_solve_info):
        _check(lib().dctk_lsqr_tik_solve(ctx, ws, _ptr(C), _ptr(X), ctypes.byref(opts), ctypes.byref(info)),
               "dctk_lsqr_tik_solve")
        return info
    if not info:
        _check(lib().dctk_lsqr_tik_solve(ctx, ws, _ptr(C), _ptr(X), ctypes.byref(opts), None),
               "dctk_lsqr_tik_solve")
        return None
    out = dctk_solve_info()
    _check(lib().dctk_lsqr_tik_solve(ctx, ws, _ptr(C), _ptr(X), ctypes.byref(opts), ctypes.byref(out)),
           "dctk_lsqr_tik_solve")
    return out


def dctk_lsqr_lcurve_solve(ctx, ws, C, X, opts):
    """LSQR stopped at the L-curve corner; returns (info, k_opt)."""
    out = dctk_solve_info()
    k = _I()
    _check(lib().dctk_lsqr_lcurve_solve(ctx, ws, _ptr(C), _ptr(X), ctypes.byref(opts), ctypes.byref(out),
                                        ctypes.byref(k)), "dctk_lsqr_lcurve_solve")
    return out, k.value


def dctk_gmres_tik_solve(ctx, ws, C, X, cycles, opts):
    info = dctk_solve_info()
    _check(lib().dctk_gmres_tik_solve(ctx, ws, _ptr(C), _ptr(X), int(cycles), ctypes.byref(opts),
                                      ctypes.byref(info)), "dctk_gmres_tik_solve")
    return info


def dctk_krylov_project(ctx, ws, k, opts, X):
    """Algorithm 5 at step count k from a stepped GKB workspace into X."""
    info = dctk_solve_info()
    _check(lib().dctk_krylov_project(ctx, ws, int(k), ctypes.byref(opts), _ptr(X), ctypes.byref(info)),
           "dctk_krylov_project")
    return info


def dctk_mlp_create(ctx, seed=0):
    h = ctypes.c_void_p()
    _check(lib().dctk_mlp_create(ctx, ctypes.c_uint64(seed), ctypes.byref(h)), "dctk_mlp_create")
    return h.value


def dctk_mlp_destroy(m):
    return _check(lib().dctk_mlp_destroy(m), "dctk_mlp_destroy")


def dctk_mlp_set_params(ctx, m, params):
    """params: sequence of DCTK_MLP_PARAMS floats (host)."""
    arr = (ctypes.c_float * DCTK_MLP_PARAMS)(*[float(x) for x in params])
    return _check(lib().dctk_mlp_set_params(ctx, m, arr), "dctk_mlp_set_params")


def dctk_mlp_get_params(ctx, m):
    """Returns (FP32 master params, bfloat16 bit patterns) as Python lists."""
    arr = (ctypes.c_float * DCTK_MLP_PARAMS)()
    bits = (ctypes.c_uint16 * DCTK_MLP_PARAMS)()
    _check(lib().dctk_mlp_get_params(ctx, m, arr, bits), "dctk_mlp_get_params")
    return list(arr), list(bits)


def dctk_mlp_set_scaling(m, mu, sigma, k_scale, k_offset=0.0):
    return _check(lib().dctk_mlp_set_scaling(m, float(mu), float(sigma), float(k_scale), float(k_offset)),
                  "dctk_mlp_set_scaling")


def dctk_mlp_forward(ctx, m, X, out):
    return _check(lib().dctk_mlp_forward(ctx, m, int(X.shape[0]), _ptr(X), _ptr(out)), "dctk_mlp_forward")


def dctk_mlp_gradient(ctx, m, X, dout, grad):
    return _check(lib().dctk_mlp_gradient(ctx, m, int(X.shape[0]), _ptr(X), _ptr(dout), _ptr(grad)),
                  "dctk_mlp_gradient")


def dctk_mlp_train_step(ctx, m, X, T, w_lambda, w_k, lr, want_loss=False):
    loss = ctypes.c_double()
    _check(lib().dctk_mlp_train_step(ctx, m, int(X.shape[0]), _ptr(X), _ptr(T), float(w_lambda), float(w_k),
                                     float(lr), ctypes.byref(loss) if want_loss else None),
           "dctk_mlp_train_step")
    return loss.value if want_loss else None


def dctk_mlp_features(ctx, ws, out16):
    return _check(lib().dctk_mlp_features(ctx, ws, _ptr(out16)), "dctk_mlp_features")


def dctk_lsqr_learned_solve(ctx, ws, m, C, X, opts, gate=1.05):
    """Returns (info, predicted k or -1, 1 if the predicted lambda passed the gate)."""
    info = dctk_solve_info()
    k, acc = ctypes.c_int(), ctypes.c_int()
    _check(lib().dctk_lsqr_learned_solve(ctx, ws, m, _ptr(C), _ptr(X), ctypes.byref(opts), float(gate),
                                         ctypes.byref(info), ctypes.byref(k), ctypes.byref(acc)),
           "dctk_lsqr_learned_solve")
    return info, k.value, acc.value


def dctk_batch_create(ctx, ws_list, C_list, X_list, opts, use_graph=True, mlp=None, gate=1.05):
    """Plan a batch of DC-LSQR / DC-GK solves: ws_list[i] solves C_list[i] into X_list[i]
    (with the device-side learned stop when mlp is given)."""
    n = len(ws_list)
    if len(C_list) != n or len(X_list) != n:
        raise ValueError("dctk_batch_create: ws, C and X lists differ in length")
    arr = ctypes.c_void_p * n
    ws_a = arr(*[w for w in ws_list])
    c_a = arr(*[_ptr(c) for c in C_list])
    x_a = arr(*[_ptr(x) for x in X_list])
    h = ctypes.c_void_p()
    _check(lib().dctk_batch_create(ctx, n, ws_a, c_a, x_a, ctypes.byref(opts), mlp, float(gate),
                                   1 if use_graph else 0, ctypes.byref(h)), "dctk_batch_create")
    return h.value


def dctk_batch_run(ctx, batch):
    return _check(lib().dctk_batch_run(ctx, batch), "dctk_batch_run")


def dctk_batch_info(ctx, batch, count):
    infos = (dctk_solve_info * count)()
    _check(lib().dctk_batch_info(ctx, batch, infos), "dctk_batch_info")
    return list(infos)


def dctk_batch_learned(ctx, batch, count):
    """Per instance: (learned step limit, 1 if the proposed lambda passed the gate)."""
    kl = (ctypes.c_int * count)()
    acc = (ctypes.c_int * count)()
    _check(lib().dctk_batch_learned(ctx, batch, kl, acc), "dctk_batch_learned")
    return list(kl), list(acc)


def dctk_batch_stats(batch):
    m, s = ctypes.c_int(), ctypes.c_int()
    _check(lib().dctk_batch_stats(batch, ctypes.byref(m), ctypes.byref(s)), "dctk_batch_stats")
    return m.value, s.value


def dctk_batch_lsqr_tik_solve(ctx, ops, C_list, X_list, opts, infos=None):
    """One-shot batch of DC-LSQR / DC-GK solves on distinct operators; returns the infos
    (a list of dctk_solve_info, optionally the caller's own, e.g. with alpha/beta arrays)."""
    n = len(ops)
    if len(C_list) != n or len(X_list) != n:
        raise ValueError("dctk_batch_lsqr_tik_solve: ops, C and X lists differ in length")
    arr = ctypes.c_void_p * n
    infos_a = (dctk_solve_info * n)(*(infos if infos is not None else []))
    _check(lib().dctk_batch_lsqr_tik_solve(ctx, n, arr(*ops), arr(*[_ptr(c) for c in C_list]),
                                           arr(*[_ptr(x) for x in X_list]), ctypes.byref(opts), infos_a),
           "dctk_batch_lsqr_tik_solve")
    return list(infos_a)


def dctk_batch_destroy(batch):
    return _check(lib().dctk_batch_destroy(batch), "dctk_batch_destroy")


def dctk_krylov_copy(ctx, ws, which, j, dst):
    """Copy basis vector j of basis `which` (or X / W) into the GPU tensor dst."""
    return _check(lib().dctk_krylov_copy(ctx, ws, int(which), int(j), _ptr(dst)), "dctk_krylov_copy")
