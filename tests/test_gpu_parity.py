"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances (relative Frobenius unless stated):
  * c-product / adjoint / tube transform: 1e-10 in FP64, 1e-5 in FP32; the
    BF16/FP16 GEMM modes are held to the oracle's product with the same
    16-bit roundings of the operands (tests/rounding_model.py: 4e-4 in BF16,
    1e-4 in FP16, where the 16-bit rounding itself moves the product by
    1e-3..3e-3 and 3e-4..4e-4), and their error against the exact product
    may not exceed 1.25x the modelled one;
  * Golub-Kahan / Arnoldi scalars and solver iterates in FP64 with full
    reorthogonalisation on both sides: 1e-9 (the Krylov recurrences amplify
    the 1e-16 product error by the conditioning of the projected problem);
  * GCV: the GCV value at the library's lambda is within 1e-9 of the
    oracle's minimum, and X equals the oracle's X at the library's lambda.
"""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, metrics, tikhonov
from oracle import tube as otube
from oracle.cprod import Operator, fro
from tests import rounding_model as RM
from tests.gpu_util import rel, say, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2103_11847_amd as dk  # noqa: E402

F64, F32 = torch.float64, torch.float32
VT = {dk.DCTK_F64: F64, dk.DCTK_F32: F32, dk.DCTK_BF16: F32, dk.DCTK_F16: F32}
TOL_PROD = {dk.DCTK_F64: 1e-10, dk.DCTK_F32: 1e-5}
LOWP = {dk.DCTK_BF16: "bf16", dk.DCTK_F16: "f16"}


def assert_product(got, gdt, A, B, X, exact, adjoint=False, tube="th", label=""):
    """FP64/FP32: relative Frobenius error within TOL_PROD; BF16/FP16: within
    the rounding model's gap of the same roundings, and no worse than them."""
    if gdt not in LOWP:
        e = rel(got, exact)
        assert e <= TOL_PROD[gdt], (label, e)
        return e
    kind = LOWP[gdt]
    L = otube.transform_matrix(A.shape[0], tube)
    gap, e, e_model = RM.check_lowp(got, A, B, L, X, kind, exact, adjoint)
    say("  ", label, kind, "gap to rounding model", gap, "rel", e, "model", e_model)
    assert gap <= RM.MODEL_TOL[kind], (label, gap)
    assert e <= 1.25 * e_model, (label, e, e_model)
    return e


_OPS = []   # operator handles created by the tests, destroyed with the context


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dk.dctk_create(0)
    yield c
    dk.dctk_synchronize(c)
    while _OPS:
        dk.dctk_op_destroy(_OPS.pop())
    dk.dctk_destroy(c)


@pytest.fixture(autouse=True)
def _release_ops():
    """Destroy each test's operators when it ends (also when it fails)."""
    n = len(_OPS)
    yield
    torch.cuda.synchronize()
    while len(_OPS) > n:
        dk.dctk_op_destroy(_OPS.pop())


class Op:
    """Operator handle; destroyed by the fixtures above, never by __del__."""

    def __init__(self, ctx, A, B, s, gemm_dtype, tube="th"):
        self.ctx = ctx
        self.h = dk.dctk_op_create(ctx, dk.TUBES[tube], gemm_dtype, to_gpu(A, F64), s,
                                   None if B is None else to_gpu(B, F64))
        _OPS.append(self.h)
        self.vt = VT[gemm_dtype]
        self.oracle = Operator(A, B, tube)


# ------------------------------------------------------------------ transforms

@pytest.mark.parametrize("dtype", [dk.DCTK_F64, dk.DCTK_F32])
@pytest.mark.parametrize("tb", ["th", "dct2"])
@pytest.mark.parametrize("p,count", [(1, 37), (3, 4 * 1000 + 3), (8, 257), (31, 129), (64, 1024)])
def test_tube_transforms(ctx, dtype, tb, p, count):
    say("tube", dtype, tb, p, count)
    rng = np.random.default_rng(p * 7 + count)
    x = rng.standard_normal((p, count))
    xt = to_gpu(x, VT[dtype])
    L = otube.transform_matrix(p, tb)
    Li = np.linalg.inv(L)
    cases = [(dk.dctk_tube_fwd, 0, L), (dk.dctk_tube_fwd, 1, Li.T), (dk.dctk_tube_inv, 0, Li),
             (dk.dctk_tube_inv, 1, L.T)]
    for fn, adj, G in cases:
        out = torch.empty_like(xt)
        fn(ctx, dk.TUBES[tb], adj, xt, out)
        ref = G @ x
        assert rel(to_np(out), ref) <= TOL_PROD[dtype] * max(1.0, np.sqrt(p) / 4), (fn.__name__, adj)


# ------------------------------------------------------------------ c-product

PROD_SHAPES = [
    (3, 32, 32, 32),      # colour, one tile
    (3, 70, 45, 33),      # several tiles, ragged in every dimension
    (8, 64, 64, 64),
    (31, 17, 23, 5),
    (1, 100, 80, 7),
    (2, 129, 3, 65),
]


@pytest.mark.parametrize("gdt", [dk.DCTK_F64, dk.DCTK_F32])
@pytest.mark.parametrize("two_sided", [False, True])
@pytest.mark.parametrize("shape", PROD_SHAPES)
def test_cprod_and_adjoint(ctx, gdt, two_sided, shape):
    p, n1, n2, s = shape
    say("cprod", gdt, two_sided, shape)
    w = W.tiny_random(sum(shape), p, n1, n2, s, two_sided)
    op = Op(ctx, w["A"], w["B"], s, gdt)
    X = to_gpu(w["X"], op.vt)
    Y = torch.empty((p, n1, s), dtype=op.vt, device="cuda:0")
    dk.dctk_cprod(ctx, op.h, 1.0, X, 0.0, Y)
    assert rel(to_np(Y), op.oracle.apply(w["X"])) <= TOL_PROD[gdt]
    Yin = to_gpu(w["Y"], op.vt)
    Z = torch.empty((p, n2, s), dtype=op.vt, device="cuda:0")
    dk.dctk_cprod_T(ctx, op.h, 1.0, Yin, 0.0, Z)
    assert rel(to_np(Z), op.oracle.adjoint(w["Y"])) <= TOL_PROD[gdt]


@pytest.mark.parametrize("tb", ["th", "dct2"])
def test_cprod_epilogue_and_tubes(ctx, tb):
    say("epilogue", tb)
    p, n1, n2, s = 5, 40, 36, 24
    w = W.tiny_random(99, p, n1, n2, s, False)
    op = Op(ctx, w["A"], None, s, dk.DCTK_F64, tb)
    X = to_gpu(w["X"], F64)
    Y0 = w["Y"]
    Y = to_gpu(Y0, F64)
    dk.dctk_cprod(ctx, op.h, -0.75, X, 1.5, Y)
    assert rel(to_np(Y), -0.75 * op.oracle.apply(w["X"]) + 1.5 * Y0) <= 1e-10
    # b = 0 never reads Y (NaN in Y must not leak)
    Y.fill_(float("nan"))
    dk.dctk_cprod(ctx, op.h, 2.0, X, 0.0, Y)
    assert rel(to_np(Y), 2.0 * op.oracle.apply(w["X"])) <= 1e-10


def test_cprod_matches_definition_on_gpu(ctx):
    """The GPU product equals the literal Toeplitz-plus-Hankel Definition (brute force)."""
    from oracle.cprod import cprod_definition
    w = W.tiny_random(5, 4, 6, 5, 3, False)
    op = Op(ctx, w["A"], None, 3, dk.DCTK_F64)
    Y = torch.empty((4, 6, 3), dtype=F64, device="cuda:0")
    dk.dctk_cprod(ctx, op.h, 1.0, to_gpu(w["X"], F64), 0.0, Y)
    assert rel(to_np(Y), cprod_definition(w["A"], w["X"])) <= 1e-10


@pytest.mark.parametrize("gdt", [dk.DCTK_BF16, dk.DCTK_F16])
@pytest.mark.parametrize("two_sided", [False, True])
def test_low_precision_gemm_modes(ctx, gdt, two_sided):
    p, n1, n2, s = 3, 96, 80, 48
    say("lowp", gdt, two_sided)
    w = W.tiny_random(11, p, n1, n2, s, two_sided)
    op = Op(ctx, w["A"], w["B"], s, gdt)
    Y = torch.empty((p, n1, s), dtype=F32, device="cuda:0")
    dk.dctk_cprod(ctx, op.h, 1.0, to_gpu(w["X"], F32), 0.0, Y)
    assert_product(to_np(Y), gdt, w["A"], w["B"], w["X"], op.oracle.apply(w["X"]), label="lowp")
    Z = torch.empty((p, n2, s), dtype=F32, device="cuda:0")
    dk.dctk_cprod_T(ctx, op.h, 1.0, to_gpu(w["Y"], F32), 0.0, Z)
    assert_product(to_np(Z), gdt, w["A"], w["B"], w["Y"], op.oracle.adjoint(w["Y"]), adjoint=True,
                   label="lowp adjoint")


PATHS = [(1, 16), (1, 32), (1, 64), (0, 32), (0, 64), (0, 128), (0, 256)]


@pytest.mark.parametrize("gdt", [dk.DCTK_F64, dk.DCTK_F32, dk.DCTK_BF16, dk.DCTK_F16])
@pytest.mark.parametrize("shape,two_sided", [((3, 96, 80, 72), False), ((8, 64, 64, 64), False),
                                             ((5, 40, 56, 44), False), ((3, 33, 37, 29), False),
                                             ((4, 48, 48, 48), True), ((12, 70, 70, 36), False),
                                             ((64, 96, 96, 96), False), ((64, 96, 96, 96), True),
                                             ((64, 97, 83, 71), False)])
def test_every_product_path_and_tile(ctx, gdt, shape, two_sided):
    """Each product path / tile the operator can take (fused 16/32/64, three kernels with
    32/64/128 GEMM tiles) gives the oracle's product and adjoint."""
    p, n1, n2, s = shape
    w = W.tiny_random(sum(shape) + 5, p, n1, n2, s, two_sided)
    op = Op(ctx, w["A"], w["B"], s, gdt)
    X, Yin = to_gpu(w["X"], op.vt), to_gpu(w["Y"], op.vt)
    ref, ref_t = op.oracle.apply(w["X"]), op.oracle.adjoint(w["Y"])
    ran = 0
    for path, tile in PATHS:
        ok = True
        for adj in (0, 1):
            try:
                dk.dctk_op_set_path(op.h, adj, path, tile)
            except dk.DctkError:
                ok = False
        if not ok:
            continue
        say("path", shape, two_sided, gdt, path, tile)
        Y = torch.empty((p, n1, s), dtype=op.vt, device="cuda:0")
        dk.dctk_cprod(ctx, op.h, 1.0, X, 0.0, Y)
        assert_product(to_np(Y), gdt, w["A"], w["B"], w["X"], ref, label=("fwd", path, tile))
        Z = torch.empty((p, n2, s), dtype=op.vt, device="cuda:0")
        dk.dctk_cprod_T(ctx, op.h, 1.0, Yin, 0.0, Z)
        assert_product(to_np(Z), gdt, w["A"], w["B"], w["Y"], ref_t, adjoint=True, label=("adj", path, tile))
        ran += 1
    fusable = not two_sided and p <= 8
    assert ran >= (5 if fusable else 3) - (1 if fusable and gdt == dk.DCTK_F64 else 0)


def test_autotune_keeps_products_exact(ctx):
    p, n1, n2, s = 3, 128, 128, 128
    w = W.tiny_random(77, p, n1, n2, s, False)
    op = Op(ctx, w["A"], None, s, dk.DCTK_F32)
    ch = dk.dctk_op_autotune(ctx, op.h, 5)
    say("autotune", ch)
    assert ch["fwd_path"] in (0, 1) and ch["adj_path"] in (0, 1)
    assert ch["fwd_tile"] in (16, 32, 64, 128) and ch["adj_tile"] in (16, 32, 64, 128)
    Y = torch.empty((p, n1, s), dtype=F32, device="cuda:0")
    dk.dctk_cprod(ctx, op.h, 1.0, to_gpu(w["X"], F32), 0.0, Y)
    assert rel(to_np(Y), op.oracle.apply(w["X"])) <= 1e-5
    Z = torch.empty((p, n2, s), dtype=F32, device="cuda:0")
    dk.dctk_cprod_T(ctx, op.h, 1.0, to_gpu(w["Y"], F32), 0.0, Z)
    assert rel(to_np(Z), op.oracle.adjoint(w["Y"])) <= 1e-5
    with pytest.raises(dk.DctkError):
        dk.dctk_op_set_path(op.h, 0, 1, 128)
    with pytest.raises(dk.DctkError):
        dk.dctk_op_set_path(op.h, 2, 0, 32)


def test_ragged_and_degenerate_shapes(ctx):
    """n = 1 slices and s = 1 (a single column) run and agree."""
    for (p, n1, n2, s) in [(1, 1, 1, 1), (3, 1, 5, 1), (4, 5, 1, 2), (2, 3, 3, 1)]:
        w = W.tiny_random(3, p, n1, n2, s, True)
        op = Op(ctx, w["A"], w["B"], s, dk.DCTK_F64)
        Y = torch.empty((p, n1, s), dtype=F64, device="cuda:0")
        dk.dctk_cprod(ctx, op.h, 1.0, to_gpu(w["X"], F64), 0.0, Y)
        assert rel(to_np(Y), op.oracle.apply(w["X"])) <= 1e-10


def test_validation_errors(ctx):
    w = W.tiny_random(1, 3, 8, 8, 4, False)
    with pytest.raises(dk.DctkError) as e:
        dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, 9, to_gpu(w["A"], F64), 4)
    assert e.value.status == dk.DCTK_EDTYPE
    op = Op(ctx, w["A"], None, 4, dk.DCTK_F64)
    X = to_gpu(w["X"], F64)
    with pytest.raises(dk.DctkError) as e:
        dk.dctk_cprod(ctx, op.h, 1.0, X, 0.0, X)   # overlapping in/out
    assert e.value.status == dk.DCTK_EINVAL
    with pytest.raises(dk.DctkError) as e:
        dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, 65)
    assert e.value.status == dk.DCTK_EINVAL
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, 4)
    with pytest.raises(dk.DctkError) as e:
        dk.dctk_gkb_step(ctx, ws)                   # step before init
    assert e.value.status == dk.DCTK_ESTATE
    dk.dctk_krylov_destroy(ws)


# ---------------------------------------------------------- Krylov processes

def _krylov_problem(seed, p=3, n=24, s=10, two_sided=False):
    rng = np.random.default_rng(seed)
    A = 0.3 * rng.standard_normal((p, n, n)) / np.sqrt(n)
    A[0] += np.eye(n)
    B = None
    if two_sided:
        B = 0.3 * rng.standard_normal((p, s, s)) / np.sqrt(s)
        B[0] += np.eye(s)
    C = rng.standard_normal((p, n, s))
    return A, B, C


@pytest.mark.parametrize("two_sided", [False, True])
@pytest.mark.parametrize("reorth", [dk.DCTK_REORTH_FULL, dk.DCTK_REORTH_V])
def test_gkb_steps_match_oracle(ctx, two_sided, reorth):
    say("gkb", two_sided, reorth)
    A, B, C = _krylov_problem(3, two_sided=two_sided)
    k = 12
    op = Op(ctx, A, B, C.shape[2], dk.DCTK_F64)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    dk.dctk_gkb_init(ctx, ws, to_gpu(C, F64), reorth, 0.0)
    for _ in range(k):
        dk.dctk_gkb_step(ctx, ws)
    r = dk.dctk_krylov_read(ctx, ws, k, dk.DCTK_KRYLOV_GKB)
    g = krylov.gkb(op.oracle, C, k, "full" if reorth == dk.DCTK_REORTH_FULL else "v")
    assert r["steps"] == k and r["status"] == 0
    assert rel(r["alpha"][: k + 1], g.alpha[: k + 1]) <= 1e-9
    assert rel(r["beta"][: k + 1], g.beta[: k + 1]) <= 1e-9
    # bases: V_k and U_{k+1}
    v = torch.empty(C.shape, dtype=F64, device="cuda:0")
    dk.dctk_krylov_copy(ctx, ws, 1, k - 1, v)
    assert rel(to_np(v), g.V[k - 1]) <= 1e-8
    dk.dctk_krylov_copy(ctx, ws, 0, k, v)
    assert rel(to_np(v), g.U[k]) <= 1e-8
    dk.dctk_krylov_destroy(ws)


@pytest.mark.parametrize("ortho", [dk.DCTK_ORTHO_MGS, dk.DCTK_ORTHO_CGS2])
def test_arnoldi_steps_match_oracle(ctx, ortho):
    say("arnoldi", ortho)
    A, _, C = _krylov_problem(5)
    m = 10
    op = Op(ctx, A, None, C.shape[2], dk.DCTK_F64)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_ARNOLDI, m, ortho)
    dk.dctk_arnoldi_init(ctx, ws, to_gpu(C, F64))
    for _ in range(m):
        dk.dctk_arnoldi_step(ctx, ws)
    r = dk.dctk_krylov_read(ctx, ws, m, dk.DCTK_KRYLOV_ARNOLDI)
    ar = krylov.Arnoldi(op.oracle, C, m, "mgs" if ortho == dk.DCTK_ORTHO_MGS else "cgs2")
    for _ in range(m):
        ar.step()
    assert r["steps"] == m
    assert abs(r["beta0"] - ar.beta) <= 1e-12 * ar.beta
    assert rel(np.array(r["H"]), ar.H) <= 1e-9
    dk.dctk_krylov_destroy(ws)


@pytest.mark.parametrize("two_sided", [False, True])
def test_lsqr_iterate_matches_oracle(ctx, two_sided):
    """lambda = 0: the Algorithm 6 iterate, with full reorthogonalisation on both sides."""
    say("lsqr", two_sided)
    A, B, C = _krylov_problem(7, two_sided=two_sided)
    k = 15
    op = Op(ctx, A, B, C.shape[2], dk.DCTK_F64)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    X = torch.empty(C.shape, dtype=F64, device="cuda:0")
    info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(k, dk.DCTK_REORTH_FULL, 0, 0.0))
    ref = krylov.dc_lsqr(op.oracle, C, k, reorth="full")
    assert info.iters == k
    assert rel(to_np(X), ref["X"]) <= 1e-9
    assert abs(info.resnorm - ref["resnorm"]) <= 1e-9 * fro(C)
    dk.dctk_krylov_destroy(ws)


@pytest.mark.parametrize("lam", [0.05, 0.5])
def test_gk_fixed_lambda_matches_oracle(ctx, lam):
    A, _, C = _krylov_problem(9)
    k = 12
    op = Op(ctx, A, None, C.shape[2], dk.DCTK_F64)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    X = torch.empty(C.shape, dtype=F64, device="cuda:0")
    dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(k, dk.DCTK_REORTH_FULL, 0, lam))
    ref = krylov.dc_gk(op.oracle, C, k, lam=lam, reorth="full")
    assert rel(to_np(X), ref["X"]) <= 1e-9
    dk.dctk_krylov_destroy(ws)


@pytest.mark.parametrize("p,n,s,two_sided,pm", [(16, 40, 24, False, 16), (33, 32, 20, False, 48),
                                                (64, 24, 16, True, 64), (24, 36, 28, False, 32)])
def test_gk_paired_transforms_match_oracle(ctx, p, n, s, two_sided, pm):
    """Tikhonov solve with three-kernel products and FP32 vectors (every tile
    width of the paired transform kernel): each product's inverse transform
    also forms the next product's transformed input, and the basis vectors
    stay unnormalised in their slots.  The Golub-Kahan scalars match the
    oracle's FP64 process (no reorthogonalisation; 10 steps of a
    well-conditioned operator, where FP32 rounding moves them by ~1e-6), the
    last basis vectors (normalised by the flush) and X at a fixed lambda match
    the oracle's to FP32 accuracy."""
    say("paired", p, n, s, two_sided)
    A, B, C = _krylov_problem(50 + p, p=p, n=n, s=s, two_sided=two_sided)
    k = 10
    op = Op(ctx, A, B, s, dk.DCTK_F32)
    for adj in (0, 1):
        dk.dctk_op_set_path(op.h, adj, 0, 0)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    X = torch.empty(C.shape, dtype=F32, device="cuda:0")
    dk.dctk_profile_begin(ctx)
    info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F32), X, dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, 0.3))
    prof = dk.dctk_profile_end(ctx)
    # the paired path ran: two paired kernels per step; forward transforms only
    # for the initial adjoint product M*(C) and the first step, one inverse (M*(C)'s)
    assert prof["tube_pair"][1] == 2 * k and prof["tube_fwd"][1] == 2 and prof["tube_inv"][1] == 1
    g = krylov.gkb(op.oracle, C, k, "none")
    r = dk.dctk_krylov_read(ctx, ws, k, dk.DCTK_KRYLOV_GKB)
    assert r["steps"] == k and info.iters == k
    ea, eb = rel(r["alpha"][: k + 1], g.alpha[: k + 1]), rel(r["beta"][: k + 1], g.beta[: k + 1])
    v = torch.empty(C.shape, dtype=F32, device="cuda:0")
    dk.dctk_krylov_copy(ctx, ws, 1, k, v)
    ev = rel(to_np(v), g.V[k])
    dk.dctk_krylov_copy(ctx, ws, 0, k, v)
    eu = rel(to_np(v), g.U[k])
    ref = krylov.dc_gk(op.oracle, C, k, lam=0.3, reorth="none")
    ex = rel(to_np(X), ref["X"])
    say("  alpha", ea, "beta", eb, "V", ev, "U", eu, "X", ex)
    assert ea <= 1e-5 and eb <= 1e-5
    assert ev <= 1e-4 and eu <= 1e-4
    assert ex <= 1e-4
    dk.dctk_krylov_destroy(ws)


@pytest.mark.parametrize("gdt,p,tol", [(dk.DCTK_F64, 3, 1e-9), (dk.DCTK_F32, 16, 1e-5)])
def test_gkb_steps_continue_after_tikhonov_solve(ctx, gdt, p, tol):
    """A Tikhonov solve leaves its intermediate basis vectors unnormalised and
    normalises the last U and V in place; single GKB steps taken after it
    continue the same process: alpha, beta of the continued steps and the last
    basis vectors match the oracle's longer process (FP64 fused products; FP32
    three-kernel products with paired transforms)."""
    say("continue", gdt, p)
    A, _, C = _krylov_problem(70 + p, p=p, n=24, s=12)
    k, extra = 8, 3
    op = Op(ctx, A, None, C.shape[2], gdt)
    if gdt == dk.DCTK_F32:
        for adj in (0, 1):
            dk.dctk_op_set_path(op.h, adj, 0, 0)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k + extra)
    vt = VT[gdt]
    X = torch.empty(C.shape, dtype=vt, device="cuda:0")
    dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, vt), X, dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, 0.1))
    for _ in range(extra):
        dk.dctk_gkb_step(ctx, ws)
    g = krylov.gkb(op.oracle, C, k + extra, "none")
    r = dk.dctk_krylov_read(ctx, ws, k + extra, dk.DCTK_KRYLOV_GKB)
    ea = rel(r["alpha"][: k + extra + 1], g.alpha[: k + extra + 1])
    eb = rel(r["beta"][: k + extra + 1], g.beta[: k + extra + 1])
    v = torch.empty(C.shape, dtype=vt, device="cuda:0")
    dk.dctk_krylov_copy(ctx, ws, 1, k + extra, v)
    ev = rel(to_np(v), g.V[k + extra])
    say("  alpha", ea, "beta", eb, "V", ev)
    assert r["steps"] == k + extra
    assert ea <= tol and eb <= tol and ev <= 10 * tol
    dk.dctk_krylov_destroy(ws)


def _colour_small_problem():
    w = W.colour_small()
    orc = Operator(w["A"])
    Ch = orc.apply(w["X_true"])
    return w, w["N0"], Ch + w["nu"] * fro(Ch) / fro(w["N0"]) * w["N0"]


@pytest.mark.parametrize("mode", [0, 1])
def test_gk_gcv_matches_oracle(ctx, mode):
    """GCV at k = 12 on the 32 x 32 x 3 colour problem (where the FP64 process is
    stable: a 1e-16 perturbation of C moves alpha_j by < 1e-13): the GCV value at
    the library's lambda equals the oracle's minimum; X equals the oracle's X at
    the library's lambda."""
    say("gcv", mode)
    w, _, C = _colour_small_problem()
    op = Op(ctx, w["A"], None, 32, dk.DCTK_F64)
    k = 12
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    X = torch.empty(C.shape, dtype=F64, device="cuda:0")
    info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(k, dk.DCTK_REORTH_FULL, mode, -1.0))
    gmode = "rect" if mode == 0 else "paper"
    ref = krylov.dc_gk(op.oracle, C, k, lam=None, gcv_mode=gmode, reorth="full")
    g = ref["gkb"]
    sig, Vt, gg = tikhonov.projected_svd(g.bidiagonal(k), g.beta[0])
    f = tikhonov.gcv_rect if mode == 0 else tikhonov.gcv_paper
    gmin = f(sig, gg, ref["lambda"])
    assert f(sig, gg, info.lam) <= gmin * (1.0 + 1e-9)
    assert abs(info.gcv - f(sig, gg, info.lam)) <= 1e-9 * abs(info.gcv)
    at_lam = krylov.dc_gk(op.oracle, C, k, lam=info.lam, reorth="full")
    assert rel(to_np(X), at_lam["X"]) <= 1e-9
    dk.dctk_krylov_destroy(ws)


def test_gk_projected_gcv_every_k(ctx):
    """The DC-GK projected solve (sigma_1 by Sturm counts, GCV from the damped
    rotations, no SVD) at every k from 1 to 12 of one FP64 GKB run on the
    32 x 32 x 3 colour problem, against the oracle's SVD definitions at the
    same k: the GCV value at the library's lambda is the oracle's minimum (to
    1e-9) and equals the oracle's GCV there (to 1e-9); X is the oracle's X at
    the library's lambda; a fixed lambda gives the oracle's X (1e-9)."""
    w, _, C = _colour_small_problem()
    op = Op(ctx, w["A"], None, 32, dk.DCTK_F64)
    kmax = 12
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, kmax)
    X = torch.empty(C.shape, dtype=F64, device="cuda:0")
    dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(kmax, dk.DCTK_REORTH_FULL, 0, -1.0))
    g = krylov.gkb(op.oracle, C, kmax, reorth="full")
    for k in range(1, kmax + 1):
        info = dk.dctk_krylov_project(ctx, ws, k, dk.make_opts(kmax, dk.DCTK_REORTH_FULL, 0, -1.0), X)
        sig, Vt, gg = tikhonov.projected_svd(g.bidiagonal(k), g.beta[0])
        lam_ref, gmin = tikhonov.gcv_minimize(sig, gg, "rect")
        got = tikhonov.gcv_rect(sig, gg, info.lam)
        say("k", k, "lambda", info.lam, lam_ref, "gcv", info.gcv, gmin)
        assert got <= gmin * (1.0 + 1e-9)
        assert abs(info.gcv - got) <= 1e-9 * abs(got)
        ref = krylov.dc_gk(op.oracle, C, k, lam=info.lam, reorth="full")
        assert rel(to_np(X), ref["X"]) <= 1e-9
        dk.dctk_krylov_project(ctx, ws, k, dk.make_opts(kmax, dk.DCTK_REORTH_FULL, 0, 0.03), X)
        ref = krylov.dc_gk(op.oracle, C, k, lam=0.03, reorth="full")
        assert rel(to_np(X), ref["X"]) <= 1e-9
    dk.dctk_krylov_destroy(ws)


@pytest.mark.parametrize("where", ["noise", "middle"])
def test_gk_discrepancy_matches_oracle(ctx, where):
    """lambda by the discrepancy principle (gcv_mode 2) at k = 12 on the
    32 x 32 x 3 colour problem, FP64: the target is 1.05 times the norm of the
    added noise, or the middle of the residuals reachable on the lambda range.
    The library's lambda is the oracle's (1e-8), its projected residual meets
    the target (1e-8, when inside the range), X is the oracle's X at it, and
    dctk_krylov_project gives the same lambda from the stepped workspace."""
    w, N0, C = _colour_small_problem()
    op = Op(ctx, w["A"], None, 32, dk.DCTK_F64)
    k = 12
    g = krylov.gkb(op.oracle, C, k, reorth="full")
    sig, Vt, gg = tikhonov.projected_svd(g.bidiagonal(k), g.beta[0])
    if where == "noise":
        Ch = op.oracle.apply(w["X_true"])
        target = 1.05 * w["nu"] * fro(Ch)
    else:
        r_lo = tikhonov.projected_residual(sig, gg, sig[0] * 1e-8)
        r_hi = tikhonov.projected_residual(sig, gg, sig[0])
        target = np.sqrt(r_lo * r_hi)
    lam_ref, res_ref = tikhonov.discrepancy_lambda(sig, gg, target)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    X = torch.empty(C.shape, dtype=F64, device="cuda:0")
    opts = dk.make_opts(k, dk.DCTK_REORTH_FULL, 2, -1.0, 0.0, target)
    info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, opts)
    say("discrepancy", where, "target", target, "lambda", info.lam, lam_ref, "res", res_ref)
    assert abs(info.lam - lam_ref) <= 1e-8 * lam_ref
    inside = sig[0] * 1e-8 * (1 + 1e-9) < lam_ref < sig[0] * (1 - 1e-9)
    if inside:
        assert abs(tikhonov.projected_residual(sig, gg, info.lam) - target) <= 1e-8 * target
    ref = krylov.dc_gk(op.oracle, C, k, lam=info.lam, reorth="full")
    assert rel(to_np(X), ref["X"]) <= 1e-9
    Xp = torch.empty_like(X)
    ip = dk.dctk_krylov_project(ctx, ws, k, opts, Xp)
    assert ip.lam == info.lam
    assert np.array_equal(to_np(Xp), to_np(X))
    # a non-positive target and DC-GMRES are rejected
    with pytest.raises(dk.DctkError) as e:
        dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(k, dk.DCTK_REORTH_FULL, 2, -1.0, 0.0, 0.0))
    assert e.value.status == dk.DCTK_EINVAL
    wa = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_ARNOLDI, 4)
    with pytest.raises(dk.DctkError) as e:
        dk.dctk_gmres_tik_solve(ctx, wa, to_gpu(C, F64), X, 1, dk.make_opts(4, 0, 2, -1.0, 0.0, target))
    assert e.value.status == dk.DCTK_EINVAL
    dk.dctk_krylov_destroy(wa)
    dk.dctk_krylov_destroy(ws)


@pytest.mark.parametrize("case", ["colour", "random"])
def test_lsqr_lcurve_matches_oracle(ctx, case):
    """LSQR stopped at the L-curve corner (FP64, full reorthogonalisation):
    the library's corner index is the oracle's (curvature of the points from
    least squares on the leading blocks of the oracle's bidiagonal), X is the
    oracle's LSQR iterate at that index (1e-9) and the reported residual norm
    is its residual (1e-9)."""
    if case == "colour":
        w, _, C = _colour_small_problem()
        A, s_ = w["A"], 32
        K = 12
    else:
        A, _, C = _krylov_problem(9)
        s_ = C.shape[2]
        K = 10
    op = Op(ctx, A, None, s_, dk.DCTK_F64)
    g = krylov.gkb(op.oracle, C, K, reorth="full")
    Kt = g.steps
    res, nrm = tikhonov.lcurve_points(g.bidiagonal(Kt), g.beta[0], Kt)
    k_ref = tikhonov.lcurve_corner(res, nrm)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, K)
    X = torch.empty((C.shape[0], A.shape[2], C.shape[2]), dtype=F64, device="cuda:0")
    info, k_opt = dk.dctk_lsqr_lcurve_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(K, dk.DCTK_REORTH_FULL, 0, 0.0))
    say("lcurve", case, "k_opt", k_opt, k_ref, "res", info.resnorm, res[k_ref - 1])
    assert k_opt == k_ref
    ref = krylov.dc_lsqr(op.oracle, C, k_ref, reorth="full")
    assert rel(to_np(X), ref["X"]) <= 1e-9
    assert abs(info.resnorm - res[k_ref - 1]) <= 1e-9 * res[k_ref - 1]
    dk.dctk_krylov_destroy(ws)


@pytest.mark.parametrize("lam", [0.05, -1.0])
def test_gk_folded_updates_match_oracle(ctx, lam):
    """Tikhonov solve (no reorthogonalisation, both products fused), where each
    LSQR update runs inside the next forward product and the last one in its
    own kernel: the Golub-Kahan scalars, the last basis vectors U_{k+1},
    V_{k+1} and X match the oracle's process on the 32 x 32 x 3 colour problem
    (fixed lambda: X to 1e-9; GCV: the GCV value at the library's lambda is the
    oracle's minimum and X is the oracle's X at that lambda)."""
    say("folded", lam)
    w, _, C = _colour_small_problem()
    k = 12
    op = Op(ctx, w["A"], None, 32, dk.DCTK_F64)
    for adj in (0, 1):
        dk.dctk_op_set_path(op.h, adj, 1, 16)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    X = torch.empty(C.shape, dtype=F64, device="cuda:0")
    info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, lam))
    g = krylov.gkb(op.oracle, C, k, "none")
    r = dk.dctk_krylov_read(ctx, ws, k, dk.DCTK_KRYLOV_GKB)
    assert r["steps"] == k and r["status"] == 0 and info.iters == k
    assert rel(r["alpha"][: k + 1], g.alpha[: k + 1]) <= 1e-9
    assert rel(r["beta"][: k + 1], g.beta[: k + 1]) <= 1e-9
    v = torch.empty(C.shape, dtype=F64, device="cuda:0")
    dk.dctk_krylov_copy(ctx, ws, 1, k, v)
    assert rel(to_np(v), g.V[k]) <= 1e-8
    dk.dctk_krylov_copy(ctx, ws, 0, k, v)
    assert rel(to_np(v), g.U[k]) <= 1e-8
    if lam > 0:
        ref = krylov.dc_gk(op.oracle, C, k, lam=lam, reorth="none")
        assert rel(to_np(X), ref["X"]) <= 1e-9
    else:
        ref = krylov.dc_gk(op.oracle, C, k, lam=None, gcv_mode="rect", reorth="none")
        sig, _, gg = tikhonov.projected_svd(ref["gkb"].bidiagonal(k), ref["gkb"].beta[0])
        assert tikhonov.gcv_rect(sig, gg, info.lam) <= tikhonov.gcv_rect(sig, gg, ref["lambda"]) * (1.0 + 1e-9)
        at_lam = krylov.dc_gk(op.oracle, C, k, lam=info.lam, reorth="none")
        assert rel(to_np(X), at_lam["X"]) <= 1e-9
    dk.dctk_krylov_destroy(ws)


def test_folded_and_three_kernel_solves_agree(ctx):
    """FP32 Tikhonov solve (GCV, no reorthogonalisation) through the folded-
    update path (fused products) and through the three-kernel products
    (separate LSQR updates), at k = 12 on the 32 x 32 x 3 colour problem.
    The two paths round differently, so they are held to each other (X within
    2e-3) and to the FP64 oracle's restoration error (within 3%), not bit for
    bit.  (Past k = 12 this problem's FP32 process drifts on its own: rounding
    only the basis vectors to FP32 in the FP64 oracle already costs 8% of
    restoration error at k = 16.)"""
    w, _, C = _colour_small_problem()
    k = 12
    ref = krylov.dc_gk(Operator(w["A"]), C, k, lam=None, gcv_mode="rect", reorth="none")
    e_ref = metrics.relative_error(w["X_true"], ref["X"])
    xs = []
    for path in (1, 0):
        op = Op(ctx, w["A"], None, 32, dk.DCTK_F32)
        for adj in (0, 1):
            dk.dctk_op_set_path(op.h, adj, path, 16 if path else 32)
        ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
        X = torch.empty(C.shape, dtype=F32, device="cuda:0")
        info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F32), X, dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0))
        xs.append(to_np(X).astype(np.float64))
        e = metrics.relative_error(w["X_true"], xs[-1])
        say("path", path, "relerr", e, "oracle", e_ref, "lambda", info.lam, ref["lambda"])
        assert e <= 1.03 * e_ref
        dk.dctk_krylov_destroy(ws)
    assert rel(xs[0], xs[1]) <= 2e-3


def test_enqueued_solves_match_synchronous_solve(ctx):
    """dctk_lsqr_tik_solve with info NULL only enqueues: three solves back to
    back (different right-hand sides into different outputs, no read-back in
    between) give bit for bit the X, lambda and steps of the same solves run
    one at a time with their info read back."""
    w, _, C = _colour_small_problem()
    k = 12
    op = Op(ctx, w["A"], None, 32, dk.DCTK_F32)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0)
    Cs = [to_gpu(C * (1.0 + 0.1 * i), F32) for i in range(3)]
    ref = []
    for Ci in Cs:
        X = torch.empty(C.shape, dtype=F32, device="cuda:0")
        info = dk.dctk_lsqr_tik_solve(ctx, ws, Ci, X, opts)
        ref.append((to_np(X), info.lam, info.iters))
    outs = [torch.empty(C.shape, dtype=F32, device="cuda:0") for _ in Cs]
    for Ci, Xi in zip(Cs, outs):
        assert dk.dctk_lsqr_tik_solve(ctx, ws, Ci, Xi, opts, info=False) is None
    dk.dctk_synchronize(ctx)
    for (xr, lam, it), Xi in zip(ref, outs):
        assert np.array_equal(to_np(Xi), xr)
    # the workspace holds the last solve's state: its info matches the last reference
    info = dk.dctk_lsqr_tik_solve(ctx, ws, Cs[-1], outs[-1], opts)
    assert info.lam == ref[-1][1] and info.iters == ref[-1][2]
    dk.dctk_krylov_destroy(ws)


def test_solves_on_two_streams_match_one_stream(ctx):
    """Independent enqueue-only solves alternating over two contexts on two
    streams (each with its own operator and workspace) give bit for bit the X
    of the same solve on the default context."""
    w, _, C = _colour_small_problem()
    k = 12
    opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0)
    Cg = to_gpu(C, F32)
    op = Op(ctx, w["A"], None, 32, dk.DCTK_F32)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    Xr = torch.empty(C.shape, dtype=F32, device="cuda:0")
    dk.dctk_lsqr_tik_solve(ctx, ws, Cg, Xr, opts)
    dk.dctk_krylov_destroy(ws)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ctxs = [dk.dctk_create(0, st) for st in streams]
    A = torch.from_numpy(w["A"]).to("cuda:0")
    ops = [dk.dctk_op_create(c, dk.DCTK_TUBE_TH, dk.DCTK_F32, A, 32) for c in ctxs]
    wss = [dk.dctk_krylov_create(c, o, dk.DCTK_KRYLOV_GKB, k) for c, o in zip(ctxs, ops)]
    Xs = [torch.empty(C.shape, dtype=F32, device="cuda:0") for _ in range(4)]
    torch.cuda.synchronize()
    for i in range(4):
        j = i % 2
        dk.dctk_lsqr_tik_solve(ctxs[j], wss[j], Cg, Xs[i], opts, info=False)
    torch.cuda.synchronize()
    for Xi in Xs:
        assert torch.equal(Xi, Xr)
    for j in range(2):
        dk.dctk_krylov_destroy(wss[j])
        dk.dctk_op_destroy(ops[j])
        dk.dctk_destroy(ctxs[j])


def test_gk_gcv_20_steps_restoration_level(ctx):
    """k = 20 on the same problem: past step ~15 rounding is amplified by the
    process itself (oracle vs oracle with C perturbed by 1e-16: alpha moves 3%,
    X moves 5e-6), so X is compared at 1e-4 and the restoration error at 1.001x."""
    w, _, C = _colour_small_problem()
    op = Op(ctx, w["A"], None, 32, dk.DCTK_F64)
    k = 20
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    X = torch.empty(C.shape, dtype=F64, device="cuda:0")
    dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(k, dk.DCTK_REORTH_FULL, 0, -1.0))
    ref = krylov.dc_gk(op.oracle, C, k, lam=None, reorth="full")
    Xg = to_np(X)
    assert rel(Xg, ref["X"]) <= 1e-4
    assert metrics.relative_error(w["X_true"], Xg) <= 1.001 * metrics.relative_error(w["X_true"], ref["X"])
    dk.dctk_krylov_destroy(ws)


@pytest.mark.parametrize("ortho", [dk.DCTK_ORTHO_MGS, dk.DCTK_ORTHO_CGS2])
@pytest.mark.parametrize("lam", [0.0, 0.2, -1.0])
def test_gmres_matches_oracle(ctx, ortho, lam):
    say("gmres", ortho, lam)
    A, _, C = _krylov_problem(11)
    m, cycles = 8, 3
    op = Op(ctx, A, None, C.shape[2], dk.DCTK_F64)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_ARNOLDI, m, ortho)
    X0 = 0.1 * np.random.default_rng(1).standard_normal(C.shape)
    X = to_gpu(X0, F64)
    info = dk.dctk_gmres_tik_solve(ctx, ws, to_gpu(C, F64), X, cycles, dk.make_opts(m, 0, 0, lam))
    ref = krylov.dc_gmres(op.oracle, C, X0, m, cycles, lam=None if lam < 0 else lam,
                          ortho="mgs" if ortho == dk.DCTK_ORTHO_MGS else "cgs2")
    assert info.cycles == cycles
    tol = 1e-9 if lam >= 0 else 1e-6   # GCV: lambda agrees to the minimiser's accuracy
    assert rel(to_np(X), ref["X"]) <= tol
    assert abs(info.resnorm - ref["resnorm"]) <= 1e-6 * ref["resnorm"]
    dk.dctk_krylov_destroy(ws)


def test_breakdown_identity_operator(ctx):
    """A = e_1 (x) I: breakdown after one step, exact recovery (X = C)."""
    p, n, s = 3, 16, 8
    A = np.zeros((p, n, n))
    A[0] = np.eye(n)
    C = np.random.default_rng(2).standard_normal((p, n, s))
    op = Op(ctx, A, None, s, dk.DCTK_F64)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, 5)
    X = torch.empty(C.shape, dtype=F64, device="cuda:0")
    info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(5, 0, 0, 0.0))
    assert info.status == dk.DCTK_BREAKDOWN and info.iters == 1
    assert rel(to_np(X), C) <= 1e-13
    # GK with GCV on the breakdown also recovers C
    info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(5, 0, 0, 1e-12))
    assert rel(to_np(X), C) <= 1e-10
    dk.dctk_krylov_destroy(ws)
    wa = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_ARNOLDI, 4)
    X.zero_()
    info = dk.dctk_gmres_tik_solve(ctx, wa, to_gpu(C, F64), X, 2, dk.make_opts(4, 0, 0, 0.0))
    assert info.status == dk.DCTK_BREAKDOWN
    assert rel(to_np(X), C) <= 1e-13
    dk.dctk_krylov_destroy(wa)


def test_zero_rhs(ctx):
    A, _, C = _krylov_problem(13)
    op = Op(ctx, A, None, C.shape[2], dk.DCTK_F32)
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, 4)
    X = torch.full(C.shape, 7.0, dtype=F32, device="cuda:0")
    info = dk.dctk_lsqr_tik_solve(ctx, ws, torch.zeros(C.shape, dtype=F32, device="cuda:0"), X,
                                  dk.make_opts(4, 0, 0, -1.0))
    assert info.status == dk.DCTK_BREAKDOWN and info.iters == 0
    assert float(X.abs().max()) == 0.0
    dk.dctk_krylov_destroy(ws)


# ---------------------------------------------------------- workload sizes

@pytest.mark.parametrize("gdt", [dk.DCTK_F32, dk.DCTK_BF16])
def test_colour_256_restoration(ctx, gdt):
    """The benchmarked solve (256 x 256 x 3, 40 GKB steps, GCV): restoration error
    within 1.05x of the FP64 oracle's on the same input; c-product parity at size."""
    say("colour256", gdt)
    w = W.colour_256()
    orc = Operator(w["A"])
    Ch = orc.apply(w["X_true"])
    C = Ch + w["nu"] * fro(Ch) / fro(w["N0"]) * w["N0"]
    k = w["iters"]
    ref = krylov.dc_gk(orc, C, k, lam=None, gcv_mode="rect", reorth="none")
    e_ref = metrics.relative_error(w["X_true"], ref["X"])
    op = Op(ctx, w["A"], None, 256, gdt)
    # product parity at full size
    Y = torch.empty(C.shape, dtype=F32, device="cuda:0")
    dk.dctk_cprod(ctx, op.h, 1.0, to_gpu(w["X_true"], F32), 0.0, Y)
    assert_product(to_np(Y), gdt, w["A"], None, w["X_true"], Ch, label="colour256")
    ws = dk.dctk_krylov_create(ctx, op.h, dk.DCTK_KRYLOV_GKB, k)
    X = torch.empty(C.shape, dtype=F32, device="cuda:0")
    info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F32), X, dk.make_opts(k, 0, 0, -1.0))
    e = metrics.relative_error(w["X_true"], to_np(X))
    say("  relerr gpu", e, "oracle", e_ref, "lambda", info.lam, ref["lambda"])
    assert info.iters == k
    assert e <= 1.05 * e_ref
    dk.dctk_krylov_destroy(ws)
