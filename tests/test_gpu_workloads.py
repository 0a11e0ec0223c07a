"""The larger workloads at their full sizes, against the FP64 oracle.

Video: two-sided A *c X *c B, 256 x 256 x 32 frames: the whole product and
its adjoint element-wise (FP32 to 1e-5; FP16 to the rounding model of the
16-bit GEMM mode), and DC-GMRES with Tikhonov/GCV (40 Arnoldi steps) with
restoration error within 1.05x of the oracle's on the same input.

Hyperspectral-like: 512 x 512 x 64, band-dependent blur: the whole product
and adjoint element-wise (FP32 to 1e-5; BF16 to the rounding model and to
the roundoff bound of its operands), DC-GK (40 GKB steps, GCV) in FP32 and
BF16 with restoration error within 1.05x of a full FP64 oracle solve of the
same C, and the FP32 LSQR iterate's residual identity |phibar_{k+1}| =
||C - M(X_k)|| (Algorithm 6), the right side evaluated by the oracle.

Paper-shaped (Sec. 4, Tables 1 and 3): two-sided colour deblurring with the
A_color tube, sigma = 4, r = 6.  At 256 x 256 x 3 DC-GMRES(10) (10 cycles),
DC-GK (15 steps) and DC-LSQR (14 steps) in FP64 and FP32 within 1.05x of the
oracle's restoration error; at 1024 x 1024 x 3 one product and one adjoint
element-wise.

Every C here is formed by the oracle (FP64) and handed to the GPU.
"""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, metrics
from oracle import tube as otube
from oracle.cprod import Operator, fro
from tests import rounding_model as RM
from tests.gpu_util import rel, say, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2103_11847_amd as dk  # noqa: E402

F64, F32 = torch.float64, torch.float32
KIND = {dk.DCTK_BF16: "bf16", dk.DCTK_F16: "f16"}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dk.dctk_create(0)
    yield c
    dk.dctk_synchronize(c)
    dk.dctk_destroy(c)


def _noisy(orc, w):
    Ch = orc.apply(w["X_true"])
    return Ch + w["nu"] * fro(Ch) / fro(w["N0"]) * w["N0"]


def _check_products(ctx, op, gdt, w, orc, X, Yin, label, bound_exact=False):
    """Product of X and adjoint of Yin on the GPU against the oracle, element-wise."""
    p = X.shape[0]
    A, B = w["A"], w.get("B")
    L = otube.transform_matrix(p, "th")
    vt = F64 if gdt == dk.DCTK_F64 else F32
    out = {}
    for adj, inp in ((False, X), (True, Yin)):
        rows = A.shape[2] if adj else A.shape[1]
        Yg = torch.empty((p, rows, inp.shape[2]), dtype=vt, device="cuda:0")
        fn = dk.dctk_cprod_T if adj else dk.dctk_cprod
        fn(ctx, op, 1.0, to_gpu(inp, vt), 0.0, Yg)
        got = to_np(Yg)
        del Yg
        exact = orc.adjoint(inp) if adj else orc.apply(inp)
        if gdt in (dk.DCTK_F64, dk.DCTK_F32):
            e = rel(got, exact)
            tol = 1e-10 if gdt == dk.DCTK_F64 else 1e-5
            say(label, "adjoint" if adj else "product", "rel", e, "tol", tol)
            assert e <= tol
            out[adj] = e
            continue
        kind = KIND[gdt]
        gap, e, e_model = RM.check_lowp(got, A, B, L, inp, kind, exact, adj)
        say(label, "adjoint" if adj else "product", kind, "gap to rounding model", gap,
            "rel", e, "model rel", e_model)
        assert gap <= RM.MODEL_TOL[kind]
        assert e <= 1.25 * e_model
        if bound_exact:
            b = RM.roundoff_bound(A, B, L, inp, kind, adj) / np.linalg.norm(exact.ravel())
            say(label, "  roundoff bound", b)
            assert e <= b
        out[adj] = e
    return out


# ------------------------------------------------------------------- video

@pytest.fixture(scope="module")
def video(ctx):
    w = W.video_256()
    orc = Operator(w["A"], w["B"])
    C = _noisy(orc, w)
    ref = krylov.dc_gmres(orc, C, np.zeros_like(C), 40, 1, lam=None)
    e_ref = metrics.relative_error(w["X_true"], ref["X"])
    say("video oracle relerr", e_ref, "lambda", ref["lambdas"])
    return w, orc, C, e_ref


@pytest.mark.parametrize("gdt", [dk.DCTK_F32, dk.DCTK_F16])
def test_video_two_sided_gmres(ctx, video, gdt):
    w, orc, C, e_ref = video
    p, n, s = w["X_true"].shape
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(w["A"], F64), s, to_gpu(w["B"], F64))
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_ARNOLDI, 40)
    try:
        rng = np.random.default_rng(31)
        _check_products(ctx, op, gdt, w, orc, w["X_true"], rng.standard_normal((p, n, s)), "video")
        X = torch.zeros((p, n, s), dtype=F32, device="cuda:0")
        info = dk.dctk_gmres_tik_solve(ctx, ws, to_gpu(C, F32), X, 1, dk.make_opts(40, 0, 0, -1.0))
        e = metrics.relative_error(w["X_true"], to_np(X))
        say("video gmres", gdt, "relerr", e, "oracle", e_ref, "lambda", info.lam, "steps", info.iters)
        assert info.iters == 40
        assert e <= 1.05 * e_ref
    finally:
        torch.cuda.synchronize()
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)


# ---------------------------------------------------- hyperspectral 512 x 512 x 64

@pytest.fixture(scope="module")
def hyper(ctx):
    """The 512 x 512 x 64 problem, its C from the oracle and a full FP64 oracle
    DC-GK solve (40 GKB steps, GCV) of that C."""
    w = W.hyperspectral(0)
    orc = Operator(w["A"])
    C = _noisy(orc, w)
    ref = krylov.dc_gk(orc, C, 40, lam=None, gcv_mode="rect", reorth="none")
    e_ref = metrics.relative_error(w["X_true"], ref["X"])
    say("hyper512 oracle relerr", e_ref, "lambda", ref["lambda"])
    return w, orc, C, e_ref, ref["lambda"]


@pytest.mark.parametrize("gdt", [dk.DCTK_F32, dk.DCTK_BF16])
def test_hyperspectral_512_product_and_adjoint(ctx, hyper, gdt):
    """Every output element of one product (of X_true) and one adjoint (of C)."""
    w, orc, C, _, _ = hyper
    s = w["X_true"].shape[2]
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(w["A"], F64), s)
    try:
        _check_products(ctx, op, gdt, w, orc, w["X_true"], C, "hyper512", bound_exact=True)
    finally:
        torch.cuda.synchronize()
        dk.dctk_op_destroy(op)


@pytest.mark.parametrize("gdt", [dk.DCTK_F32, dk.DCTK_BF16])
def test_hyperspectral_512_restoration(ctx, hyper, gdt):
    """DC-GK, 40 GKB steps, lambda by GCV: restoration error within 1.05x of the
    FP64 oracle's solve of the same C."""
    w, orc, C, e_ref, lam_ref = hyper
    p, n, s = w["X_true"].shape
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(w["A"], F64), s)
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, 40)
    try:
        X = torch.empty((p, n, s), dtype=F32, device="cuda:0")
        info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F32), X, dk.make_opts(40, 0, 0, -1.0))
        e = metrics.relative_error(w["X_true"], to_np(X))
        say("hyper512 GCV", gdt, "relerr", e, "oracle", e_ref, "ratio", e / e_ref, "lambda", info.lam, lam_ref)
        assert info.iters == 40
        assert e <= 1.05 * e_ref
    finally:
        torch.cuda.synchronize()
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)


def test_hyperspectral_512_lsqr_residual_identity(ctx, hyper):
    """FP32 DC-LSQR (lambda = 0, 40 steps): the recurrence's |phibar_{k+1}|
    equals the true residual ||C - M(X_k)||, M applied by the oracle in FP64,
    to 2e-3 of the residual (FP32 vectors and products over 40 steps)."""
    w, orc, C, _, _ = hyper
    p, n, s = w["X_true"].shape
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F32, to_gpu(w["A"], F64), s)
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, 40)
    try:
        X = torch.empty((p, n, s), dtype=F32, device="cuda:0")
        info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F32), X, dk.make_opts(40, 0, 0, 0.0))
        Xk = to_np(X)
        res = fro(C - orc.apply(Xk))
        say("hyper512 LSQR |phibar|", info.resnorm, "true residual", res, "||C||", fro(C))
        assert abs(info.resnorm - res) <= 2e-3 * res
    finally:
        torch.cuda.synchronize()
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)


@pytest.mark.parametrize("gdt", [dk.DCTK_F32, dk.DCTK_BF16])
def test_hyperspectral_128_restoration(ctx, gdt):
    """The same family at 128 x 128 x 64 (another instance)."""
    w = W.hyperspectral(1, n=128, p=64)
    orc = Operator(w["A"])
    C = _noisy(orc, w)
    ref = krylov.dc_gk(orc, C, 40, lam=None, gcv_mode="rect", reorth="none")
    e_ref = metrics.relative_error(w["X_true"], ref["X"])
    p, n, s = w["X_true"].shape
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(w["A"], F64), s)
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, 40)
    try:
        X = torch.empty((p, n, s), dtype=F32, device="cuda:0")
        info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F32), X, dk.make_opts(40, 0, 0, -1.0))
        e = metrics.relative_error(w["X_true"], to_np(X))
        say("hyper 128", gdt, "relerr", e, "oracle", e_ref, "lambda", info.lam, ref["lambda"])
        assert e <= 1.05 * e_ref
    finally:
        torch.cuda.synchronize()
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)


# ----------------------------------------------------------- paper-shaped runs

# Sec. 4, Table 1 (nu = 1e-3): DC-GMRES(10) with 10 restart cycles, DC-GK with
# mmax = 15, DC-LSQR with k_opt = 14.
PAPER_256 = {"gmres": 10, "gk": 15, "lsqr": 14}


@pytest.fixture(scope="module")
def paper256(ctx):
    w = W.paper_shaped(256, 1e-3)
    orc = Operator(w["A"], w["B"])
    C = _noisy(orc, w)
    refs = {
        "gmres": krylov.dc_gmres(orc, C, np.zeros_like(C), 10, PAPER_256["gmres"], lam=None)["X"],
        "gk": krylov.dc_gk(orc, C, PAPER_256["gk"], lam=None)["X"],
        "lsqr": krylov.dc_lsqr(orc, C, PAPER_256["lsqr"])["X"],
    }
    errs = {k: metrics.relative_error(w["X_true"], v) for k, v in refs.items()}
    say("paper 256 oracle relerr", errs)
    return w, orc, C, refs, errs


@pytest.mark.parametrize("gdt", [dk.DCTK_F64, dk.DCTK_F32])
@pytest.mark.parametrize("meth", ["gmres", "gk", "lsqr"])
def test_paper_shaped_256_solves(ctx, paper256, gdt, meth):
    w, orc, C, refs, errs = paper256
    p, n, s = w["X_true"].shape
    vt = F64 if gdt == dk.DCTK_F64 else F32
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(w["A"], F64), s, to_gpu(w["B"], F64))
    its = PAPER_256[meth]
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_ARNOLDI if meth == "gmres" else dk.DCTK_KRYLOV_GKB,
                               10 if meth == "gmres" else its)
    try:
        X = torch.zeros((p, n, s), dtype=vt, device="cuda:0")
        if meth == "gmres":
            info = dk.dctk_gmres_tik_solve(ctx, ws, to_gpu(C, vt), X, its, dk.make_opts(10, 0, 0, -1.0))
        else:
            info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, vt), X,
                                          dk.make_opts(its, 0, 0, -1.0 if meth == "gk" else 0.0))
        Xg = to_np(X)
        e = metrics.relative_error(w["X_true"], Xg)
        say("paper256", meth, gdt, "relerr", e, "oracle", errs[meth], "X gap", rel(Xg, refs[meth]),
            "lambda", info.lam)
        assert e <= 1.05 * errs[meth]
        if gdt == dk.DCTK_F64:
            # These short runs are stable: a 1e-15 change of C moves the oracle's X by
            # <= 3e-10.  With lambda = 0 the FP64 iterate is the oracle's; with GCV the
            # two minimisers agree to ~1e-5 in lambda (the GCV minimum is flat) and X
            # moves by 3.9e-3 times the relative change of lambda.
            assert rel(Xg, refs[meth]) <= (1e-8 if meth == "lsqr" else 1e-6)
    finally:
        torch.cuda.synchronize()
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)


@pytest.mark.parametrize("gdt", [dk.DCTK_F64, dk.DCTK_F32])
def test_paper_shaped_1024_product_and_adjoint(ctx, gdt):
    w = W.paper_shaped(1024, 1e-3)
    orc = Operator(w["A"], w["B"])
    s = w["X_true"].shape[2]
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(w["A"], F64), s, to_gpu(w["B"], F64))
    try:
        Y = np.random.default_rng(37).standard_normal(w["X_true"].shape)
        _check_products(ctx, op, gdt, w, orc, w["X_true"], Y, "paper1024")
    finally:
        torch.cuda.synchronize()
        dk.dctk_op_destroy(op)
