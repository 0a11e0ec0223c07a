"""The larger workloads at their full sizes.

Video: two-sided A *c X *c B, 256 x 256 x 32 frames, DC-GMRES with Tikhonov/GCV
(40 Arnoldi steps, one cycle) with FP32 and FP16 slice GEMMs: restoration error
within 1.05x of the FP64 oracle's on the same input.

Hyperspectral: 512 x 512 x 64 with band-dependent blur, DC-GK (40 GKB steps,
GCV), FP32 and BF16 slice GEMMs.  At this size the oracle computes sampled
output tubes of one product (each from its own tube transforms and slice
rows), and the solve is checked through the LSQR residual identity
|phibar_{k+1}| = ||C - M(X_k)|| (Algorithm 6 / Proposition 3.2), which holds
at any size (to the slices' rounding); the restoration error
is compared with the oracle's on the same problem family at 128 x 128 x 64.
"""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, metrics
from oracle import tube as otube
from oracle.cprod import Operator, fro
from tests.gpu_util import rel, say, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2103_11847_amd as dk  # noqa: E402

F64, F32 = torch.float64, torch.float32


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
        # product parity at full size
        Y = torch.empty((p, n, s), dtype=F32, device="cuda:0")
        dk.dctk_cprod(ctx, op, 1.0, to_gpu(w["X_true"], F32), 0.0, Y)
        Yref = orc.apply(w["X_true"])
        bound = 1e-5 if gdt == dk.DCTK_F32 else 2 * 8.0 * 2.0 ** -11 * np.sqrt(p)
        say("video cprod rel", rel(to_np(Y), Yref), "bound", bound)
        assert rel(to_np(Y), Yref) <= bound
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


def _sampled_tubes(A, X, L, Linv, pts):
    """Output tubes Y(i, j, :) of A *c X from the transform formula, one tube at a time."""
    Ah = (L @ A.reshape(A.shape[0], -1)).reshape(A.shape)   # A~_k, every slice
    out = {}
    for (i, j) in pts:
        Xh_col = L @ X[:, :, j]                   # X~_k(:, j) for every k
        yh = np.array([Ah[k, i, :] @ Xh_col[k] for k in range(A.shape[0])])
        out[(i, j)] = Linv @ yh
    return out


@pytest.mark.parametrize("gdt,bound", [(dk.DCTK_F32, 1e-5), (dk.DCTK_BF16, 8.0 * 2.0 ** -8)])
def test_hyperspectral_512_product_and_residual_identity(ctx, gdt, bound):
    w = W.hyperspectral(0)
    p, n, s = w["X_true"].shape
    A64 = to_gpu(w["A"], F64)
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, A64, s)
    op64 = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F64, A64, s)
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, 40)
    try:
        # sampled output tubes of one product against the oracle's transform formula
        Xt = to_gpu(w["X_true"], F32)
        Y = torch.empty((p, n, s), dtype=F32, device="cuda:0")
        dk.dctk_cprod(ctx, op, 1.0, Xt, 0.0, Y)
        L = otube.transform_matrix(p, "th")
        rng = np.random.default_rng(4)
        pts = [(int(rng.integers(0, n)), int(rng.integers(0, s))) for _ in range(12)] + [(0, 0), (n - 1, s - 1)]
        ref = _sampled_tubes(w["A"], w["X_true"], L, np.linalg.inv(L), pts)
        Yn = to_np(Y)
        got = np.stack([Yn[:, i, j] for (i, j) in pts])
        want = np.stack([ref[q] for q in pts])
        say("hyper sampled tubes rel", gdt, rel(got, want), "bound", bound)
        assert rel(got, want) <= bound
        # the solve: C from the library's FP64 product (an input, not an expected value)
        Ch = torch.empty((p, n, s), dtype=F64, device="cuda:0")
        dk.dctk_cprod(ctx, op64, 1.0, to_gpu(w["X_true"], F64), 0.0, Ch)
        N0 = to_gpu(w["N0"], F64)
        C = (Ch + w["nu"] * torch.linalg.norm(Ch) / torch.linalg.norm(N0) * N0).to(F32).contiguous()
        X = torch.empty((p, n, s), dtype=F32, device="cuda:0")
        info = dk.dctk_lsqr_tik_solve(ctx, ws, C, X, dk.make_opts(40, 0, 0, 0.0))   # LSQR iterate
        # the identity holds for the operator the solver applied.  With FP32 slices that
        # is the FP64 operator up to FP32 rounding.  With BF16 slices every product also
        # rounds its transformed input to bfloat16, so M(X_k) differs from the
        # combination of the products the recurrence saw by up to ~u ||C||, u = 2^-8.
        MX = torch.empty((p, n, s), dtype=F64, device="cuda:0")
        dk.dctk_cprod(ctx, op64, 1.0, X.double().contiguous(), 0.0, MX)
        res = float(torch.linalg.norm(C.double() - MX))
        cn = float(torch.linalg.norm(C.double()))
        tol = 2e-3 * res if gdt == dk.DCTK_F32 else 4.0 * 2.0 ** -8 * cn
        say("hyper LSQR residual identity", info.resnorm, res, "||C||", cn, "tol", tol)
        assert abs(info.resnorm - res) <= tol
        infog = dk.dctk_lsqr_tik_solve(ctx, ws, C, X, dk.make_opts(40, 0, 0, -1.0))
        e = float(torch.linalg.norm(X.double() - to_gpu(w["X_true"], F64)) / torch.linalg.norm(to_gpu(w["X_true"], F64)))
        say("hyper 512 GCV relerr", gdt, e, "lambda", infog.lam)
        assert np.isfinite(e) and e < 1.0
    finally:
        torch.cuda.synchronize()
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)
        dk.dctk_op_destroy(op64)


@pytest.mark.parametrize("gdt", [dk.DCTK_F32, dk.DCTK_BF16])
def test_hyperspectral_128_restoration(ctx, gdt):
    """The same family at 128 x 128 x 64, where the oracle runs the whole solve."""
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
