"""Operators with tubes longer than 64 (power-of-two p from 128 to 2048, the
O(p log p) transform of Sec. 1 / Sec. 2.1 inside every product) against the
FP64 oracle, whose operator applies the dense p x p matrices.

Tolerances (relative Frobenius):
  * FP64 products: 1e-13 p.  The oracle's dense M carries about 25 p u of
    relative error (it is formed as W^{-1}(C_n(I+Z))); the fast steps are the
    more accurate side, and a product applies two transforms.
  * FP32 products: 3 (1e-6 + 8e-9 p).  One FP32 fast transform is within
    1e-6 + 8e-9 p of the exact one (the factor D^{-1}, up to 2p/pi, scales the
    FFT's rounding in the last rows); a product applies two of them and the
    slice GEMM adds a few u.
  * BF16 / FP16 GEMM modes: the rounding model of the 16-bit operands (as for
    short tubes), with the gap allowed to grow by what the larger FP32
    transform error eps_T = 1e-6 + 8e-9 p does to the 16-bit roundings.  An
    operand element x whose FP32 value is off by d rounds differently from
    the model's only when a rounding boundary lies between them, with
    probability <= |d| / ulp, and then by one ulp <= 2u|x| (u the 16-bit unit
    roundoff); summed over elements, E||change||^2 <= 2u sum |d||x| <=
    2 u eps_T ||x||^2.  So the gap may exceed the short-tube allowance by
    sqrt(2 u eps_T) (taken 3x) plus eps_T of the output transform.  The
    error against the exact product stays within 1.25x the model's.
  * Solves: the FP64 process with full reorthogonalisation equals the
    oracle's to 1e-9; FP32 / BF16 DC-GK with GCV restores within 1.05x of the
    FP64 oracle's error; DC-GMRES restarts match the oracle to 1e-9 (FP64,
    fixed lambda); a batch of long-tube solves equals the single solves bit
    for bit.
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
VT = {dk.DCTK_F64: F64, dk.DCTK_F32: F32, dk.DCTK_BF16: F32, dk.DCTK_F16: F32}
LOWP = {dk.DCTK_BF16: "bf16", dk.DCTK_F16: "f16"}
TUBES = {dk.DCTK_TUBE_TH: "th", dk.DCTK_TUBE_DCT2: "dct2"}


def tol_prod(gdt, p):
    return 1e-13 * p if gdt == dk.DCTK_F64 else 3.0 * (1e-6 + 8e-9 * p)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dk.dctk_create(0)
    yield c
    dk.dctk_synchronize(c)
    dk.dctk_destroy(c)


def _check(got, gdt, A, B, X, exact, adjoint, tube, label):
    p = A.shape[0]
    if gdt not in LOWP:
        e = rel(got, exact)
        say(label, "rel", e, "tol", tol_prod(gdt, p))
        assert e <= tol_prod(gdt, p), (label, e)
        return
    kind = LOWP[gdt]
    L = otube.transform_matrix(p, TUBES[tube])
    gap, e, e_model = RM.check_lowp(got, A, B, L, X, kind, exact, adjoint)
    eps_t = 1e-6 + 8e-9 * p
    gap_tol = RM.MODEL_TOL[kind] + 3.0 * np.sqrt(2.0 * RM.UNIT[kind] * eps_t) + eps_t
    say(label, kind, "gap", gap, "tol", gap_tol, "rel", e, "model", e_model)
    assert gap <= gap_tol, (label, gap)
    assert e <= 1.25 * e_model, (label, e, e_model)


# (p, n1, n2, s): ragged slices at p = 128 and 256; p = 2048 (one tube per
# FP64 workgroup, two per FP32 one); p = 128 with 65536 positions per slice,
# so every resident workgroup walks several blocks of tubes
SHAPES = [(128, 24, 20, 7), (256, 9, 13, 5), (2048, 5, 4, 3), (128, 256, 256, 256)]


@pytest.mark.parametrize("gdt", [dk.DCTK_F64, dk.DCTK_F32, dk.DCTK_BF16, dk.DCTK_F16])
@pytest.mark.parametrize("two_sided", [False, True])
@pytest.mark.parametrize("shape", SHAPES)
def test_long_tube_product_and_adjoint(ctx, gdt, two_sided, shape):
    p, n1, n2, s = shape
    if n1 >= 256 and (two_sided or gdt == dk.DCTK_F16):
        pytest.skip("the large-count case runs one-sided FP64, FP32 and BF16")
    rng = np.random.default_rng(p + n1 + (3 if two_sided else 0))
    A = rng.standard_normal((p, n1, n2))
    B = rng.standard_normal((p, s, s)) if two_sided else None
    X = rng.standard_normal((p, n2, s))
    Y = rng.standard_normal((p, n1, s))
    orc = Operator(A, B)
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(A, F64), s, None if B is None else to_gpu(B, F64))
    try:
        info = dk.dctk_op_info(op)
        assert (info["p"], info["n1"], info["n2"], info["s"]) == (p, n1, n2, s)
        vt = VT[gdt]
        print("long tube product", shape, gdt, two_sided, flush=True)
        Yg = torch.empty((p, n1, s), dtype=vt, device="cuda:0")
        dk.dctk_cprod(ctx, op, 1.0, to_gpu(X, vt), 0.0, Yg)
        _check(to_np(Yg), gdt, A, B, X, orc.apply(X), False, dk.DCTK_TUBE_TH, ("fwd", shape, two_sided))
        Zg = torch.empty((p, n2, s), dtype=vt, device="cuda:0")
        dk.dctk_cprod_T(ctx, op, 1.0, to_gpu(Y, vt), 0.0, Zg)
        _check(to_np(Zg), gdt, A, B, Y, orc.adjoint(Y), True, dk.DCTK_TUBE_TH, ("adj", shape, two_sided))
    finally:
        torch.cuda.synchronize()
        dk.dctk_op_destroy(op)


@pytest.mark.parametrize("gdt", [dk.DCTK_F64, dk.DCTK_F32])
def test_long_tube_epilogue_and_plain_dct(ctx, gdt):
    """Y = a M(X) + b Y (the epilogue reads Y as src) and the adjoint's
    X = a M*(Y) + b X, with the plain DCT as the tube transform."""
    p, n1, n2, s = 256, 33, 17, 6
    rng = np.random.default_rng(91)
    A = rng.standard_normal((p, n1, n2))
    X = rng.standard_normal((p, n2, s))
    Y0 = rng.standard_normal((p, n1, s))
    for tube in (dk.DCTK_TUBE_TH, dk.DCTK_TUBE_DCT2):
        orc = Operator(A, None, tube=TUBES[tube])
        op = dk.dctk_op_create(ctx, tube, gdt, to_gpu(A, F64), s)
        try:
            vt = VT[gdt]
            Yg = to_gpu(Y0, vt)
            dk.dctk_cprod(ctx, op, 0.5, to_gpu(X, vt), -2.0, Yg)
            ref = 0.5 * orc.apply(X) - 2.0 * Y0
            e = rel(to_np(Yg), ref)
            say("epilogue", TUBES[tube], gdt, e)
            assert e <= tol_prod(gdt, p)
            Xg = to_gpu(X, vt)
            dk.dctk_cprod_T(ctx, op, -1.5, to_gpu(Y0, vt), 0.25, Xg)
            ref = -1.5 * orc.adjoint(Y0) + 0.25 * X
            e = rel(to_np(Xg), ref)
            say("adjoint epilogue", TUBES[tube], gdt, e)
            assert e <= tol_prod(gdt, p)
        finally:
            torch.cuda.synchronize()
            dk.dctk_op_destroy(op)


def test_long_tube_validation(ctx):
    # not a power of two
    with pytest.raises(dk.DctkError) as ei:
        dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F32, torch.zeros((96, 4, 4), dtype=F64, device="cuda:0"), 4)
    assert ei.value.status == dk.DCTK_ESHAPE
    # beyond 2048
    with pytest.raises(dk.DctkError) as ei:
        dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F32, torch.zeros((4096, 2, 2), dtype=F64, device="cuda:0"), 2)
    assert ei.value.status == dk.DCTK_ESHAPE
    # an order-4 operator keeps the product of its tube modes <= 64
    with pytest.raises(dk.DctkError) as ei:
        dk.dctk_op_create_nd(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F32, torch.zeros((2, 64, 4, 4), dtype=F64, device="cuda:0"), 4)
    assert ei.value.status == dk.DCTK_ESHAPE


def _problem(seed, p, n, s, two_sided=False):
    rng = np.random.default_rng(seed)
    A = W.band_blur(p, n, last_weight=W.HYPER_LAST_WEIGHT) + 0.01 * rng.standard_normal((p, n, n)) / n
    B = None
    if two_sided:
        B = W.mixed_blur(W.tube_for(p), W.gaussian_toeplitz(s, 1.0, 3).T)
    Xt = W.spectral_field(rng, p, n, s)
    orc = Operator(A, B)
    Ch = orc.apply(Xt)
    N0 = rng.standard_normal(Ch.shape)
    C = Ch + 5e-3 * fro(Ch) / fro(N0) * N0
    return A, B, Xt, C, orc


def test_long_tube_fp64_lsqr_process(ctx):
    """FP64 DC-LSQR (Algorithm 6) with full reorthogonalisation, 12 steps at
    p = 256: the GPU iterate and the Golub-Kahan scalars are the oracle's."""
    p, n, s = 256, 24, 16
    A, _, _, C, orc = _problem(5, p, n, s)
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F64, to_gpu(A, F64), s)
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, 12)
    try:
        X = torch.empty((p, n, s), dtype=F64, device="cuda:0")
        dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F64), X, dk.make_opts(12, dk.DCTK_REORTH_FULL, 0, 0.0))
        ref = krylov.dc_lsqr(orc, C, 12, reorth="full")
        e = rel(to_np(X), ref["X"])
        kr = dk.dctk_krylov_read(ctx, ws, 12, dk.DCTK_KRYLOV_GKB)
        g = krylov.gkb(orc, C, 12, reorth="full")
        ea = max(abs(a - b) / abs(b) for a, b in zip(kr["alpha"][:12], g.alpha[:12]))
        say("long tube FP64 LSQR gap", e, "alpha gap", ea)
        assert e <= 1e-9
        assert ea <= 1e-9
    finally:
        torch.cuda.synchronize()
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)


@pytest.fixture(scope="module")
def hyper256(ctx):
    """A hyperspectral-like 64 x 64 x 256 problem (256 bands, band-dependent
    blur) and the FP64 oracle's DC-GK restoration (40 steps, GCV)."""
    w = W.hyperspectral(3, n=64, p=256)
    orc = Operator(w["A"])
    Ch = orc.apply(w["X_true"])
    C = Ch + w["nu"] * fro(Ch) / fro(w["N0"]) * w["N0"]
    ref = krylov.dc_gk(orc, C, 40, lam=None, gcv_mode="rect", reorth="none")
    e_ref = metrics.relative_error(w["X_true"], ref["X"])
    say("hyperspectral 64x64x256 oracle relerr", e_ref, "lambda", ref["lambda"])
    return w, C, e_ref


@pytest.mark.parametrize("gdt", [dk.DCTK_F32, dk.DCTK_BF16])
def test_long_tube_restoration(ctx, hyper256, gdt):
    w, C, e_ref = hyper256
    p, n, s = w["X_true"].shape
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(w["A"], F64), s)
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, 40)
    try:
        X = torch.empty((p, n, s), dtype=F32, device="cuda:0")
        info = dk.dctk_lsqr_tik_solve(ctx, ws, to_gpu(C, F32), X, dk.make_opts(40, 0, 0, -1.0))
        e = metrics.relative_error(w["X_true"], to_np(X))
        say("long tube restoration", gdt, "relerr", e, "oracle", e_ref, "lambda", info.lam)
        assert info.iters == 40
        assert e <= 1.05 * e_ref
    finally:
        torch.cuda.synchronize()
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)


def test_long_tube_two_sided_gmres_restarts(ctx):
    """DC-GMRES(6), 3 restart cycles, fixed lambda, two-sided, p = 128, FP64:
    the GPU iterate equals the oracle's Algorithm 3."""
    p, n, s = 128, 16, 12
    A, B, _, C, orc = _problem(7, p, n, s, two_sided=True)
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F64, to_gpu(A, F64), s, to_gpu(B, F64))
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_ARNOLDI, 6)
    try:
        X0 = 0.1 * np.random.default_rng(2).standard_normal(C.shape)
        X = to_gpu(X0, F64)
        info = dk.dctk_gmres_tik_solve(ctx, ws, to_gpu(C, F64), X, 3, dk.make_opts(6, 0, 0, 0.05))
        ref = krylov.dc_gmres(orc, C, X0, 6, 3, lam=0.05)
        e = rel(to_np(X), ref["X"])
        say("long tube GMRES restarts gap", e)
        assert info.cycles == 3
        assert e <= 1e-9
    finally:
        torch.cuda.synchronize()
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)


def test_long_tube_batch_equals_single(ctx):
    """Long-tube operators in one batch (merged launches of the fast transform
    kernels, HIP graph) give the single solves' iterates bit for bit."""
    k = 10
    shapes = [(128, 24, 16, dk.DCTK_F32), (256, 16, 16, dk.DCTK_F32), (128, 32, 24, dk.DCTK_BF16)]
    ops, wss, Cs, refs = [], [], [], []
    try:
        for i, (p, n, s, gdt) in enumerate(shapes):
            A, _, _, C, _ = _problem(20 + i, p, n, s)
            op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(A, F64), s)
            ops.append(op)
            ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, k)
            wss.append(ws)
            Cg = to_gpu(C, F32)
            Cs.append(Cg)
            X = torch.full((p, n, s), float("nan"), dtype=F32, device="cuda:0")
            dk.dctk_lsqr_tik_solve(ctx, ws, Cg, X, dk.make_opts(k, 0, 0, -1.0))
            refs.append(X)
        outs = [torch.full_like(r, float("nan")) for r in refs]
        infos = dk.dctk_batch_lsqr_tik_solve(ctx, ops, Cs, outs, dk.make_opts(k, 0, 0, -1.0))
        for out, ref, info in zip(outs, refs, infos):
            assert info.iters == k
            assert torch.equal(out, ref)
    finally:
        torch.cuda.synchronize()
        for ws in wss:
            dk.dctk_krylov_destroy(ws)
        for op in ops:
            dk.dctk_op_destroy(op)
