"""Batched DC-LSQR / DC-GK solves (merged launches, HIP graph).

Every instance of a batch must compute exactly what its own
dctk_lsqr_tik_solve computes: the merged launches run the same kernels with
the same per-instance workgroup decomposition, so the iterates are compared
bit for bit with single solves, over several graph replays with eager work in
between.  The small FP64 instance is also checked against the FP64 oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, metrics
from oracle.cprod import Operator, fro
from tests.gpu_util import rel, say, to_gpu, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2103_11847_amd as dk  # noqa: E402

F64, F32 = torch.float64, torch.float32
VT = {dk.DCTK_F64: F64, dk.DCTK_F32: F32, dk.DCTK_BF16: F32, dk.DCTK_F16: F32}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dk.dctk_create(0)
    yield c
    dk.dctk_synchronize(c)
    dk.dctk_destroy(c)


class Inst:
    """One problem instance: operator, workspace, C and X buffers (explicitly freed)."""

    def __init__(self, ctx, seed, p, n1, n2, s, gdt, k, two_sided=False):
        rng = np.random.default_rng(seed)
        if n1 == n2:
            T = W.gaussian_toeplitz(n1, 1.5, 4)
            A = W.mixed_blur(W.tube_for(p), T) + 0.02 * rng.standard_normal((p, n1, n2))
        else:
            A = rng.standard_normal((p, n1, n2)) / np.sqrt(n2)
        B = None
        if two_sided:
            B = W.mixed_blur(W.tube_for(p), W.gaussian_toeplitz(s, 1.0, 3).T)
        Xt = W.smooth_field(rng, p, n2, s)
        self.orc = Operator(A, B)
        Ch = self.orc.apply(Xt)
        N0 = rng.standard_normal(Ch.shape)
        self.C_np = Ch + 1e-2 * fro(Ch) / fro(N0) * N0
        self.X_true = Xt
        self.gdt = gdt
        self.vt = VT[gdt]
        self.op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, to_gpu(A, F64), s,
                                    None if B is None else to_gpu(B, F64))
        self.ws = dk.dctk_krylov_create(ctx, self.op, dk.DCTK_KRYLOV_GKB, k)
        self.C = to_gpu(self.C_np, self.vt)
        self.X = torch.full((p, n2, s), float("nan"), dtype=self.vt, device="cuda:0")

    def free(self):
        dk.dctk_krylov_destroy(self.ws)
        dk.dctk_op_destroy(self.op)


# (seed, p, n1, n2, s, gemm dtype, two-sided): fused FP32 (square, ragged, p = 8),
# unfused (p > 8, two-sided), BF16 and FP64 fused kernels, a 512 x 512 slice
# size that takes the 32 x 32 fused tiles, and three-kernel products whose
# Golub-Kahan steps pair the transforms (16 <= p <= 64: 24, 33 with BF16
# operands, 64)
SHAPES = [
    (1, 3, 40, 40, 40, dk.DCTK_F32, False),
    (2, 3, 64, 48, 56, dk.DCTK_F32, False),
    (3, 8, 33, 33, 33, dk.DCTK_F32, False),
    (4, 12, 32, 32, 24, dk.DCTK_F32, False),
    (5, 4, 24, 24, 24, dk.DCTK_F32, True),
    (6, 5, 30, 30, 20, dk.DCTK_BF16, False),
    (7, 3, 20, 20, 20, dk.DCTK_F64, False),
    (8, 3, 512, 512, 512, dk.DCTK_F32, False),
    (9, 3, 40, 40, 40, dk.DCTK_F32, False),
    (10, 24, 40, 40, 32, dk.DCTK_F32, False),
    (11, 33, 32, 32, 24, dk.DCTK_BF16, False),
    (12, 64, 48, 48, 40, dk.DCTK_F32, False),
]


@pytest.mark.parametrize("use_graph,reorth", [(True, dk.DCTK_REORTH_NONE), (False, dk.DCTK_REORTH_NONE),
                                              (True, dk.DCTK_REORTH_FULL)])
def test_batch_equals_single_solves(ctx, use_graph, reorth):
    k = 12
    opts = dk.make_opts(k, reorth, 0, -1.0)
    insts = [Inst(ctx, *sh[:6], k, two_sided=sh[6]) for sh in SHAPES]
    try:
        # single solves first: the reference iterates and infos
        ref_X, ref_info = [], []
        for it in insts:
            say("single", it.C.shape, it.gdt)
            info = dk.dctk_lsqr_tik_solve(ctx, it.ws, it.C, it.X, opts)
            ref_X.append(it.X.clone())
            ref_info.append(info.as_dict())
        for it in insts:
            it.X.fill_(float("nan"))
        say("batch create, graph", use_graph)
        b = dk.dctk_batch_create(ctx, [it.ws for it in insts], [it.C for it in insts],
                                 [it.X for it in insts], opts, use_graph)
        merged, single = dk.dctk_batch_stats(b)
        say("launches merged", merged, "single", single)
        assert merged < single
        try:
            for rep in range(3):
                say("batch run", rep)
                dk.dctk_batch_run(ctx, b)
                infos = dk.dctk_batch_info(ctx, b, len(insts))
                for i, it in enumerate(insts):
                    assert torch.equal(it.X, ref_X[i]), "instance %d differs on replay %d" % (i, rep)
                    got = infos[i].as_dict()
                    assert got["iters"] == ref_info[i]["iters"]
                    assert got["lambda"] == ref_info[i]["lambda"]
                    assert got["gcv"] == ref_info[i]["gcv"]
                # eager work between replays: a single solve of one instance into a scratch X
                scratch = torch.empty_like(insts[0].X)
                dk.dctk_lsqr_tik_solve(ctx, insts[0].ws, insts[0].C, scratch, opts)
                assert torch.equal(scratch, ref_X[0])
                for it in insts:
                    it.X.fill_(float("nan"))
        finally:
            dk.dctk_batch_destroy(b)
    finally:
        torch.cuda.synchronize()
        for it in insts:
            it.free()


def test_batch_fp64_instance_matches_oracle(ctx):
    k = 10
    opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0)
    insts = [Inst(ctx, 7, 3, 20, 20, 20, dk.DCTK_F64, k), Inst(ctx, 11, 3, 24, 24, 16, dk.DCTK_F64, k)]
    try:
        b = dk.dctk_batch_create(ctx, [it.ws for it in insts], [it.C for it in insts],
                                 [it.X for it in insts], opts, True)
        try:
            dk.dctk_batch_run(ctx, b)
            infos = dk.dctk_batch_info(ctx, b, len(insts))
        finally:
            dk.dctk_batch_destroy(b)
        for it, info in zip(insts, infos):
            ref = krylov.dc_gk(it.orc, it.C_np, k, lam=info.lam, reorth="none")
            say("fp64 batch vs oracle", rel(to_np(it.X), ref["X"]))
            assert rel(to_np(it.X), ref["X"]) <= 1e-9
    finally:
        torch.cuda.synchronize()
        for it in insts:
            it.free()


def test_batch_validation(ctx):
    k = 4
    a = Inst(ctx, 21, 3, 16, 16, 16, dk.DCTK_F32, k)
    try:
        opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0)
        with pytest.raises(dk.DctkError):   # the same workspace twice
            dk.dctk_batch_create(ctx, [a.ws, a.ws], [a.C, a.C], [a.X, a.X], opts)
        with pytest.raises(dk.DctkError):   # more steps than the workspace holds
            dk.dctk_batch_create(ctx, [a.ws], [a.C], [a.X], dk.make_opts(k + 1, dk.DCTK_REORTH_NONE, 0, -1.0))
        with pytest.raises(dk.DctkError):
            dk.dctk_batch_create(ctx, [], [], [], opts)
    finally:
        torch.cuda.synchronize()
        a.free()


def test_uneven_batch_of_64_restoration(ctx):
    """The 64-instance uneven workload (n in {64..512}, n3 in {3, 8, 31}, 40 steps):
    the batch equals the single solves bit for bit; the instances with n <= 128 are
    also within 1.05x of the FP64 oracle's restoration error."""
    k = 40
    opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0)
    insts, ws = [], []
    try:
        for i in range(64):
            w = W.batch_instance(i)
            p, n = w["A"].shape[0], w["A"].shape[1]
            op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F32, to_gpu(w["A"], F64), n)
            wk = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, k)
            Xt = to_gpu(w["X_true"], F64)
            Ch = torch.empty_like(Xt)
            op64 = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F64, to_gpu(w["A"], F64), n)
            dk.dctk_cprod(ctx, op64, 1.0, Xt, 0.0, Ch)
            dk.dctk_op_destroy(op64)
            N0 = to_gpu(w["N0"], F64)
            C = (Ch + w["nu"] * torch.linalg.norm(Ch) / torch.linalg.norm(N0) * N0).to(F32).contiguous()
            insts.append({"w": w, "op": op, "ws": wk, "C": C,
                          "X": torch.empty(Xt.shape, dtype=F32, device="cuda:0")})
        say("64 instances ready")
        ref = []
        for it in insts:
            dk.dctk_lsqr_tik_solve(ctx, it["ws"], it["C"], it["X"], opts)
            ref.append(it["X"].clone())
        b = dk.dctk_batch_create(ctx, [it["ws"] for it in insts], [it["C"] for it in insts],
                                 [it["X"] for it in insts], opts, True)
        try:
            merged, single = dk.dctk_batch_stats(b)
            say("launches merged", merged, "single", single)
            for it in insts:
                it["X"].fill_(float("nan"))
            dk.dctk_batch_run(ctx, b)
            dk.dctk_batch_info(ctx, b, len(insts))
        finally:
            dk.dctk_batch_destroy(b)
        for i, it in enumerate(insts):
            assert torch.equal(it["X"], ref[i]), "instance %d" % i
        # restoration against the oracle on the small instances (C formed by the oracle)
        checked = 0
        for i, it in enumerate(insts):
            w = it["w"]
            if w["A"].shape[1] > 128 or checked >= 3:
                continue
            orc = Operator(w["A"])
            Ch = orc.apply(w["X_true"])
            C = Ch + w["nu"] * fro(Ch) / fro(w["N0"]) * w["N0"]
            r = krylov.dc_gk(orc, C, k, lam=None, gcv_mode="rect", reorth="none")
            e_ref = metrics.relative_error(w["X_true"], r["X"])
            e = metrics.relative_error(w["X_true"], to_np(it["X"]))
            say("instance", i, w["A"].shape, "relerr", e, "oracle", e_ref)
            assert e <= 1.05 * e_ref
            checked += 1
        assert checked >= 1
    finally:
        torch.cuda.synchronize()
        for it in insts:
            dk.dctk_krylov_destroy(it["ws"])
            dk.dctk_op_destroy(it["op"])


def test_one_shot_batch_and_scalar_arrays(ctx):
    """dctk_batch_lsqr_tik_solve (workspaces, plan, run, info and clean-up in one
    call) gives the single solves' iterates bit for bit, and fills the caller's
    alpha / beta arrays with the Golub-Kahan scalars the workspace recorded."""
    k = 12
    shapes = SHAPES[:5]
    insts = [Inst(ctx, sd, p, n1, n2, s, g, k, ts) for (sd, p, n1, n2, s, g, ts) in shapes]
    try:
        opts = dk.make_opts(k, 0, 0, -1.0)
        refs, ref_scalars = [], []
        for it in insts:
            info, a, b = dk.solve_info_with_scalars(k + 1)
            dk.dctk_lsqr_tik_solve(ctx, it.ws, it.C, it.X, opts, info)
            kr = dk.dctk_krylov_read(ctx, it.ws, k, dk.DCTK_KRYLOV_GKB)
            assert list(a) == kr["alpha"][:k + 1] and list(b) == kr["beta"][:k + 1]
            assert b[0] == pytest.approx(float(torch.linalg.norm(it.C.double())), rel=1e-6)
            refs.append(it.X.clone())
            ref_scalars.append((list(a), list(b)))
        outs = [torch.full_like(it.X, float("nan")) for it in insts]
        bufs = [dk.solve_info_with_scalars(k + 1) for _ in insts]
        infos = dk.dctk_batch_lsqr_tik_solve(ctx, [it.op for it in insts], [it.C for it in insts], outs, opts,
                                             [bf[0] for bf in bufs])
        for it, out, ref, info, (_, a, b), (ra, rb) in zip(insts, outs, refs, infos, bufs, ref_scalars):
            assert torch.equal(out, ref)
            assert info.iters == k
            assert list(a) == ra and list(b) == rb
        # distinct operators only
        with pytest.raises(dk.DctkError):
            dk.dctk_batch_lsqr_tik_solve(ctx, [insts[0].op, insts[0].op], [insts[0].C] * 2, outs[:2], opts)
    finally:
        torch.cuda.synchronize()
        for it in insts:
            it.free()
