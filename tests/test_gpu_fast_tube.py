"""Parity of the O(p log p) tube transform (dctk_tube_fast) with the FP64 oracle.

The oracle's dense transform matrices (closed forms of eq. (dft1) and
Remark 2.1, inverses by LAPACK) give the expected values up to p = 2048; at
p = 4096 the checks are properties that hold at any size: the inverse and
adjoint identities, and sampled rows of M, whose entries have the closed
form M[k][0] = 1, M[k][t] = 2 cos(pi k t / p) for t >= 1 (the product of
W^{-1} C_n with (I + Z) collapses each pair of neighbouring cosines).

Tolerances (relative 2-norm over the whole output): FP64 1e-14 p, FP32
1e-6 + 8e-9 p.  In FP64 the bound is the oracle's: its dense M is formed as
W^{-1} (C_n (I + Z)), whose rows k near p are sums of two nearly opposite
cosines divided by cos(pi k / (2p)), so its entries carry about 25 p u of
relative error (5.9e-12 against the closed form at p = 2048), while the
fast steps stay within 1.7e-13 of the closed form there.  The row scaling D^{-1} = diag(1 / cos(pi k / (2p))) of M
(and D of its inverse) amplifies the FFT's rounding by up to 2p / pi in the
last rows, so the bound grows with p; a numpy model of the same steps gives
3.7e-6 (FP32) and 1.6e-12 (FP64) at p = 1024.
"""
import functools

import numpy as np
import pytest
import torch

from oracle import tube as otube
from tests.gpu_util import rel, say, to_gpu, to_np

pytestmark = pytest.mark.gpu

import paper_2103_11847_amd as dk  # noqa: E402

VT = {dk.DCTK_F64: torch.float64, dk.DCTK_F32: torch.float32}
E = {dk.DCTK_F64: 2048, dk.DCTK_F32: 4096}   # elements one workgroup holds
WHICH = [dk.DCTK_MAT_L, dk.DCTK_MAT_LINV, dk.DCTK_MAT_LINVT, dk.DCTK_MAT_LT]


def tol(dtype, p):
    return 1e-14 * p if dtype == dk.DCTK_F64 else 1e-6 + 8e-9 * p


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dk.dctk_create(0)
    yield c
    dk.dctk_synchronize(c)
    dk.dctk_destroy(c)


@functools.lru_cache(maxsize=None)
def family(p, tb):
    L = otube.transform_matrix(p, tb)
    Li = otube.inverse_transform_matrix(p, tb)
    return {dk.DCTK_MAT_L: L, dk.DCTK_MAT_LINV: Li, dk.DCTK_MAT_LINVT: Li.T.copy(), dk.DCTK_MAT_LT: L.T.copy()}


def run(ctx, tb, which, x, dtype):
    xt = to_gpu(x, VT[dtype])
    out = torch.full_like(xt, float("nan"))
    dk.dctk_tube_fast(ctx, dk.TUBES[tb], which, xt, out)
    return to_np(out)


@pytest.mark.parametrize("dtype", [dk.DCTK_F64, dk.DCTK_F32])
@pytest.mark.parametrize("tb", ["th", "dct2"])
@pytest.mark.parametrize("p", [16, 32, 64, 128, 256, 1024, 2048])
def test_fast_tube_matches_oracle(ctx, dtype, tb, p):
    nb = E[dtype] // p
    count = 3 * nb + 5          # three full workgroups and a ragged one
    say("fast tube", dtype, tb, p, count)
    x = np.random.default_rng(p + 11 * dtype).standard_normal((p, count))
    G = family(p, tb)
    for which in WHICH:
        got = run(ctx, tb, which, x, dtype)
        assert np.all(np.isfinite(got)), which
        err = rel(got, G[which] @ x)
        assert err <= tol(dtype, p), (which, err)


@pytest.mark.parametrize("dtype", [dk.DCTK_F64, dk.DCTK_F32])
def test_fast_tube_single_position_and_routing(ctx, dtype):
    # one position (count = 1) and the dense entry points handing p = 128 over
    p = 128
    say("fast tube routing", dtype)
    G = family(p, "th")
    x = np.random.default_rng(5).standard_normal((p, 1))
    assert rel(run(ctx, "th", dk.DCTK_MAT_L, x, dtype), G[dk.DCTK_MAT_L] @ x) <= tol(dtype, p)
    x = np.random.default_rng(6).standard_normal((p, 333))
    xt = to_gpu(x, VT[dtype])
    cases = [(dk.dctk_tube_fwd, 0, dk.DCTK_MAT_L), (dk.dctk_tube_fwd, 1, dk.DCTK_MAT_LINVT),
             (dk.dctk_tube_inv, 0, dk.DCTK_MAT_LINV), (dk.dctk_tube_inv, 1, dk.DCTK_MAT_LT)]
    for fn, adj, which in cases:
        out = torch.empty_like(xt)
        fn(ctx, dk.TUBES["th"], adj, xt, out)
        assert rel(to_np(out), G[which] @ x) <= tol(dtype, p), (fn.__name__, adj)


def test_fast_tube_rejects_bad_shapes(ctx):
    x = torch.zeros((96, 10), dtype=torch.float32, device="cuda:0")
    out = torch.empty_like(x)
    with pytest.raises(dk.DctkError):
        dk.dctk_tube_fwd(ctx, dk.TUBES["th"], 0, x, out)       # p > 64, not a power of two
    with pytest.raises(dk.DctkError):
        dk.dctk_tube_fast(ctx, dk.TUBES["th"], 0, x, out)
    x = torch.zeros((8, 10), dtype=torch.float32, device="cuda:0")
    with pytest.raises(dk.DctkError):
        dk.dctk_tube_fast(ctx, dk.TUBES["th"], 0, x, torch.empty_like(x))  # below the shortest tube
    x = torch.zeros((4096, 3), dtype=torch.float64, device="cuda:0")
    with pytest.raises(dk.DctkError):
        dk.dctk_tube_fast(ctx, dk.TUBES["th"], 0, x, torch.empty_like(x))  # FP64 tube beyond one workgroup


@pytest.mark.parametrize("tb", ["th", "dct2"])
def test_fast_tube_longest_properties(ctx, tb):
    # p = 4096 in FP32: inverse pairs, the adjoint identity and sampled rows
    p, count = 4096, 7
    say("fast tube 4096", tb)
    rng = np.random.default_rng(4096)
    x = rng.standard_normal((p, count))
    y = rng.standard_normal((p, count))
    f32 = dk.DCTK_F32
    t = tol(f32, p)
    Lx = run(ctx, tb, dk.DCTK_MAT_L, x, f32)
    assert rel(run(ctx, tb, dk.DCTK_MAT_LINV, Lx, f32), x) <= 2 * t
    Ltx = run(ctx, tb, dk.DCTK_MAT_LINVT, x, f32)
    assert rel(run(ctx, tb, dk.DCTK_MAT_LT, Ltx, f32), x) <= 2 * t
    LTy = run(ctx, tb, dk.DCTK_MAT_LT, y, f32)
    lhs = np.sum(Lx * y, axis=0)
    rhs = np.sum(x * LTy, axis=0)
    scale = np.linalg.norm(Lx, axis=0) * np.linalg.norm(y, axis=0)
    assert np.max(np.abs(lhs - rhs) / scale) <= 2 * t
    rows = [0, 1, 7, p // 2, p - 2, p - 1]
    tt = np.arange(p)
    for k in rows:
        if tb == "th":
            row = 2.0 * np.cos(np.pi * k * tt / p)
            row[0] = 1.0
        else:
            row = np.sqrt((1.0 if k == 0 else 2.0) / p) * np.cos(np.pi * k * (2 * tt + 1) / (2.0 * p))
        ref = row @ x
        assert np.linalg.norm(Lx[k] - ref) <= t * np.linalg.norm(Lx), k


@pytest.mark.parametrize("p,count", [(256, 512 * 512), (512, 65536)])
def test_fast_tube_resident_loop_matches_oracle(ctx, p, count):
    """Many more groups of tube blocks than resident workgroups (2 per CU), so
    every workgroup walks the grid stride with the next block prefetched:
    512 x 512 positions at p = 256 (16384 blocks in 8192 groups) and 65536
    positions at p = 512 (8192 blocks in 2048 groups), element-wise."""
    say("fast tube resident loop", p, count)
    x = np.random.default_rng(p + 3).standard_normal((p, count))
    G = family(p, "th")
    for which in (dk.DCTK_MAT_L, dk.DCTK_MAT_LINV):
        got = run(ctx, "th", which, x, dk.DCTK_F32)
        ref = G[which] @ x
        err = rel(got, ref)
        say("  which", which, "rel", err)
        assert err <= tol(dk.DCTK_F32, p)
        # no position is skipped or written twice: every column within its own bound
        col = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert np.max(col) <= 50 * tol(dk.DCTK_F32, p)


@pytest.mark.parametrize("p", [64, 256])
def test_fast_tube_paired_tubes_error_bound(ctx, p):
    """Two tubes share one complex FFT (tube j of a block of nb = E / p tubes is
    the real part, tube j + nb / 2 the imaginary part), so a tube's rounding
    error scales with the pair's norm, not its own: the bound the header
    states is 4x the whole-array tolerance (a maximum over tubes rather than
    an average) relative to the norm of the pair's outputs.  With every
    partner 1e4 times larger that bound holds per tube, and the small tubes'
    own relative error (~1e-2 here) shows the coupling."""
    nb = E[dk.DCTK_F32] // p
    count = 8 * nb
    rng = np.random.default_rng(p)
    x = rng.standard_normal((p, count))
    big = (np.arange(count) % nb) >= nb // 2
    x[:, big] *= 1e4
    G = family(p, "th")
    for which in WHICH:
        got = run(ctx, "th", which, x, dk.DCTK_F32)
        ref = G[which] @ x
        err = np.linalg.norm(got - ref, axis=0)
        nrm = np.linalg.norm(ref, axis=0)
        partner = np.arange(count) ^ (nb // 2)
        pair_rel = err / (nrm + nrm[partner])
        own_rel = err / nrm
        say("fast tube pairs", p, which, "max pair-relative", pair_rel.max(),
            "max own relative (small tubes)", own_rel[~big].max())
        assert pair_rel.max() <= 4 * tol(dk.DCTK_F32, p)
