"""The no-allocation tube transform (dctk_tube_apply_noalloc) against the
allocating entry points dctk_tube_fwd / dctk_tube_inv, through the C-ABI:
two calls in a row on the same GPU (the second one smaller, so it reuses the
staging array the first one filled), every matrix of both transforms, FP64
to 1e-10 and FP32 to 1e-5 relative Frobenius error."""
import numpy as np
import pytest

from tests.gpu_util import rel, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2103_11847_amd as dk  # noqa: E402

# which matrix -> (allocating entry point, its adjoint_pair flag)
REF = {dk.DCTK_MAT_L: (dk.dctk_tube_fwd, 0), dk.DCTK_MAT_LINVT: (dk.dctk_tube_fwd, 1),
       dk.DCTK_MAT_LINV: (dk.dctk_tube_inv, 0), dk.DCTK_MAT_LT: (dk.dctk_tube_inv, 1)}
TOL = {torch.float64: 1e-10, torch.float32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dk.dctk_create(0)
    yield c
    dk.dctk_synchronize(c)
    dk.dctk_destroy(c)


def _pair(ctx, tube, which, dtype, p, count, seed):
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    x = torch.randn((p, count), device="cuda:0", generator=g, dtype=torch.float64).to(dtype).contiguous()
    got = torch.full_like(x, float("nan"))
    want = torch.empty_like(x)
    dk.dctk_tube_apply_noalloc(ctx, tube, which, x, got)
    fn, adj = REF[which]
    fn(ctx, tube, adj, x, want)
    torch.cuda.synchronize()
    return rel(got.double().cpu().numpy(), want.double().cpu().numpy())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("tube", [dk.DCTK_TUBE_TH, dk.DCTK_TUBE_DCT2])
@pytest.mark.parametrize("which", [dk.DCTK_MAT_L, dk.DCTK_MAT_LINV, dk.DCTK_MAT_LINVT, dk.DCTK_MAT_LT])
def test_noalloc_matches_allocating_transform(ctx, dtype, tube, which):
    for p, count, seed in ((64, 70001, 1), (5, 333, 2)):   # the second call is smaller
        say("noalloc", dtype, tube, which, p, count)
        e = _pair(ctx, tube, which, dtype, p, count, seed)
        say("  rel", e)
        assert e <= TOL[dtype]


def test_noalloc_long_tubes_and_errors(ctx):
    """p = 256 goes to the fast transform (no staging); p = 65 (not a power of two)
    and p = 0 are refused before anything is enqueued."""
    e = _pair(ctx, dk.DCTK_TUBE_TH, dk.DCTK_MAT_L, torch.float32, 256, 4096, 3)
    say("noalloc p=256 rel", e)
    assert e <= 1e-5
    x = torch.zeros((65, 16), device="cuda:0")
    with pytest.raises(dk.DctkError) as ei:
        dk.dctk_tube_apply_noalloc(ctx, dk.DCTK_TUBE_TH, dk.DCTK_MAT_L, x, torch.empty_like(x))
    assert ei.value.status == dk.DCTK_ESHAPE
    assert dk.lib().dctk_tube_apply_noalloc(ctx, 0, 0, dk.DCTK_F32, 0, 16, x.data_ptr(), x.data_ptr() + 4096) \
        == dk.DCTK_ESHAPE
    assert dk.lib().dctk_tube_apply_noalloc(ctx, 0, 9, dk.DCTK_F32, 4, 16, x.data_ptr(), x.data_ptr() + 4096) \
        == dk.DCTK_EINVAL
