"""What the 16-bit slice-GEMM product modes round, applied to the oracle's
FP64 products (test infrastructure).

A product with BF16 or FP16 slice GEMMs rounds, to the 16-bit type and to
nearest even: the transformed operator slices (formed in FP64, narrowed
through FP32), the transformed input tubes (an FP32 transform's output), and,
for the two-sided operator, the left slice product before the right factor
multiplies it.  Accumulation, the inverse transform and the epilogue stay in
FP32.  ``rounded_product`` applies exactly those roundings to FP64
transforms, so a GPU product can be held close to it (the remaining gap is
FP32 rounding, plus the rare 16-bit rounding decision that an FP32 transform
takes differently from the FP64 one); ``roundoff_bound`` is the elementwise
forward-error bound of the same roundings against the exact product.
"""
import numpy as np

from oracle.tube import mode3

UNIT = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


def round_bf16(x):
    """x -> FP32 -> bfloat16 (round to nearest even) -> FP64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f16(x):
    """x -> FP32 -> IEEE half (round to nearest even) -> FP64."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def rounder(kind):
    return {"bf16": round_bf16, "f16": round_f16}[kind]


def rounded_product(A, B, L, X, kind, adjoint=False):
    """The product (adjoint=False: A *c X [*c B]; True: the exact adjoint
    applied to X) with the 16-bit roundings of the GEMM modes, in FP64."""
    r = rounder(kind)
    Linv = np.linalg.inv(L)
    Ah = r(mode3(A, L))
    Bh = None if B is None else r(mode3(B, L))
    if not adjoint:
        T = np.matmul(Ah, r(mode3(X, L)))
        if Bh is not None:
            T = np.matmul(r(T), Bh)
        return mode3(T, Linv)
    T = np.matmul(np.transpose(Ah, (0, 2, 1)), r(mode3(X, Linv.T)))
    if Bh is not None:
        T = np.matmul(r(T), np.transpose(Bh, (0, 2, 1)))
    return mode3(T, L.T)


def roundoff_bound(A, B, L, X, kind, adjoint=False):
    """Frobenius-norm bound on (16-bit product - exact product): each of
    the two (three, two-sided) operands of a slice product carries a relative
    error <= u, so the slice product's error is elementwise <= (2u + u^2)
    |A~| |X~| (two-sided: (3u + 3u^2 + u^3) |A~| |X~| |B~|); the output
    transform G maps it to at most |G| x_3 that.  FP32 accumulation and
    transforms add a few 1e-7 of the same quantity, covered by 1.05x."""
    u = UNIT[kind]
    Linv = np.linalg.inv(L)
    Ah = np.abs(mode3(A, L))
    if adjoint:
        Ah = np.transpose(Ah, (0, 2, 1))
        Xh = np.abs(mode3(X, Linv.T))
        G = np.abs(L.T)
    else:
        Xh = np.abs(mode3(X, L))
        G = np.abs(Linv)
    E = np.matmul(Ah, Xh)
    c = 2 * u + u * u
    if B is not None:
        Bh = np.abs(mode3(B, L))
        E = np.matmul(E, np.transpose(Bh, (0, 2, 1)) if adjoint else Bh)
        c = 3 * u + 3 * u * u + u ** 3
    return 1.05 * c * float(np.linalg.norm(mode3(E, G).ravel()))


# Gap allowed between a GPU product and ``rounded_product``: the 16-bit
# rounding decisions that an FP32 transform takes differently from the FP64
# one (measured with an FP32 model of the same steps: <= 1.6e-5 one-sided and
# <= 8.2e-5 two-sided in BF16, <= 2.4e-5 in FP16), with a 4-5x margin.  The
# error of the 16-bit product itself is 1e-3..3e-3 (BF16) and 3e-4..4e-4 (FP16).
MODEL_TOL = {"bf16": 4e-4, "f16": 1e-4}


def check_lowp(got, A, B, L, X, kind, exact, adjoint=False):
    """(gap to the rounding model, error against the exact product, the model's
    own error against it); the caller asserts gap <= MODEL_TOL[kind] and
    err <= 1.25 * model_err (the GPU rounds like the model, no worse)."""
    model = rounded_product(A, B, L, X, kind, adjoint)
    nm = np.linalg.norm(exact.ravel())
    gap = np.linalg.norm((got - model).ravel()) / np.linalg.norm(model.ravel())
    return gap, np.linalg.norm((got - exact).ravel()) / nm, np.linalg.norm((model - exact).ravel()) / nm
