"""Tube transforms of the c-product, built in FP64 from their closed forms.

Test infrastructure only (see the package docstring).

Readings of the paper taken here:
  * The index range of C_n printed in Sec. 2.1 (eq. dft1) is read as
    1 <= i, j <= n (the printed strict inequalities would leave the first and
    last rows undefined).
  * Remark 2.1 calls Z "circulant" but builds it as ones on the first
    superdiagonal; the superdiagonal shift is taken.
  * Two transforms appear in Sec. 2.2: the plain orthonormal DCT used by
    Algorithm 1 (Matlab ``dct`` along mode 3) and M = W^{-1} C_n (I + Z) of
    Remark 2.1, which is the one that reproduces the Definition
    A *c B = ten(mat(A) mat(B)).  Both are provided; 'th' (M) is the default.
"""
import numpy as np


def dct_matrix(n):
    """The n x n DCT matrix C_n of Sec. 2.1, eq. (dft1).

    (C_n)_{ij} = sqrt((2 - delta_{i1}) / n) * cos((i-1)(2j-1) pi / (2n)),
    for 1 <= i, j <= n.  Written with explicit loops over 1-based indices.
    """
    C = np.zeros((n, n), dtype=np.float64)
    for i in range(1, n + 1):
        scale = np.sqrt((2.0 - (1.0 if i == 1 else 0.0)) / n)
        for j in range(1, n + 1):
            C[i - 1, j - 1] = scale * np.cos((i - 1) * (2 * j - 1) * np.pi / (2.0 * n))
    return C


def th(v):
    """Toeplitz-plus-Hankel matrix th(v) of Sec. 2.1 (display after eq. dft5).

    Toeplitz part: symmetric, first row (v_1, ..., v_n).
    Hankel part: first row (v_2, ..., v_n, 0), last row (0, v_n, ..., v_2).
    """
    v = np.asarray(v, dtype=np.float64)
    n = v.shape[0]
    T = np.zeros((n, n))
    H = np.zeros((n, n))
    for r in range(n):
        for c in range(n):
            T[r, c] = v[abs(r - c)]
    # Hankel entry depends on r + c only: h(m) for m = 0 .. 2n-2.
    for r in range(n):
        for c in range(n):
            m = r + c
            if m <= n - 2:
                H[r, c] = v[m + 1]
            elif m == n - 1:
                H[r, c] = 0.0
            else:
                H[r, c] = v[2 * n - 1 - m]
    return T + H


def shift_matrix(n):
    """Z of Remark 2.1: ones on the first superdiagonal."""
    Z = np.zeros((n, n))
    for i in range(n - 1):
        Z[i, i + 1] = 1.0
    return Z


def m_matrix(n):
    """M = W^{-1} C_n (I + Z) of Remark 2.1, W = diag(C_n(:, 1))."""
    C = dct_matrix(n)
    W = np.diag(C[:, 0])
    return np.linalg.solve(W, C @ (np.eye(n) + shift_matrix(n)))


def transform_matrix(n, tube="th"):
    """The mode-3 transform L used by the c-product.

    tube='th'   -> L = M (Remark 2.1), the transform that realises the
                   Toeplitz-plus-Hankel Definition of the c-product.
    tube='dct2' -> L = C_n, the orthonormal DCT of Algorithm 1 step 1.
    """
    if tube == "th":
        return m_matrix(n)
    if tube == "dct2":
        return dct_matrix(n)
    raise ValueError("unknown tube transform %r" % (tube,))


def inverse_transform_matrix(n, tube="th"):
    """L^{-1}, by a dense LAPACK solve (no closed form is used here)."""
    return np.linalg.inv(transform_matrix(n, tube))


def mode3(X, G):
    """Mode-3 product X x_3 G (Kolda-Bader): tube (i, j, :) maps to G @ tube.

    With the (n3, n1, n2) storage this is slice k of the result equal to
    sum_t G[k, t] * X[t].
    """
    X = np.asarray(X, dtype=np.float64)
    p = X.shape[0]
    assert G.shape == (p, p)
    return (G @ X.reshape(p, -1)).reshape(X.shape)


def mat(A):
    """mat(A) of Sec. 2.2: block Toeplitz plus block Hankel, (n1 n3) x (n2 n3).

    Block (r, c) (0-based) is A_{|r-c|} + H_{r+c}, where the Hankel blocks
    follow th(v) with tube entries replaced by frontal slices.
    """
    A = np.asarray(A, dtype=np.float64)
    p, n1, n2 = A.shape
    out = np.zeros((n1 * p, n2 * p))
    for r in range(p):
        for c in range(p):
            blk = A[abs(r - c)].copy()
            m = r + c
            if m <= p - 2:
                blk += A[m + 1]
            elif m >= p:
                blk += A[2 * p - 1 - m]
            out[r * n1:(r + 1) * n1, c * n2:(c + 1) * n2] = blk
    return out


def ten(Mt, n1, n2, p):
    """ten = inverse of mat, read off the first block column of mat(A).

    Block r of the first block column is A_r + A_{r+1} (r < p-1) and A_{p-1}
    for r = p-1, so the slices follow by back substitution.
    """
    col = [Mt[r * n1:(r + 1) * n1, 0:n2] for r in range(p)]
    A = np.zeros((p, n1, n2))
    A[p - 1] = col[p - 1]
    for r in range(p - 2, -1, -1):
        A[r] = col[r] - A[r + 1]
    return A
