"""Order-N tensors and their cosine product, built recursively from the
order-3 Definition (test infrastructure only; see the package docstring).

Sec. 1 states that the methods extend to higher-order tensors in a recursive
manner but prints no definition.  Reading taken here (the same recursion the
order-3 Definition of Sec. 2.2 itself performs on frontal slices):

  * Storage: A in R^{n1 x n2 x n3 x ... x nN} is a numpy array of shape
    (nN, ..., n3, n1, n2).  A[k] is the order-(N-1) tensor of mode-N slice k;
    N = 3 is the (n3, n1, n2) storage of the order-3 oracle.
  * Product: A *c B splits both operands along the last mode, arranges the
    slices of A in the block Toeplitz-plus-Hankel pattern of mat (Sec. 2.2),
    multiplies blocks by the order-(N-1) product, and recovers the slices as
    ten does.  At order 2 the product is the matrix product, which makes
    N = 3 the Definition of Sec. 2.2.
  * The transform form: the same product by the mode-m transform L_{n_m}
    (Remark 2.1's M, or the plain DCT) along every tube mode, frontal-face
    matrix products, and the inverse transforms -- the order-N counterpart of
    Algorithm 1.

The Krylov solvers of oracle.krylov act on any operator with apply/adjoint,
so OperatorND runs them on order-N tensors unchanged.
"""
import numpy as np

from .tube import transform_matrix


def _hankel_block(A, m):
    """Hankel part of block (r, c) with r + c = m in mat's pattern (as tube.mat)."""
    p = A.shape[0]
    if m <= p - 2:
        return A[m + 1]
    if m == p - 1:
        return np.zeros_like(A[0])
    return A[2 * p - 1 - m]


def cprod_recursive(A, B):
    """A *c B by the recursive block definition (dense, tiny sizes only).

    A: (nN, ..., n3, n1, n2), B: (nN, ..., n3, n2, s) with equal tube modes.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if A.ndim == 2:
        return A @ B
    assert A.ndim == B.ndim and A.shape[0] == B.shape[0]
    p = A.shape[0]
    # first block column of mat(B): B_c + (Hankel part at row c, column 0)
    Bcol = [B[c] + _hankel_block(B, c) for c in range(p)]
    D = []
    for r in range(p):
        acc = None
        for c in range(p):
            blk = A[abs(r - c)] + _hankel_block(A, r + c)
            term = cprod_recursive(blk, Bcol[c])
            acc = term if acc is None else acc + term
        D.append(acc)
    # ten: block r of the first block column is C_r + C_{r+1} (r < p-1), C_{p-1} last
    C = [None] * p
    C[p - 1] = D[p - 1]
    for r in range(p - 2, -1, -1):
        C[r] = D[r] - C[r + 1]
    return np.stack(C)


def tube_dims(X):
    """The tube modes (n3, ..., nN) of an order-N tensor in the storage above."""
    return tuple(reversed(np.asarray(X).shape[:-2]))


def transform_nd(X, mats):
    """Apply mats[m] along tube mode m + 3 (mats listed for n3, ..., nN):
    X x_3 mats[0] x_4 mats[1] ... (each a mode product of Kolda-Bader)."""
    Y = np.asarray(X, dtype=np.float64)
    nt = Y.ndim - 2
    assert len(mats) == nt
    for m, G in enumerate(mats):
        ax = nt - 1 - m          # storage axis of mode m + 3
        Y = np.moveaxis(np.tensordot(G, Y, axes=(1, ax)), 0, ax)
    return Y


class OperatorND:
    """M(X) = A *c X (or A *c X *c B) for order-N tensors, by the transform form,
    and its exact adjoint (transposed faces, transposed inverse transforms).

    A: (nN, ..., n3, n1, n2); optional B: (nN, ..., n3, s, s).
    """

    def __init__(self, A, B=None, tube="th"):
        self.A = np.asarray(A, dtype=np.float64)
        self.B = None if B is None else np.asarray(B, dtype=np.float64)
        self.dims = tube_dims(self.A)
        self.L = [transform_matrix(n, tube) for n in self.dims]
        self.Linv = [np.linalg.inv(L) for L in self.L]
        self.Ah = transform_nd(self.A, self.L)
        self.Bh = None if self.B is None else transform_nd(self.B, self.L)

    def apply(self, X):
        Ch = np.matmul(self.Ah, transform_nd(X, self.L))
        if self.Bh is not None:
            Ch = np.matmul(Ch, self.Bh)
        return transform_nd(Ch, self.Linv)

    def adjoint(self, Y):
        Zh = np.matmul(np.swapaxes(self.Ah, -1, -2), transform_nd(Y, [G.T for G in self.Linv]))
        if self.Bh is not None:
            Zh = np.matmul(Zh, np.swapaxes(self.Bh, -1, -2))
        return transform_nd(Zh, [L.T for L in self.L])

    def dense(self, s):
        """The matrix of M on vec(X) in storage order (tiny sizes only)."""
        shape = self.A.shape[:-1] + (s,)
        n = int(np.prod(shape))
        cols = []
        for e in range(n):
            x = np.zeros(n)
            x[e] = 1.0
            cols.append(self.apply(x.reshape(shape)).ravel())
        return np.stack(cols, axis=1)
