"""The c-product, its exact adjoint, and the operators of eq. (2).

Test infrastructure only (see the package docstring).

Readings of the paper taken here:
  * The transpose A^T *c used by Algorithms 4 and 6 is never defined for the
    c-product.  It is read as the exact adjoint of X -> A *c X under the
    inner product of Sec. 2.2 (the elementwise sum of products), since that is
    what the Golub-Kahan relations of Proposition 3.2 require.  For an
    orthogonal transform (the plain DCT) this reduces to transposing every
    transform-domain frontal slice; for M of Remark 2.1 it does not.
  * The algorithms of Sec. 3 are written for A *c X only; the experiments of
    Sec. 4 use A *c X *c B (eq. tensor_form).  Both are provided as one
    operator with an optional right factor.
"""
import numpy as np

from .tube import mat, mode3, ten, transform_matrix


def cprod_definition(A, B):
    """A *c B = ten(mat(A) mat(B)), the Definition of Sec. 2.2 (dense, tiny sizes)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    p, n1, n2 = A.shape
    pb, n2b, m = B.shape
    assert p == pb and n2 == n2b
    return ten(mat(A) @ mat(B), n1, m, p)


def cprod(A, B, tube="th"):
    """Algorithm 1: transform tubes, multiply frontal slices, transform back.

    Step 1: A~ = A x_3 L, B~ = B x_3 L.  Step 2: C~^(i) = A~^(i) B~^(i).
    Step 3: C = C~ x_3 L^{-1}.  L is M (Remark 2.1) or C_n (see tube.py).
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    p = A.shape[0]
    L = transform_matrix(p, tube)
    Ah = mode3(A, L)
    Bh = mode3(B, L)
    Ch = np.matmul(Ah, Bh)
    return mode3(Ch, np.linalg.inv(L))


def cprod_adjoint(A, Y, tube="th"):
    """Exact adjoint of X -> A *c X: the Z with <A *c X, Y> = <X, Z> for all X.

    With vec over (k, i, j): A *c X = (L^{-1} (x) I) blkdiag(A~_k) (L (x) I) x,
    so the adjoint is (L^T (x) I) blkdiag(A~_k^T) (L^{-T} (x) I) y.
    """
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    p = A.shape[0]
    L = transform_matrix(p, tube)
    Ah = mode3(A, L)
    Yh = mode3(Y, np.linalg.inv(L).T)
    Zh = np.matmul(np.transpose(Ah, (0, 2, 1)), Yh)
    return mode3(Zh, L.T)


class Operator:
    """M(X) = A *c X, or A *c X *c B (eq. 2), and its exact adjoint M*.

    A: (p, n1, n2); optional B: (p, s, s).  X: (p, n2, s); M(X): (p, n1, s).
    """

    def __init__(self, A, B=None, tube="th"):
        self.A = np.asarray(A, dtype=np.float64)
        self.B = None if B is None else np.asarray(B, dtype=np.float64)
        self.tube = tube
        p = self.A.shape[0]
        self.p = p
        self.L = transform_matrix(p, tube)
        self.Linv = np.linalg.inv(self.L)
        self.Ah = mode3(self.A, self.L)
        self.Bh = None if self.B is None else mode3(self.B, self.L)

    def apply(self, X):
        Xh = mode3(np.asarray(X, dtype=np.float64), self.L)
        Ch = np.matmul(self.Ah, Xh)
        if self.Bh is not None:
            Ch = np.matmul(Ch, self.Bh)
        return mode3(Ch, self.Linv)

    def adjoint(self, Y):
        Yh = mode3(np.asarray(Y, dtype=np.float64), self.Linv.T)
        Zh = np.matmul(np.transpose(self.Ah, (0, 2, 1)), Yh)
        if self.Bh is not None:
            Zh = np.matmul(Zh, np.transpose(self.Bh, (0, 2, 1)))
        return mode3(Zh, self.L.T)

    def dense(self, s):
        """The matrix of M acting on vec(X) (index order (k, i, j)); tiny sizes only."""
        p, n1, n2 = self.A.shape
        n = p * n2 * s
        cols = []
        for e in range(n):
            x = np.zeros(n)
            x[e] = 1.0
            cols.append(self.apply(x.reshape(p, n2, s)).ravel())
        return np.stack(cols, axis=1)


def inner(X, Y):
    """<X, Y> = sum of elementwise products (Sec. 2.2, Definition)."""
    return float(np.sum(np.asarray(X, dtype=np.float64) * np.asarray(Y, dtype=np.float64)))


def fro(X):
    """||X||_F = sqrt(<X, X>)."""
    return float(np.sqrt(inner(X, X)))


def diamond(As, Bs):
    """The c-diamond product A^T <> B of Sec. 2.2: the p x l matrix of <A_i, B_j>."""
    return np.array([[inner(a, b) for b in Bs] for a in As])


def combine(Vs, y):
    """V (*) y = sum_j y_j V_j (eq. ev1 and the display after it)."""
    out = np.zeros_like(np.asarray(Vs[0], dtype=np.float64))
    for v, c in zip(Vs, y):
        out = out + c * v
    return out
