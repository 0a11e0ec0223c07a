"""Pins of the order-N oracle (oracle/ordern.py) against the order-3
Definition, brute force and library routines."""
import numpy as np
import pytest
import scipy.fft
import scipy.sparse.linalg

from oracle import krylov
from oracle import ordern as ON
from oracle import tube
from oracle.cprod import cprod_definition, inner


def _rand(rng, *shape):
    return rng.standard_normal(shape)


@pytest.mark.parametrize("p,n1,n2,s", [(1, 2, 3, 2), (2, 3, 2, 3), (3, 2, 2, 2), (5, 2, 3, 1)])
def test_recursion_at_order3_is_the_definition(p, n1, n2, s):
    """At N = 3 the recursion (blocks multiplied as matrices) is ten(mat(A) mat(B))."""
    rng = np.random.default_rng(p * 7 + n1)
    A, B = _rand(rng, p, n1, n2), _rand(rng, p, n2, s)
    assert np.allclose(ON.cprod_recursive(A, B), cprod_definition(A, B), atol=1e-12)


def test_recursion_at_order4_is_definition_of_block_slices_by_hand():
    """Order 4 with n4 = 2, written out: mat over mode 4 has blocks
    [[A0 + A1, A1], [A1, A0 + A1]] (th(v1, v2) = [[v1 + v2, v2], [v2, v1 + v2]]
    for p = 2); the blocks multiply by the order-3 Definition; ten: C1 = D1,
    C0 = D0 - C1."""
    rng = np.random.default_rng(3)
    A, B = _rand(rng, 2, 3, 2, 2), _rand(rng, 2, 3, 2, 2)
    P = cprod_definition
    B0c, B1c = B[0] + B[1], B[1]           # first block column of mat(B)
    D0 = P(A[0] + A[1], B0c) + P(A[1], B1c)
    D1 = P(A[1], B0c) + P(A[0] + A[1], B1c)
    ref = np.stack([D0 - D1, D1])
    assert np.allclose(ON.cprod_recursive(A, B), ref, atol=1e-12)


@pytest.mark.parametrize("dims", [(2, 2), (3, 2), (2, 3), (3, 4), (2, 2, 2), (3, 1, 2)])
def test_transform_form_equals_recursive_definition(dims):
    """The order-N transform form (M along every tube mode, face products,
    inverses) equals the recursive block definition, brute force."""
    rng = np.random.default_rng(sum(dims) * 11 + len(dims))
    n1, n2, s = 2, 3, 2
    shp = tuple(reversed(dims))
    A, X = _rand(rng, *shp, n1, n2), _rand(rng, *shp, n2, s)
    ref = ON.cprod_recursive(A, X)
    got = ON.OperatorND(A).apply(X)
    assert np.abs(got - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())


def test_two_sided_order4_is_recursive_product_applied_twice():
    rng = np.random.default_rng(5)
    A, X, B = _rand(rng, 3, 2, 2, 3), _rand(rng, 3, 2, 3, 2), _rand(rng, 3, 2, 2, 2)
    ref = ON.cprod_recursive(ON.cprod_recursive(A, X), B)
    assert np.allclose(ON.OperatorND(A, B).apply(X), ref, atol=1e-11)


def test_plain_dct_transform_nd_matches_scipy():
    """With the plain DCT on every tube mode, transform_nd is scipy's
    multidimensional orthonormal DCT-II over the tube axes."""
    rng = np.random.default_rng(7)
    X = _rand(rng, 4, 3, 5, 2, 2)
    mats = [tube.dct_matrix(n) for n in (5, 3, 4)]
    ref = scipy.fft.dctn(X, type=2, norm="ortho", axes=(0, 1, 2))
    assert np.allclose(ON.transform_nd(X, mats), ref, atol=1e-13)


def test_identity_tensor_order4():
    """e_1 (x) e_1 (x) I (every tube mode's first entry) is the identity."""
    rng = np.random.default_rng(9)
    I = np.zeros((3, 2, 4, 4))
    I[0, 0] = np.eye(4)
    X = _rand(rng, 3, 2, 4, 3)
    assert np.allclose(ON.cprod_recursive(I, X), X, atol=1e-13)
    assert np.allclose(ON.OperatorND(I).apply(X), X, atol=1e-13)


def test_associativity_order4():
    rng = np.random.default_rng(11)
    A, B, X = _rand(rng, 2, 3, 2, 2), _rand(rng, 2, 3, 2, 2), _rand(rng, 2, 3, 2, 2)
    lhs = ON.cprod_recursive(ON.cprod_recursive(A, B), X)
    rhs = ON.cprod_recursive(A, ON.cprod_recursive(B, X))
    assert np.allclose(lhs, rhs, atol=1e-11)


def test_singleton_last_mode_reduces_to_order3():
    rng = np.random.default_rng(13)
    A, X = _rand(rng, 1, 4, 3, 2), _rand(rng, 1, 4, 2, 3)
    assert np.allclose(ON.cprod_recursive(A, X)[0], cprod_definition(A[0], X[0]), atol=1e-12)


def test_kronecker_transform_of_flattened_tube_index():
    """The tube modes taken together: transforming every tube mode equals one
    mode-3 product with L_{nN} (x) ... (x) L_{n3} on the flattened tube index
    (storage order, mode N most significant)."""
    rng = np.random.default_rng(17)
    X = _rand(rng, 4, 3, 2, 5)        # n4 = 4, n3 = 3
    L3, L4 = tube.m_matrix(3), tube.m_matrix(4)
    ref = (np.kron(L4, L3) @ X.reshape(12, -1)).reshape(X.shape)
    assert np.allclose(ON.transform_nd(X, [L3, L4]), ref, atol=1e-12)


@pytest.mark.parametrize("two_sided", [False, True])
def test_adjoint_is_dense_transpose_order4(two_sided):
    rng = np.random.default_rng(19)
    A = _rand(rng, 2, 3, 2, 2)
    B = _rand(rng, 2, 3, 2, 2) if two_sided else None
    op = ON.OperatorND(A, B)
    X, Y = _rand(rng, 2, 3, 2, 2), _rand(rng, 2, 3, 2, 2)
    assert abs(inner(op.apply(X), Y) - inner(X, op.adjoint(Y))) < 1e-11
    D = op.dense(2)
    cols = []
    for e in range(Y.size):
        y = np.zeros(Y.size)
        y[e] = 1.0
        cols.append(op.adjoint(y.reshape(Y.shape)).ravel())
    assert np.allclose(np.stack(cols, axis=1), D.T, atol=1e-11)


def test_lsqr_order4_equals_scipy_lsqr_on_dense_operator():
    """DC-LSQR (Algorithm 6) on an order-4 operator is textbook LSQR on its matrix."""
    rng = np.random.default_rng(23)
    A = _rand(rng, 2, 2, 3, 3)
    A[0, 0] += 3.0 * np.eye(3)
    op = ON.OperatorND(A)
    C = _rand(rng, 2, 2, 3, 2)
    D = op.dense(2)
    for k in range(1, 6):
        ours = krylov.dc_lsqr(op, C, k)["X"].ravel()
        ref = scipy.sparse.linalg.lsqr(D, C.ravel(), damp=0.0, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
        assert np.linalg.norm(ours - ref) <= 1e-10 * np.linalg.norm(ref)
