"""Pins of the FP64 oracle against facts fixed by the paper or by mathematics.

Each test checks an oracle function against something other than itself: a
library routine, a brute-force definition, a closed form, an invariant the
paper proves, or a matrix the paper prints.
"""
import os

import numpy as np
import pytest
import scipy.fft
import scipy.linalg
import scipy.sparse.linalg

from oracle import krylov, metrics, tikhonov, tube
from oracle.cprod import (Operator, combine, cprod, cprod_adjoint, cprod_definition,
                          diamond, fro, inner)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- transforms

@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8, 31, 64])
def test_dct_matrix_is_scipy_orthonormal_dct2(n):
    """C_n (eq. dft1) is the orthonormal DCT-II, and C_n C_n^T = I."""
    ref = scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0)
    C = tube.dct_matrix(n)
    assert np.allclose(C, ref, atol=1e-14)
    assert np.allclose(C @ C.T, np.eye(n), atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_dct_diagonalises_th_with_eigenvalues_Mv(n):
    """eq. (dft5): C_n th(v) C_n^{-1} is diagonal; its diagonal is M v (Remark 2.1)."""
    rng = np.random.default_rng(n)
    v = rng.standard_normal(n)
    C = tube.dct_matrix(n)
    D = C @ tube.th(v) @ C.T
    assert np.abs(D - np.diag(np.diag(D))).max() < 1e-13
    assert np.allclose(np.diag(D), tube.m_matrix(n) @ v, atol=1e-13)
    # eigenvalues by LAPACK agree as a set
    ev = np.sort(np.linalg.eigvalsh(tube.th(v)))
    assert np.allclose(ev, np.sort(tube.m_matrix(n) @ v), atol=1e-12)


def test_th_reproduces_printed_colour_matrix():
    """th(0.8, 0, 0.1) equals the A_color printed in Sec. 4 (golden fixture)."""
    rows = []
    tube_vals = None
    with open(os.path.join(GOLDEN, "colour_mixing.txt")) as f:
        for line in f:
            if line.startswith("# tube:"):
                tube_vals = [float(x) for x in line.split(":")[1].split()]
            elif line.strip() and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    A_color = np.array(rows)
    assert np.allclose(tube.th(tube_vals), A_color, atol=1e-15)
    # rows sum to one, as the paper states for A_color
    assert np.allclose(A_color.sum(axis=1), 1.0)


def test_mat_of_mixed_blur_is_kronecker():
    """With A(:,:,k) = t_k T (eq. tensor_form), mat(A) = th(t) (x) T."""
    rng = np.random.default_rng(1)
    t = np.array([0.8, 0.0, 0.1])
    T = rng.standard_normal((4, 4))
    A = np.stack([c * T for c in t])
    assert np.allclose(tube.mat(A), np.kron(tube.th(t), T), atol=1e-14)


@pytest.mark.parametrize("n", [2, 3, 6])
def test_M_inverse_closed_form(n):
    """M^{-1} = (I+Z)^{-1} C_n^T W with (I+Z)^{-1}_{ij} = (-1)^{j-i} (j >= i)."""
    IZinv = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            IZinv[i, j] = (-1.0) ** (j - i)
    C = tube.dct_matrix(n)
    W = np.diag(C[:, 0])
    assert np.allclose(tube.inverse_transform_matrix(n, "th"), IZinv @ C.T @ W, atol=1e-12)


def test_M_maps_first_unit_tube_to_ones():
    """Under M every transform-domain slice of e_1 (x) I is I (identity tensor, Sec. 2.2)."""
    for n in [1, 2, 3, 8, 31]:
        e1 = np.zeros(n)
        e1[0] = 1.0
        assert np.allclose(tube.m_matrix(n) @ e1, np.ones(n), atol=1e-13)


@pytest.mark.parametrize("p,n1,n2", [(2, 2, 3), (3, 3, 2), (5, 2, 2)])
def test_block_diagonalisation_eq_dft8(p, n1, n2):
    """eq. (dft8): (C (x) I) mat(A) (C^T (x) I) is block diagonal with blocks (A x_3 M)_k."""
    rng = np.random.default_rng(p * 100 + n1)
    A = rng.standard_normal((p, n1, n2))
    C = tube.dct_matrix(p)
    BD = np.kron(C, np.eye(n1)) @ tube.mat(A) @ np.kron(C.T, np.eye(n2))
    Ah = tube.mode3(A, tube.m_matrix(p))
    for r in range(p):
        for c in range(p):
            blk = BD[r * n1:(r + 1) * n1, c * n2:(c + 1) * n2]
            if r == c:
                assert np.allclose(blk, Ah[r], atol=1e-12)
            else:
                assert np.abs(blk).max() < 1e-12


def test_ten_inverts_mat():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 3, 5))
    assert np.allclose(tube.ten(tube.mat(A), 3, 5, 4), A, atol=1e-15)


# ------------------------------------------------------------------ c-product

SHAPES = [(1, 2, 3, 2), (2, 3, 2, 4), (3, 4, 5, 3), (4, 2, 2, 2), (6, 3, 4, 5), (5, 5, 5, 1)]


@pytest.mark.parametrize("p,n1,n2,s", SHAPES)
def test_cprod_transform_equals_definition(p, n1, n2, s):
    """Algorithm 1 with L = M equals the Definition ten(mat(A) mat(B)) (brute force)."""
    rng = np.random.default_rng(p + 10 * n1 + 100 * n2 + 1000 * s)
    A = rng.standard_normal((p, n1, n2))
    X = rng.standard_normal((p, n2, s))
    ref = cprod_definition(A, X)
    out = cprod(A, X, "th")
    assert np.abs(out - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_plain_dct_product_differs_from_definition():
    """The plain DCT of Algorithm 1 does not realise the Definition for n3 >= 2."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((3, 4, 4))
    X = rng.standard_normal((3, 4, 4))
    assert np.abs(cprod(A, X, "dct2") - cprod_definition(A, X)).max() > 1e-2


@pytest.mark.parametrize("p,n1,n2,s", SHAPES[:4])
def test_closure_mat_of_product(p, n1, n2, s):
    """mat(A) mat(X) = mat(A *c X): the product stays in the T+H algebra."""
    rng = np.random.default_rng(7 + p)
    A = rng.standard_normal((p, n1, n2))
    X = rng.standard_normal((p, n2, s))
    assert np.allclose(tube.mat(A) @ tube.mat(X), tube.mat(cprod(A, X)), atol=1e-12)


def test_identity_tensor():
    """(e_1 (x) I) *c X = X under M (identity tensor of Sec. 2.2)."""
    rng = np.random.default_rng(11)
    for p in [1, 2, 3, 8]:
        I = np.zeros((p, 4, 4))
        I[0] = np.eye(4)
        X = rng.standard_normal((p, 4, 3))
        assert np.allclose(cprod(I, X), X, atol=1e-13)
        assert np.allclose(cprod_definition(I, X), X, atol=1e-13)


@pytest.mark.parametrize("tb", ["th", "dct2"])
def test_associativity(tb):
    rng = np.random.default_rng(13)
    A = rng.standard_normal((4, 3, 3))
    B = rng.standard_normal((4, 3, 3))
    X = rng.standard_normal((4, 3, 2))
    assert np.allclose(cprod(cprod(A, B, tb), X, tb), cprod(A, cprod(B, X, tb), tb), atol=1e-12)


@pytest.mark.parametrize("tb", ["th", "dct2"])
@pytest.mark.parametrize("two_sided", [False, True])
def test_adjoint_is_dense_transpose(tb, two_sided):
    """M* is the exact adjoint: <M X, Y> = <X, M* Y>, and Mat(M*) = Mat(M)^T."""
    rng = np.random.default_rng(17)
    p, n1, n2, s = 3, 3, 2, 2
    A = rng.standard_normal((p, n1, n2))
    B = rng.standard_normal((p, s, s)) if two_sided else None
    op = Operator(A, B, tb)
    X = rng.standard_normal((p, n2, s))
    Y = rng.standard_normal((p, n1, s))
    assert abs(inner(op.apply(X), Y) - inner(X, op.adjoint(Y))) < 1e-12
    Dm = op.dense(s)
    cols = []
    for e in range(p * n1 * s):
        y = np.zeros(p * n1 * s)
        y[e] = 1.0
        cols.append(op.adjoint(y.reshape(p, n1, s)).ravel())
    Dadj = np.stack(cols, axis=1)
    assert np.allclose(Dadj, Dm.T, atol=1e-12)
    # Dense M equals the literal Definition applied column by column
    if not two_sided and tb == "th":
        for e in range(p * n2 * s):
            x = np.zeros(p * n2 * s)
            x[e] = 1.0
            assert np.allclose(Dm[:, e], cprod_definition(A, x.reshape(p, n2, s)).ravel(), atol=1e-12)


@pytest.mark.parametrize("p,n1,n2,s", [(1, 2, 3, 2), (2, 3, 2, 3), (3, 2, 4, 2), (4, 3, 3, 2), (5, 2, 2, 3)])
def test_two_sided_operator_is_definition_applied_twice(p, n1, n2, s):
    """eq. (2): A *c X *c B with L = M is (A *c X) *c B, each product the
    block Toeplitz-plus-Hankel Definition of Sec. 2.2 (brute force).  A right
    factor used transposed, or multiplied on the wrong side, fails this."""
    rng = np.random.default_rng(61 + 7 * p + n1 + 3 * s)
    A = rng.standard_normal((p, n1, n2))
    B = rng.standard_normal((p, s, s))
    X = rng.standard_normal((p, n2, s))
    ref = cprod_definition(cprod_definition(A, X), B)
    out = Operator(A, B, "th").apply(X)
    assert np.abs(out - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())
    # the dense adjoint of the two-sided operator is the transpose of the
    # literal block matrix mat(B)^T (x) mat(A) acting on the unfolded X
    Dref = []
    for e in range(p * n2 * s):
        x = np.zeros(p * n2 * s)
        x[e] = 1.0
        Dref.append(cprod_definition(cprod_definition(A, x.reshape(p, n2, s)), B).ravel())
    Dref = np.stack(Dref, axis=1)
    op = Operator(A, B, "th")
    Y = rng.standard_normal((p, n1, s))
    assert np.allclose(op.adjoint(Y).ravel(), Dref.T @ Y.ravel(), atol=1e-11)


@pytest.mark.parametrize("p,n1,n2,s", [(2, 3, 2, 3), (3, 4, 3, 2), (8, 2, 3, 2)])
def test_two_sided_dct2_operator_matches_scipy_dct(p, n1, n2, s):
    """With L = C_n (Algorithm 1's orthonormal DCT along tubes), A *c X *c B is
    idct(dct(A)_k dct(X)_k dct(B)_k) per frontal slice, the DCT taken by
    scipy's FFT-based routine and the slices multiplied in explicit loops."""
    rng = np.random.default_rng(67 + p)
    A = rng.standard_normal((p, n1, n2))
    B = rng.standard_normal((p, s, s))
    X = rng.standard_normal((p, n2, s))
    Ah, Xh, Bh = (scipy.fft.dct(T, type=2, norm="ortho", axis=0) for T in (A, X, B))
    Yh = np.zeros((p, n1, s))
    for k in range(p):
        for i in range(n1):
            for j in range(s):
                acc = 0.0
                for t in range(n2):
                    for u in range(s):
                        acc += Ah[k, i, t] * Xh[k, t, u] * Bh[k, u, j]
                Yh[k, i, j] = acc
    ref = scipy.fft.idct(Yh, type=2, norm="ortho", axis=0)
    out = Operator(A, B, "dct2").apply(X)
    assert np.abs(out - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_adjoint_for_orthogonal_dct_is_slice_transpose():
    """For L = C_n (orthogonal), M* transposes every transform-domain slice."""
    rng = np.random.default_rng(19)
    A = rng.standard_normal((3, 4, 5))
    Y = rng.standard_normal((3, 4, 2))
    C = tube.dct_matrix(3)
    Ah = tube.mode3(A, C)
    ref = tube.mode3(np.matmul(np.transpose(Ah, (0, 2, 1)), tube.mode3(Y, C)), C.T)
    assert np.allclose(cprod_adjoint(A, Y, "dct2"), ref, atol=1e-13)
    # ... and for M the slice-transpose is NOT the adjoint
    Ah = tube.mode3(A, tube.m_matrix(3))
    Minv = np.linalg.inv(tube.m_matrix(3))
    wrong = tube.mode3(np.matmul(np.transpose(Ah, (0, 2, 1)), tube.mode3(Y, tube.m_matrix(3))), Minv)
    assert np.abs(wrong - cprod_adjoint(A, Y, "th")).max() > 1e-3


def test_inner_product_remark_does_not_hold():
    """Remark 2.2 (<A,B> = <A~,B~>/n3) is false for both transforms; the oracle
    therefore computes inner products in the spatial domain."""
    rng = np.random.default_rng(23)
    X = rng.standard_normal((3, 4, 4))
    for tb in ["th", "dct2"]:
        Xh = tube.mode3(X, tube.transform_matrix(3, tb))
        assert abs(inner(X, X) - inner(Xh, Xh) / 3.0) > 1e-3 * inner(X, X)
    # Parseval with factor 1 for the orthonormal DCT
    Xh = tube.mode3(X, tube.dct_matrix(3))
    assert abs(inner(X, X) - inner(Xh, Xh)) < 1e-10


# ----------------------------------------------------------- Krylov processes

def _problem(seed=29, p=3, n=4, s=2, two_sided=False, tb="th"):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((p, n, n)) + 3.0 * np.stack([np.eye(n)] + [np.zeros((n, n))] * (p - 1))
    B = (rng.standard_normal((p, s, s)) + 2.0 * np.stack([np.eye(s)] + [np.zeros((s, s))] * (p - 1))) if two_sided else None
    op = Operator(A, B, tb)
    C = rng.standard_normal((p, n, s))
    return op, C


@pytest.mark.parametrize("two_sided", [False, True])
def test_gkb_relations_prop_3_2(two_sided):
    """Proposition 3.2 relations and orthonormality under the c-diamond product."""
    op, C = _problem(two_sided=two_sided)
    m = 5
    g = krylov.gkb(op, C, m, reorth="full")
    assert g.steps == m and not g.breakdown
    Ct = g.bidiagonal(m)
    # A *c V_m = U_{m+1} (*) C~_m
    for j in range(m):
        lhs = op.apply(g.V[j])
        rhs = combine(g.U[: m + 1], Ct[:, j])
        assert fro(lhs - rhs) < 1e-12
    # A^T *c U_m = V_m (*) C_m^T  (C_m = first m rows of C~_m)
    Cm = Ct[:m, :]
    for j in range(m):
        lhs = op.adjoint(g.U[j])
        rhs = combine(g.V[:m], Cm.T[:, j])
        assert fro(lhs - rhs) < 1e-12
    # U_{m+1} (*) (beta_1 e_1) = C
    e = np.zeros(m + 1)
    e[0] = g.beta[0]
    assert fro(combine(g.U[: m + 1], e) - C) < 1e-12
    # orthonormality and norm preservation
    assert np.allclose(diamond(g.U[: m + 1], g.U[: m + 1]), np.eye(m + 1), atol=1e-13)
    assert np.allclose(diamond(g.V[:m], g.V[:m]), np.eye(m), atol=1e-13)
    z = np.random.default_rng(1).standard_normal(m + 1)
    assert abs(fro(combine(g.U[: m + 1], z)) - np.linalg.norm(z)) < 1e-12


@pytest.mark.parametrize("ortho", ["mgs", "cgs2"])
def test_arnoldi_relations_prop_3_1(ortho):
    """Proposition 3.1 relations for Algorithm 2."""
    op, C = _problem(seed=31)
    m = 6
    ar = krylov.Arnoldi(op, C, m, ortho)
    for _ in range(m):
        assert ar.step()
    H = ar.hessenberg()
    for j in range(m):
        assert fro(op.apply(ar.V[j]) - combine(ar.V[: m + 1], H[:, j])) < 1e-12
    assert np.allclose(diamond(ar.V[: m + 1], ar.V[: m + 1]), np.eye(m + 1), atol=1e-12)
    # V_m^T <> (A *c V_m) = H_m
    AV = [op.apply(v) for v in ar.V[:m]]
    assert np.allclose(diamond(ar.V[:m], AV), H[:m, :], atol=1e-12)
    # H is upper Hessenberg
    assert np.abs(np.tril(H, -2)).max() == 0.0


def test_lsqr_equals_scipy_lsqr_on_dense_operator():
    """DC-LSQR iterates equal textbook LSQR (scipy) on the dense matrix of M."""
    op, C = _problem(seed=37, p=3, n=4, s=2)
    D = op.dense(2)
    b = C.ravel()
    for k in range(1, 7):
        ours = krylov.dc_lsqr(op, C, k)["X"].ravel()
        ref = scipy.sparse.linalg.lsqr(D, b, damp=0.0, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
        assert np.linalg.norm(ours - ref) <= 1e-10 * np.linalg.norm(ref)


def test_lsqr_equals_gk_at_lambda_zero_and_residual():
    """Algorithm 6 iterate = Algorithm 5 at lambda = 0; |phibar_{k+1}| = ||C - M(X_k)||."""
    op, C = _problem(seed=41, two_sided=True)
    for k in [1, 3, 6]:
        ls = krylov.dc_lsqr(op, C, k)
        gk = krylov.dc_gk(op, C, k, lam=0.0)
        assert fro(ls["X"] - gk["X"]) <= 1e-10 * fro(gk["X"])
        assert abs(ls["resnorm"] - fro(C - op.apply(ls["X"]))) <= 1e-10 * fro(C)


def test_gmres_lambda0_is_krylov_least_squares():
    """One DC-GMRES(m) cycle at lambda = 0 minimises ||C - M(X_0 + Z)|| over
    Z in TK_m(A, R_0) (eq. tr3), checked by brute force with the power basis."""
    op, C = _problem(seed=43, p=2, n=3, s=2)
    rng = np.random.default_rng(2)
    X0 = rng.standard_normal(C.shape)
    R0 = C - op.apply(X0)
    for m in [1, 2, 3]:
        K = [R0]
        for _ in range(m - 1):
            K.append(op.apply(K[-1]))
        Kmat = np.stack([op.apply(k).ravel() for k in K], axis=1)
        coef, *_ = np.linalg.lstsq(Kmat, R0.ravel(), rcond=None)
        ref = X0 + combine(K, coef)
        out = krylov.dc_gmres(op, C, X0, m, 1, lam=0.0)["X"]
        assert fro(out - ref) <= 1e-9 * fro(ref)


@pytest.mark.parametrize("two_sided", [False, True])
def test_restarted_gmres_lambda0_is_restarted_krylov_least_squares(two_sided):
    """Algorithm 3 with restarts at lambda = 0: every cycle c restarts from the
    true residual R = C - M(X_{c-1}) and adds the minimiser of
    ||R - M(Z)|| over Z in TK_m(A, R) (eq. tr3).  Reference: that recursion
    written out on the dense matrix of M with the power basis of each cycle's
    Krylov space and a least-squares solve; a cycle that reuses R_0 or skips
    X's update fails it."""
    op, C = _problem(seed=71, p=2, n=3, s=2, two_sided=two_sided)
    D = op.dense(2)
    b = C.ravel()
    rng = np.random.default_rng(3)
    X0 = rng.standard_normal(C.shape)
    for m, cycles in [(1, 4), (2, 3), (3, 2)]:
        x = X0.ravel().copy()
        for _ in range(cycles):
            r = b - D @ x
            K = [r]
            for _ in range(m - 1):
                K.append(D @ K[-1])
            K = np.stack(K, axis=1)
            coef, *_ = np.linalg.lstsq(D @ K, r, rcond=None)
            x = x + K @ coef
        out = krylov.dc_gmres(op, C, X0, m, cycles, lam=0.0)
        assert np.linalg.norm(out["X"].ravel() - x) <= 1e-9 * np.linalg.norm(x)
        assert abs(out["resnorm"] - np.linalg.norm(b - D @ x)) <= 1e-9 * np.linalg.norm(b)
        # restarts do make progress here: more cycles, smaller residual
        one = krylov.dc_gmres(op, C, X0, m, 1, lam=0.0)
        assert out["resnorm"] < one["resnorm"]


def test_restarted_gmres_matches_scipy_gmres():
    """DC-GMRES(m) at lambda = 0 with c cycles equals scipy's restarted GMRES
    on the dense matrix of M (restart = m, c outer iterations, no tolerance
    stop), a library implementation of the same restarted minimisation."""
    op, C = _problem(seed=73, p=2, n=3, s=2)
    D = op.dense(2)
    b = C.ravel()
    for m, cycles in [(2, 3), (4, 2)]:
        ref, info = scipy.sparse.linalg.gmres(D, b, x0=np.zeros_like(b), restart=m, maxiter=cycles,
                                              rtol=1e-300, atol=0.0)
        out = krylov.dc_gmres(op, C, np.zeros_like(C), m, cycles, lam=0.0)["X"].ravel()
        assert np.linalg.norm(out - ref) <= 1e-8 * np.linalg.norm(ref)


def test_gk_tikhonov_full_dimension_is_dense_tikhonov():
    """At k = dim, the projected Tikhonov iterate equals (M*M + l^2 I)^{-1} M* C."""
    op, C = _problem(seed=47, p=2, n=3, s=2)
    D = op.dense(2)
    dim = D.shape[1]
    lam = 0.3
    ref = np.linalg.solve(D.T @ D + lam ** 2 * np.eye(dim), D.T @ C.ravel())
    out = krylov.dc_gk(op, C, dim, lam=lam, reorth="full")
    assert np.linalg.norm(out["X"].ravel() - ref) <= 1e-10 * np.linalg.norm(ref)


def test_gk_tikhonov_krylov_restriction():
    """For k < dim, the iterate minimises the Tikhonov functional over
    K_k(M*M, M*C) (dense check with an orthonormalised power basis)."""
    op, C = _problem(seed=53, p=2, n=3, s=2)
    D = op.dense(2)
    lam = 0.2
    b = C.ravel()
    for k in [2, 4]:
        K = [D.T @ b]
        for _ in range(k - 1):
            K.append(D.T @ (D @ K[-1]))
        Q, _ = np.linalg.qr(np.stack(K, axis=1))
        A_stack = np.vstack([D @ Q, lam * np.eye(k)])
        z, *_ = np.linalg.lstsq(A_stack, np.concatenate([b, np.zeros(k)]), rcond=None)
        ref = Q @ z
        out = krylov.dc_gk(op, C, k, lam=lam, reorth="full")["X"].ravel()
        assert np.linalg.norm(out - ref) <= 1e-9 * np.linalg.norm(ref)


def test_breakdown_identity_operator():
    """A = e_1 (x) I: alpha_1 = 1, beta_2 = 0, h_21 = 0, exact recovery in one step."""
    p, n, s = 3, 4, 2
    A = np.zeros((p, n, n))
    A[0] = np.eye(n)
    rng = np.random.default_rng(59)
    C = rng.standard_normal((p, n, s))
    op = Operator(A)
    g = krylov.gkb(op, C, 5)
    assert g.breakdown and g.steps == 1
    assert abs(g.alpha[0] - 1.0) < 1e-14 and g.beta[1] < 1e-14
    ls = krylov.dc_lsqr(op, C, 5)
    assert ls["status"] == "breakdown" and fro(ls["X"] - C) < 1e-13
    gm = krylov.dc_gmres(op, C, np.zeros_like(C), 4, 1, lam=0.0)
    assert gm["status"] == "breakdown" and fro(gm["X"] - C) < 1e-13


# ------------------------------------------------------- projected problems

def _rand_projected(seed, m, bidiag):
    rng = np.random.default_rng(seed)
    if bidiag:
        a = np.exp(-0.5 * np.arange(m + 1)) * rng.uniform(0.5, 1.5, m + 1)
        b = np.exp(-0.5 * np.arange(m + 1)) * rng.uniform(0.5, 1.5, m + 1)
        H = tikhonov.lower_bidiagonal(a, b, m)
    else:
        H = np.triu(rng.standard_normal((m + 1, m)), -1) * np.exp(-0.4 * np.arange(m))[None, :]
    return H, float(rng.uniform(0.5, 2.0))


@pytest.mark.parametrize("bidiag", [True, False])
def test_projected_solve_three_ways(bidiag):
    """SVD solve = normal equations (eq. tikho2/normeq2) = stacked LS (eq. min)."""
    H, beta = _rand_projected(61, 8, bidiag)
    m = H.shape[1]
    rhs = np.zeros(m + 1)
    rhs[0] = beta
    for lam in [1e-3, 0.05, 1.0]:
        y, _ = tikhonov.solve_projected(H, beta, lam)
        y_ne = np.linalg.solve(H.T @ H + lam ** 2 * np.eye(m), H.T @ rhs)
        y_ls, *_ = np.linalg.lstsq(np.vstack([H, lam * np.eye(m)]), np.concatenate([rhs, np.zeros(m)]), rcond=None)
        assert np.allclose(y, y_ne, rtol=1e-8, atol=1e-10)
        assert np.allclose(y, y_ls, rtol=1e-8, atol=1e-10)


def _dense_gcv(H, beta, lam, square=False):
    """GCV from its definition: ||(I - Infl) b||^2 / trace(I - Infl)^2, no SVD."""
    r, m = H.shape
    b = np.zeros(r)
    b[0] = beta
    Infl = H @ np.linalg.solve(H.T @ H + lam ** 2 * np.eye(m), H.T)
    res = b - Infl @ b
    return float(res @ res) / float(np.trace(np.eye(r) - Infl)) ** 2


@pytest.mark.parametrize("bidiag", [True, False])
def test_gcv_rect_matches_definition(bidiag):
    H, beta = _rand_projected(67, 7, bidiag)
    sig, Vt, g = tikhonov.projected_svd(H, beta)
    for lam in [1e-4, 1e-2, 0.3, 3.0]:
        assert abs(tikhonov.gcv_rect(sig, g, lam) - _dense_gcv(H, beta, lam)) <= 1e-9 * _dense_gcv(H, beta, lam)


def test_gcv_paper_is_square_problem_gcv():
    """The printed eq. (gcv2) is the GCV function of a square projected problem."""
    rng = np.random.default_rng(71)
    H = rng.standard_normal((6, 6)) * np.exp(-0.5 * np.arange(6))[None, :]
    sig, Vt, g = tikhonov.projected_svd(H, 1.3)
    for lam in [1e-3, 0.1, 1.0]:
        ref = _dense_gcv(H, 1.3, lam)
        assert abs(tikhonov.gcv_paper(sig, g, lam) - ref) <= 1e-8 * ref


@pytest.mark.parametrize("mode", ["rect", "paper"])
@pytest.mark.parametrize("seed", [73, 79, 83])
def test_gcv_minimiser_against_brute_force(mode, seed):
    """The minimiser finds the minimum of a 1e5-point log grid to grid resolution."""
    H, beta = _rand_projected(seed, 12, True)
    sig, Vt, g = tikhonov.projected_svd(H, beta)
    f = tikhonov.gcv_rect if mode == "rect" else tikhonov.gcv_paper
    lam, val = tikhonov.gcv_minimize(sig, g, mode)
    grid = sig[0] * 10.0 ** np.linspace(-8, 0, 100000)
    brute = min(f(sig, g, l) for l in grid)
    assert val <= brute * (1.0 + 1e-6)
    assert abs(val - f(sig, g, lam)) <= 1e-12 * val


def _dense_residual(H, beta, lam):
    """||beta e_1 - H y_lambda|| with y_lambda from the stacked least-squares
    problem [H; lambda I] y = [beta e_1; 0] (no SVD)."""
    r, m = H.shape
    b = np.zeros(r)
    b[0] = beta
    y, *_ = np.linalg.lstsq(np.vstack([H, lam * np.eye(m)]), np.concatenate([b, np.zeros(m)]), rcond=None)
    return float(np.linalg.norm(b - H @ y))


@pytest.mark.parametrize("seed", [97, 101, 103])
def test_discrepancy_lambda_meets_target(seed):
    """The discrepancy principle's lambda: the residual of the dense stacked
    least-squares solve at that lambda equals the target (to 1e-9), for
    targets inside the attainable range; targets outside return the ends."""
    H, beta = _rand_projected(seed, 10, True)
    sig, Vt, g = tikhonov.projected_svd(H, beta)
    lo = _dense_residual(H, beta, sig[0] * 1e-8)
    hi = _dense_residual(H, beta, sig[0])
    for f in (0.1, 0.5, 0.9):
        target = lo + f * (hi - lo)
        lam, res = tikhonov.discrepancy_lambda(sig, g, target)
        assert sig[0] * 1e-8 < lam < sig[0]
        assert abs(_dense_residual(H, beta, lam) - target) <= 1e-9 * target
        assert abs(res - target) <= 1e-9 * target
    lam, _ = tikhonov.discrepancy_lambda(sig, g, 0.5 * lo)
    assert lam == pytest.approx(sig[0] * 1e-8, rel=1e-12)
    lam, _ = tikhonov.discrepancy_lambda(sig, g, 2.0 * hi)
    assert lam == pytest.approx(sig[0], rel=1e-12)


def test_discrepancy_lambda_one_step_closed_form():
    """k = 1: H = [alpha; beta_2] has sigma^2 = alpha^2 + beta_2^2,
    g_1 = beta alpha / sigma, g_2 = beta beta_2 / sigma and the residual
    r(lambda)^2 = g_2^2 + (q g_1)^2 with q = lambda^2 / (sigma^2 + lambda^2), so
    the target T is met at lambda^2 = q sigma^2 / (1 - q),
    q = sqrt(T^2 - g_2^2) / g_1 (q < 1/2 keeps lambda below sigma_1)."""
    alpha, beta2, beta = 0.8, 0.3, 1.7
    H = np.array([[alpha], [beta2]])
    sig, Vt, g = tikhonov.projected_svd(H, beta)
    s2 = alpha ** 2 + beta2 ** 2
    g1, g2 = beta * alpha / np.sqrt(s2), beta * beta2 / np.sqrt(s2)
    for q in (0.01, 0.2, 0.45):
        target = np.sqrt(g2 ** 2 + (q * g1) ** 2)
        lam_ref = np.sqrt(q * s2 / (1.0 - q))
        lam, _ = tikhonov.discrepancy_lambda(sig, g, target)
        assert lam == pytest.approx(lam_ref, rel=1e-10)


def test_lcurve_points_are_lsqr_residuals_and_norms():
    """The L-curve points from least squares on the leading blocks of C~_k
    equal Algorithm 6's |phibar_{k+1}| and ||X_k||_F of the LSQR iterates."""
    op, C = _problem(seed=107, p=3, n=6, s=4)
    K = 6
    ref = krylov.dc_lsqr(op, C, K, reorth="full", history=True)
    g = ref["gkb"]
    res, nrm = tikhonov.lcurve_points(g.bidiagonal(K), g.beta[0], K)
    for k in range(1, K + 1):
        rk = krylov.dc_lsqr(op, C, k, reorth="full")["resnorm"]
        assert abs(res[k - 1] - rk) <= 1e-10 * max(rk, 1e-300) + 1e-14
        assert abs(nrm[k - 1] - np.linalg.norm(ref["history"][k - 1])) <= 1e-10 * nrm[k - 1]


def test_menger_curvature_circle_and_sign():
    """Three points on a circle of radius 2 have curvature 1/2, positive for a
    counter-clockwise (left) turn and negative for the reverse order;
    collinear points have curvature 0."""
    pts = [(2.0 * np.cos(t), 2.0 * np.sin(t)) for t in (0.1, 0.7, 1.6)]
    assert tikhonov.menger_curvature(*pts) == pytest.approx(0.5, rel=1e-12)
    assert tikhonov.menger_curvature(*pts[::-1]) == pytest.approx(-0.5, rel=1e-12)
    assert tikhonov.menger_curvature((0, 0), (1, 1), (3, 3)) == 0.0


def test_lcurve_corner_of_a_right_angle():
    """A polyline going left along a horizontal line and then up a vertical
    one (in log-log coordinates) has its corner at the vertex."""
    xs = [4.0, 3.0, 2.0, 1.0, 1.0, 1.0, 1.0]
    ys = [0.0, 0.0, 0.0, 0.0, 1.0, 2.0, 3.0]
    res = 10.0 ** np.array(xs)
    nrm = 10.0 ** np.array(ys)
    assert tikhonov.lcurve_corner(res, nrm) == 4
    assert tikhonov.lcurve_corner(res[:2], nrm[:2]) == 2


# ------------------------------------------------------------------ metrics

def test_snr_relerr_consistency():
    """SNR = 20 log10(||X^ - E|| / ||X^||) - 20 log10(relerr) (both use ||X^ - X||)."""
    rng = np.random.default_rng(89)
    Xt = rng.uniform(0, 1, (3, 8, 8))
    X = Xt + 0.05 * rng.standard_normal(Xt.shape)
    e = metrics.relative_error(Xt, X)
    lhs = metrics.snr(Xt, X)
    rhs = 20 * np.log10(np.linalg.norm(Xt - Xt.mean()) / np.linalg.norm(Xt)) - 20 * np.log10(e)
    assert abs(lhs - rhs) < 1e-10


# ---------------------------------------------------------------- learned stop MLP
from oracle import mlp as omlp  # noqa: E402


def test_mlp_gelu_closed_forms():
    # GELU(0) = 0, GELU(x) -> x for large x, -> 0 for very negative x, and
    # GELU(1) = Phi(1) with Phi(1) = 0.841344746068543 (standard normal table)
    assert omlp.gelu(0.0) == 0.0
    assert abs(float(omlp.gelu(1.0)) - 0.841344746068543) < 1e-15
    assert abs(float(omlp.gelu(10.0)) - 10.0) < 1e-12
    assert abs(float(omlp.gelu(-10.0))) < 1e-20
    # derivative: Phi(0) = 1/2 at 0; against central differences elsewhere
    assert abs(float(omlp.gelu_grad(0.0)) - 0.5) < 1e-15
    for x in (-2.3, -0.4, 0.7, 1.9):
        h = 1e-6
        fd = (float(omlp.gelu(x + h)) - float(omlp.gelu(x - h))) / (2 * h)
        assert abs(float(omlp.gelu_grad(x)) - fd) < 1e-8


def test_mlp_zero_weights_output_is_bias():
    P = np.zeros(omlp.N_PARAMS)
    P[-2:] = [0.25, -1.5]
    out, _ = omlp.forward(P, np.random.default_rng(0).standard_normal((5, 16)))
    assert np.all(out == np.array([0.25, -1.5]))


def test_mlp_gradients_central_differences():
    rng = np.random.default_rng(3)
    P = 0.3 * rng.standard_normal(omlp.N_PARAMS)
    X = rng.standard_normal((7, 16))
    T = rng.standard_normal((7, 2))
    w = np.array([1.0, 0.5])

    def loss(Pv):
        out, _ = omlp.forward(Pv, X)
        return omlp.loss_and_dout(out, T, w)[0]

    out, cache = omlp.forward(P, X)
    _, dout = omlp.loss_and_dout(out, T, w)
    g = omlp.backward(P, cache, dout)
    idx = rng.choice(omlp.N_PARAMS, 40, replace=False)
    idx = np.concatenate([idx, [0, 1023, 1024, 1087, 1088, 5183, 5184, 5247, 5248, 5375, 5376, 5377]])
    for i in idx:
        e = np.zeros_like(P)
        e[i] = 1e-6
        fd = (loss(P + e) - loss(P - e)) / 2e-6
        assert abs(g[i] - fd) <= 1e-7 * max(1.0, abs(fd)), i


def test_mlp_bf16_rounding():
    # exactly representable values stay; halfway cases go to even; 1 + 2^-9 rounds down to 1
    vals = np.array([1.0, 0.5, -3.0, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -9, 1.0 + 3 * 2.0 ** -9], dtype=np.float32)
    r = omlp.bf16_round(vals)
    assert list(r) == [1.0, 0.5, -3.0, 1.0, 1.0, 1.0 + 2.0 ** -7]


def test_mlp_features_definition():
    alpha = np.array([2.0, 1.0, 0.5, 0.25, 0.2, 0.1, 0.05, 0.02, 0.01])
    beta = np.array([4.0, 1.0, 1.0, 0.5, 0.5, 0.2, 0.1, 0.1, 0.05])
    phibar = np.array([4.0, 2.0, 1.0, 0.5, 0.4, 0.3, 0.2, 0.1, 0.05])
    f = omlp.features(alpha, beta, phibar)
    assert f[0] == np.log(0.5) and f[8] == np.log(0.5)
    assert f[7] == np.log(0.02 / 0.1) and f[15] == np.log(0.05 / 4.0)


def test_mlp_adam_first_step_is_signed_lr():
    # the first bias-corrected Adam step moves each parameter by lr * g / (|g| + eps)
    P = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    Pn, m, v = omlp.adam(P, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(Pn, P - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
