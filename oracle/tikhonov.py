"""Projected Tikhonov problems and GCV (Sec. 3.1 and 3.2).

Test infrastructure only (see the package docstring).

The projected matrix H is (m+1) x m: the Hessenberg H~_m of the Arnoldi
process (Sec. 3.1) or the lower bidiagonal C~_k of Golub-Kahan (Sec. 3.2).
Given H = U diag(sigma) V^T (full SVD, LAPACK) and g = beta U^T e_1:

  y_lambda = argmin ||beta e_1 - H y||^2 + lambda^2 ||y||^2        (eq. leastsq)
           = sum_i v_i sigma_i g_i / (sigma_i^2 + lambda^2)

Readings of the paper taken here:
  * The penalty is lambda^2 ||y||^2 throughout (eq. tr2 prints lambda).
  * The normal-equation matrix of eq. (tikho2) is H~^T H~ + lambda^2 I (the
    printed H~^T C~ is a typo); the right side of eq. (normeq2) uses
    beta_1 = ||C||_F (Algorithm 4), not alpha_1.
  * The GCV function printed as eq. (gcv2) is the form for a square
    projected problem: it drops the component g_{m+1} of beta e_1 outside
    the range of H and the "+1" of the trace for an (m+1) x m matrix.
    The default here ('rect') is the GCV function of the rectangular
    projected problem,
        G(l) = [sum_i (l^2 g_i/(s_i^2+l^2))^2 + g_{m+1}^2] / [1 + sum_i l^2/(s_i^2+l^2)]^2,
    and the printed form is kept as mode 'paper'.
  * The paper does not say how GCV is minimised.  Both this oracle and the
    HIP library use the same deterministic rule (gcv_minimize below).
"""
import numpy as np

GCV_GRID = 400          # log-spaced grid points on [1e-8 sigma_1, sigma_1]
GCV_LO_DECADES = 8.0
GCV_GOLDEN_STEPS = 200
GCV_TOL_LOG10 = 1e-10   # golden-section stop: bracket width in log10(lambda)


def projected_svd(H, beta):
    """Full SVD of the (m+1) x m projected matrix and g = beta U^T e_1.

    Returns sigma (m,), Vt (m, m), g (m+1,) with g[m] the component of
    beta e_1 outside range(H).
    """
    U, sig, Vt = np.linalg.svd(np.asarray(H, dtype=np.float64), full_matrices=True)
    g = beta * U[0, :]
    return sig, Vt, g


def tikhonov_y(sig, Vt, g, lam):
    """y_lambda = V diag(sigma/(sigma^2 + lambda^2)) g_{1:m}."""
    m = sig.shape[0]
    coef = np.zeros(m)
    for i in range(m):
        d = sig[i] ** 2 + lam ** 2
        coef[i] = sig[i] * g[i] / d if d > 0.0 else 0.0
    return Vt.T @ coef


def gcv_rect(sig, g, lam):
    """GCV of the rectangular (m+1) x m projected problem (see module docstring)."""
    m = sig.shape[0]
    l2 = lam * lam
    num = g[m] ** 2
    tr = 1.0
    for i in range(m):
        f = l2 / (sig[i] ** 2 + l2)
        num += (f * g[i]) ** 2
        tr += f
    return num / (tr * tr)


def gcv_paper(sig, g, lam):
    """The GCV function as printed in eq. (gcv2)."""
    m = sig.shape[0]
    l2 = lam * lam
    num = 0.0
    den = 0.0
    for i in range(m):
        d = sig[i] ** 2 + l2
        num += (g[i] / d) ** 2
        den += 1.0 / d
    return num / (den * den)


def gcv_minimize(sig, g, mode="rect"):
    """Deterministic GCV minimiser shared (as a rule, not as code) with the library.

    1. Evaluate G on GCV_GRID points lambda_i = sigma_1 10^(-8 + 8 i/(GCV_GRID-1)).
    2. Take the first index of the minimum.
    3. Golden-section search on t = log10(lambda) over the neighbouring grid
       cells [t_{i-1}, t_{i+1}] (clamped to the grid) until the bracket is
       narrower than GCV_TOL_LOG10 or GCV_GOLDEN_STEPS steps were taken.
    4. Return the midpoint of the final bracket if its G is not larger than
       the grid minimum, else the grid point.
    Returns (lambda, G(lambda)).
    """
    f = gcv_rect if mode == "rect" else gcv_paper
    s1 = float(sig[0]) if sig.shape[0] > 0 else 0.0
    if not s1 > 0.0:
        return 0.0, float("nan")
    t0 = np.log10(s1) - GCV_LO_DECADES
    dt = GCV_LO_DECADES / (GCV_GRID - 1)
    ts = [t0 + i * dt for i in range(GCV_GRID)]
    vals = [f(sig, g, 10.0 ** t) for t in ts]
    ib = 0
    for i in range(1, GCV_GRID):
        if vals[i] < vals[ib]:
            ib = i
    a = ts[max(ib - 1, 0)]
    b = ts[min(ib + 1, GCV_GRID - 1)]
    invphi = (np.sqrt(5.0) - 1.0) / 2.0
    c = b - invphi * (b - a)
    d = a + invphi * (b - a)
    fc = f(sig, g, 10.0 ** c)
    fd = f(sig, g, 10.0 ** d)
    steps = 0
    while (b - a) > GCV_TOL_LOG10 and steps < GCV_GOLDEN_STEPS:
        if fc <= fd:
            b, d, fd = d, c, fc
            c = b - invphi * (b - a)
            fc = f(sig, g, 10.0 ** c)
        else:
            a, c, fc = c, d, fd
            d = a + invphi * (b - a)
            fd = f(sig, g, 10.0 ** d)
        steps += 1
    tm = 0.5 * (a + b)
    fm = f(sig, g, 10.0 ** tm)
    if fm <= vals[ib]:
        return 10.0 ** tm, fm
    return 10.0 ** ts[ib], vals[ib]


def projected_residual(sig, g, lam):
    """||beta e_1 - H y_lambda|| of the (m+1) x m projected problem:
    sqrt(g_{m+1}^2 + sum_i (lambda^2 g_i / (sigma_i^2 + lambda^2))^2),
    which for Golub-Kahan (orthonormal U) is ||C - M(X_lambda)||."""
    m = sig.shape[0]
    l2 = lam * lam
    r2 = g[m] ** 2
    for i in range(m):
        r2 += (l2 * g[i] / (sig[i] ** 2 + l2)) ** 2
    return float(np.sqrt(r2))


DISC_TOL_LOG10 = 1e-12  # bisection stop: bracket width in log10(lambda)


def discrepancy_lambda(sig, g, target):
    """The discrepancy principle (Sec. 2, named with GCV as the paper's two
    parameter rules): lambda with ||beta e_1 - H y_lambda|| = target, where the
    caller passes target = eta * delta for a noise norm delta and a safety
    factor eta >= 1.  The residual increases with lambda, so log10(lambda) is
    bisected over the GCV range [sigma_1 1e-8, sigma_1]; when the target lies
    below the residual at the smallest lambda (or above the one at sigma_1)
    that end of the range is returned.  Returns (lambda, residual)."""
    s1 = float(sig[0]) if sig.shape[0] > 0 else 0.0
    if not s1 > 0.0:
        return 0.0, float("nan")
    a = np.log10(s1) - GCV_LO_DECADES
    b = np.log10(s1)
    ra = projected_residual(sig, g, 10.0 ** a)
    rb = projected_residual(sig, g, 10.0 ** b)
    if not ra < target:
        return 10.0 ** a, ra
    if not rb > target:
        return 10.0 ** b, rb
    while b - a > DISC_TOL_LOG10:
        c = 0.5 * (a + b)
        if projected_residual(sig, g, 10.0 ** c) < target:
            a = c
        else:
            b = c
    lam = 10.0 ** (0.5 * (a + b))
    return lam, projected_residual(sig, g, lam)


def lcurve_points(H, beta, kmax):
    """The L-curve of the stopping index (Sec. 3.2, after Algorithm 6): for
    k = 1..kmax the LSQR iterate's residual ||beta e_1 - H_k y_k|| and norm
    ||y_k|| (= ||C - M(X_k)|| and ||X_k|| for Golub-Kahan), where H_k is the
    leading (k+1) x k block and y_k its least-squares solution (lstsq)."""
    res, nrm = [], []
    for k in range(1, kmax + 1):
        Hk = np.asarray(H, dtype=np.float64)[: k + 1, :k]
        b = np.zeros(k + 1)
        b[0] = beta
        y, *_ = np.linalg.lstsq(Hk, b, rcond=None)
        res.append(float(np.linalg.norm(b - Hk @ y)))
        nrm.append(float(np.linalg.norm(y)))
    return np.array(res), np.array(nrm)


def menger_curvature(p0, p1, p2):
    """Signed curvature of the circle through three points of the plane:
    2 cross(p1 - p0, p2 - p1) / (|p1 - p0| |p2 - p1| |p2 - p0|), positive
    for a left turn."""
    a = (p1[0] - p0[0], p1[1] - p0[1])
    b = (p2[0] - p1[0], p2[1] - p1[1])
    c = (p2[0] - p0[0], p2[1] - p0[1])
    den = np.hypot(*a) * np.hypot(*b) * np.hypot(*c)
    if not den > 0.0:
        return 0.0
    return 2.0 * (a[0] * b[1] - a[1] * b[0]) / den


def lcurve_corner(res, nrm):
    """The corner of the L-curve (log ||R_k||, log ||X_k||), k = 1..K: the
    interior point of largest signed curvature (first one on ties), traced
    with the residual decreasing, so the corner is a right turn and its
    curvature is taken with the sign flipped.  Returns k (1-based); K when
    there are fewer than three points or no point bends that way."""
    K = len(res)
    if K < 3:
        return K
    pts = [(np.log10(res[i]), np.log10(nrm[i])) for i in range(K)]
    best, kbest = 0.0, K
    for i in range(1, K - 1):
        kap = -menger_curvature(pts[i - 1], pts[i], pts[i + 1])
        if kap > best:
            best, kbest = kap, i + 1
    return kbest


def solve_projected(H, beta, lam=None, mode="rect", target=None):
    """Projected Tikhonov solve: lam=None selects lambda by GCV, or by the
    discrepancy principle when mode is 'discrepancy' (target = eta delta).

    Returns (y, lambda).
    """
    sig, Vt, g = projected_svd(H, beta)
    if lam is None:
        if mode == "discrepancy":
            lam, _ = discrepancy_lambda(sig, g, target)
        else:
            lam, _ = gcv_minimize(sig, g, mode)
    return tikhonov_y(sig, Vt, g, lam), lam


def lower_bidiagonal(alpha, beta, k):
    """C~_k of Sec. 3.2: (k+1) x k, alpha_1..alpha_k on the diagonal and
    beta_2..beta_{k+1} below it.  alpha[0] = alpha_1, beta[0] = beta_1.

    (The paper calls it upper bidiagonal but prints a lower one; the printed
    matrix is the one Algorithm 4 produces.)
    """
    B = np.zeros((k + 1, k))
    for j in range(k):
        B[j, j] = alpha[j]
        B[j + 1, j] = beta[j + 1]
    return B
