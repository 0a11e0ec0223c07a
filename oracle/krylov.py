"""Global Krylov processes and solvers of Sec. 3, in FP64, step by step.

Test infrastructure only (see the package docstring).

Everything acts on an ``Operator`` (oracle.cprod) through ``apply`` (M) and
``adjoint`` (M*).  Inner products and norms are the elementwise ones of the
Definition in Sec. 2.2, computed in the spatial domain.

Readings of the paper taken here:
  * Remark 2.2 (inner products through the block-diagonal transform domain
    with a 1/n3 factor) does not hold for either transform and is not used.
  * Algorithm 6 uses the symbol W both for the Golub-Kahan residual of step
    (a) and for the LSQR search direction of step (f); they are kept apart
    here (``Ut`` for the former, ``W`` for the latter), and X_i of step (f)
    is read as X_j.
  * The breakdown tests of Algorithm 4 are commented out in the paper;
    Algorithm 2 stops when h_{j+1,j} = 0.  Both processes here stop when the
    new norm is <= 64 eps times the largest alpha/beta/h seen so far, and
    report a breakdown with everything computed up to that step.
  * Reorthogonalisation is not in the paper.  It is offered as an option
    ('none', 'v' for the V basis only, 'full' for both bases; Arnoldi:
    'mgs' literal, 'cgs2' classical Gram-Schmidt applied twice), because
    Golub-Kahan without it loses orthogonality within a few tens of steps.
  * Algorithm 3 stops when "k > itermax"; itermax is read as the number of
    restart cycles, and ||R_m|| is the true residual C - M(X_m).
"""
import numpy as np

from .cprod import combine, fro, inner
from .tikhonov import lower_bidiagonal, solve_projected

EPS = np.finfo(np.float64).eps
BREAKDOWN_FACTOR = 64.0


def _cgs2(w, basis):
    """Classical Gram-Schmidt against ``basis``, applied twice."""
    for _ in range(2):
        coef = [inner(b, w) for b in basis]
        for b, c in zip(basis, coef):
            w = w - c * b
    return w


class GKB:
    """Algorithm 4, the tensor discrete cosine Golub-Kahan process.

    alpha[j-1] = alpha_j, beta[j-1] = beta_j (1-based as in the paper);
    U[j-1] = U_j, V[j-1] = V_j.
    """

    def __init__(self, op, C, reorth="none"):
        self.op = op
        self.reorth = reorth
        C = np.asarray(C, dtype=np.float64)
        b1 = fro(C)
        self.beta = [b1]
        self.U = [C / b1]
        t = op.adjoint(self.U[0])
        a1 = fro(t)
        self.alpha = [a1]
        self.V = [t / a1]
        self.steps = 0
        self.breakdown = False
        self.scale = max(a1, b1)

    def step(self):
        """One pass of step 3 (a)-(f); returns False on breakdown."""
        if self.breakdown:
            return False
        j = self.steps  # 0-based index of V_j / U_j / alpha_j
        Ut = self.op.apply(self.V[j]) - self.alpha[j] * self.U[j]
        if self.reorth == "full":
            Ut = _cgs2(Ut, self.U)
        b = fro(Ut)
        self.beta.append(b)
        self.scale = max(self.scale, b)
        if b <= BREAKDOWN_FACTOR * EPS * self.scale:
            self.steps += 1
            self.breakdown = True
            return False
        self.U.append(Ut / b)
        Vt = self.op.adjoint(self.U[j + 1]) - b * self.V[j]
        if self.reorth in ("v", "full"):
            Vt = _cgs2(Vt, self.V)
        a = fro(Vt)
        self.alpha.append(a)
        self.scale = max(self.scale, a)
        self.steps += 1
        if a <= BREAKDOWN_FACTOR * EPS * self.scale:
            self.breakdown = True
            return False
        self.V.append(Vt / a)
        return True

    def bidiagonal(self, k=None):
        k = self.steps if k is None else k
        return lower_bidiagonal(self.alpha, self.beta, k)


def gkb(op, C, k, reorth="none"):
    """Run Algorithm 4 for (at most) k steps."""
    g = GKB(op, C, reorth)
    for _ in range(k):
        if not g.step():
            break
    return g


def dc_lsqr(op, C, k, tol=0.0, reorth="none", history=False):
    """Algorithm 6 (DC-LSQR), X_0 = 0.

    Returns dict with X, iterations, |phibar_{k+1}| (the residual norm), the
    Golub-Kahan scalars, and optionally every iterate X_j.
    """
    g = GKB(op, C, reorth)
    X = np.zeros_like(g.V[0])
    W = g.V[0].copy()
    rhobar = g.alpha[0]
    phibar = g.beta[0]
    hist = []
    its = 0
    status = "ok"
    for j in range(k):
        # (a), (b): one Golub-Kahan step
        ok = g.step()
        bnext = g.beta[j + 1]
        anext = g.alpha[j + 1] if len(g.alpha) > j + 1 else 0.0
        # (c) rotation eliminating beta_{j+1}
        rho = np.sqrt(rhobar ** 2 + bnext ** 2)
        c = rhobar / rho
        s = bnext / rho
        # (d)
        theta = s * anext
        rhobar = c * anext
        # (e)
        phi = c * phibar
        phibar = -s * phibar
        # (f)
        X = X + (phi / rho) * W
        its += 1
        if history:
            hist.append(X.copy())
        if not ok:
            status = "breakdown"
            break
        W = g.V[j + 1] - (theta / rho) * W
        # (g)
        if abs(phibar) < tol:
            break
    return {"X": X, "iters": its, "resnorm": abs(phibar), "alpha": list(g.alpha),
            "beta": list(g.beta), "status": status, "history": hist, "gkb": g}


def dc_gk(op, C, k, lam=None, gcv_mode="rect", reorth="none", target=None):
    """Algorithm 5 (DC-GK): k Golub-Kahan steps, lambda by GCV (lam=None) or
    by the discrepancy principle (gcv_mode 'discrepancy', residual target) or
    fixed, projected Tikhonov solve, X = V_k (*) y (eq. xmlsqr)."""
    g = gkb(op, C, k, reorth)
    kk = g.steps
    B = g.bidiagonal(kk)
    y, lam_used = solve_projected(B, g.beta[0], lam, gcv_mode, target)
    X = combine(g.V[:kk], y)
    return {"X": X, "lambda": lam_used, "iters": kk, "y": y, "alpha": list(g.alpha),
            "beta": list(g.beta), "status": "breakdown" if g.breakdown else "ok", "gkb": g}


class Arnoldi:
    """Algorithm 2, the tensor discrete cosine (global) Arnoldi process.

    ortho='mgs' is the modified Gram-Schmidt loop printed in step 3(b);
    'cgs2' is classical Gram-Schmidt applied twice (same span, better
    orthogonality).  H[i, j] = h_{i+1, j+1}.
    """

    def __init__(self, op, R0, m, ortho="mgs"):
        self.op = op
        self.ortho = ortho
        R0 = np.asarray(R0, dtype=np.float64)
        self.beta = fro(R0)
        self.V = [R0 / self.beta]
        self.H = np.zeros((m + 1, m))
        self.steps = 0
        self.breakdown = False
        self.scale = 0.0

    def step(self):
        if self.breakdown:
            return False
        j = self.steps
        W = self.op.apply(self.V[j])
        if self.ortho == "mgs":
            for i in range(j + 1):
                h = inner(self.V[i], W)
                self.H[i, j] = h
                W = W - h * self.V[i]
        else:
            for _ in range(2):
                coef = [inner(self.V[i], W) for i in range(j + 1)]
                for i in range(j + 1):
                    self.H[i, j] += coef[i]
                    W = W - coef[i] * self.V[i]
        h = fro(W)
        self.H[j + 1, j] = h
        self.scale = max(self.scale, float(np.max(np.abs(self.H[: j + 2, j]))))
        self.steps += 1
        if h <= BREAKDOWN_FACTOR * EPS * self.scale:
            self.breakdown = True
            return False
        self.V.append(W / h)
        return True

    def hessenberg(self):
        m = self.steps
        return self.H[: m + 1, :m]


def dc_gmres(op, C, X0, m, cycles, lam=None, gcv_mode="rect", tol=0.0, ortho="mgs"):
    """Algorithm 3, DC-GMRES(m) with Tikhonov/GCV on every cycle.

    Each cycle: R_0 = C - M(X_0); m Arnoldi steps on R_0; lambda by GCV
    (lam=None) or fixed; y from eq. (leastsq); X_m = X_0 + V_m (*) y.  Runs
    ``cycles`` cycles unless ||R_m|| < tol.
    """
    C = np.asarray(C, dtype=np.float64)
    X = np.asarray(X0, dtype=np.float64).copy()
    lams = []
    status = "ok"
    R = C - op.apply(X)
    total = 0
    for _ in range(cycles):
        ar = Arnoldi(op, R, m, ortho)
        if ar.beta == 0.0:
            break
        for _ in range(m):
            if not ar.step():
                break
        total += ar.steps
        Hm = ar.hessenberg()
        y, lam_used = solve_projected(Hm, ar.beta, lam, gcv_mode)
        lams.append(lam_used)
        X = X + combine(ar.V[: ar.steps], y)
        R = C - op.apply(X)
        if ar.breakdown:
            status = "breakdown"
        if fro(R) < tol:
            break
    return {"X": X, "lambdas": lams, "resnorm": fro(R), "steps": total, "status": status}
