"""Preconditioned conjugate gradients for the shifted system A_sigma x = b.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Hestenes-Stiefel PCG as used for the inner solves of §2.1 and analysed in §3
(eq:cg-energy-norm-error-reduction); the stopping rule is the relative
2-norm of the unpreconditioned residual, ||r_k|| <= rtol ||r_0|| (§4.1).

Breakdown: A_sigma and the two-level additive Schwarz preconditioner are SPD
(§3), so p.A_sigma p <= 0 or r.z <= 0 can only come from an indefinite
operator or preconditioner; both are reported rather than hidden.
"""
import numpy as np


class PCGResult:
    def __init__(self, x, iters, status, hist, alphas, betas):
        self.x = x
        self.iters = iters
        self.status = status          # "ok", "maxit", "not_spd"
        self.hist = np.asarray(hist)  # ||r_k|| / ||r_0||, k = 0..iters
        self.alphas = np.asarray(alphas)
        self.betas = np.asarray(betas)


def pcg(apply_A, b, apply_M=None, x0=None, rtol=1e-10, maxit=1000):
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x) if x0 is not None else b.copy()
    r0n = np.linalg.norm(r)
    hist = [1.0]
    alphas, betas = [], []
    if r0n == 0.0:
        return PCGResult(x, 0, "ok", hist, alphas, betas)
    z = apply_M(r) if apply_M is not None else r.copy()
    rho = float(r @ z)
    if rho <= 0.0:
        return PCGResult(x, 0, "not_spd", hist, alphas, betas)
    p = z.copy()
    for k in range(1, maxit + 1):
        q = apply_A(p)
        gamma = float(p @ q)
        if gamma <= 0.0:
            return PCGResult(x, k - 1, "not_spd", hist, alphas, betas)
        alpha = rho / gamma
        x += alpha * p
        r -= alpha * q
        alphas.append(alpha)
        rn = np.linalg.norm(r)
        hist.append(rn / r0n)
        if rn <= rtol * r0n:
            return PCGResult(x, k, "ok", hist, alphas, betas)
        z = apply_M(r) if apply_M is not None else r.copy()
        rho_new = float(r @ z)
        if rho_new <= 0.0:
            return PCGResult(x, k, "not_spd", hist, alphas, betas)
        beta = rho_new / rho
        betas.append(beta)
        p = z + beta * p
        rho = rho_new
    return PCGResult(x, maxit, "maxit", hist, alphas, betas)


def lanczos_extremes(alphas, betas):
    """Ritz values of M^{-1} A_sigma from the CG coefficients (the Lanczos
    tridiagonal: T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T_{j,j+1} = sqrt(beta_j)/alpha_j).  Returns (lambda_min, lambda_max)."""
    k = len(alphas)
    if k == 0:
        return np.nan, np.nan
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j]
        if j > 0:
            T[j, j] += betas[j - 1] / alphas[j - 1]
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    w = np.linalg.eigvalsh(T)
    return float(w[0]), float(w[-1])
