"""Restricted additive Schwarz, the stationary RAS iteration and GMRES.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

eq:dd-preconditioners: M_RAS,1^{-1} = sum_i R_i^T D_i A_i^{-1} R_i, with the
partition of unity D_i of §2.2 (sum_i R_i^T D_i R_i = I) and exact local
solves; eq:two-level-preconditioners adds the coarse correction
R_0^T A_0^{-1} R_0 additively (M_RAS,2).  eq:stationary-ras is the fixed-point
iteration x_{k+1} = x_k + M_RAS,1^{-1} r_k; eq:two-level-stationary-ras-mult-cc
follows each such half step by the coarse correction of the new residual.
M_RAS,2 is not symmetric, so the Krylov method that uses it is GMRES (§3),
here with right preconditioning: x = x_0 + M^{-1} V y, y minimising
||beta e_1 - H y|| over the Arnoldi basis V of A M^{-1} (modified
Gram-Schmidt), Givens rotations for the small least-squares problem.

Readings: every solver stops when ||b - A x_k||_2 <= rtol ||b - A x_0||_2 (GMRES
uses its recurrence residual, which equals it in exact arithmetic); GMRES
restarts after `restart` steps (the paper reports no restart); the iteration
count of the stationary methods counts full steps (a half step and its coarse
correction are one step).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .dd import restriction


class RestrictedAdditiveSchwarz:
    """apply(r) = sum_i R_i^T D_i A_i^{-1} R_i r (+ R_0^T A_0^{-1} R_0 r if two-level)."""

    def __init__(self, A_sigma, subs, D, R0T=None):
        A = sp.csr_matrix(A_sigma)
        self.n = A.shape[0]
        self.R = [restriction(self.n, s) for s in subs]
        self.D = [np.asarray(d, dtype=np.float64) for d in D]
        self.local = [spla.splu((R @ A @ R.T).tocsc(), permc_spec="MMD_AT_PLUS_A") for R in self.R]
        self.R0T = None
        if R0T is not None:
            self.R0T = sp.csc_matrix(R0T)
            A0 = (self.R0T.T @ A @ self.R0T).toarray()
            self.A0 = 0.5 * (A0 + A0.T)

    def local_part(self, r):
        z = np.zeros(self.n)
        for R, d, lu in zip(self.R, self.D, self.local):
            z += R.T @ (d * lu.solve(R @ r))
        return z

    def coarse_part(self, r):
        return self.R0T @ np.linalg.solve(self.A0, self.R0T.T @ r)

    def apply(self, r):
        z = self.local_part(r)
        if self.R0T is not None:
            z += self.coarse_part(r)
        return z


def stationary_ras(A, b, ras, two_level=True, rtol=1e-8, maxit=10000):
    """eq:stationary-ras (two_level=False) or eq:two-level-stationary-ras-mult-cc.

    Returns dict(x, iters, hist (||r_k|| / ||r_0||), status)."""
    x = np.zeros(b.size)
    r = b.copy()
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return dict(x=x, iters=0, hist=np.array(hist), status="ok")
    for k in range(1, maxit + 1):
        x = x + ras.local_part(r)
        r = b - A @ x
        if two_level:
            x = x + ras.coarse_part(r)
            r = b - A @ x
        hist.append(np.linalg.norm(r) / r0)
        if hist[-1] <= rtol:
            return dict(x=x, iters=k, hist=np.array(hist), status="ok")
    return dict(x=x, iters=maxit, hist=np.array(hist), status="maxit")


def gmres_right(A, b, apply_M=None, rtol=1e-8, maxit=10000, restart=1000):
    """Right-preconditioned restarted GMRES from x_0 = 0.

    Returns dict(x, iters, hist (recurrence ||r_k|| / ||r_0||), status)."""
    n = b.size
    M = apply_M if apply_M is not None else (lambda v: v)
    x = np.zeros(n)
    r = b.copy()
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return dict(x=x, iters=0, hist=np.array(hist), status="ok")
    its = 0
    while its < maxit:
        beta = np.linalg.norm(r)
        m = min(restart, maxit - its)
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(m):
            w = A @ M(V[:, j])
            for i in range(j + 1):           # modified Gram-Schmidt
                H[i, j] = w @ V[:, i]
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):               # previous rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / r0)
            if hist[-1] <= rtol:
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):  # back substitution
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:]) / H[i, i]
        x = x + M(V[:, :j_done] @ y)
        r = b - A @ x
        if hist[-1] <= rtol:
            return dict(x=x, iters=its, hist=np.array(hist), status="ok")
    return dict(x=x, iters=its, hist=np.array(hist), status="maxit")
