"""Inexact shift-and-invert preconditioned LOPCG (alg:si-lopcg).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

§2.1: the smallest eigenpair of A x = lambda B x is the minimiser of the
Rayleigh quotient R(y) = y^T A y / y^T B y.  Each outer step takes the
spectral residual r_k = A x_k - R(x_k) B x_k, preconditions it with the shift
and invert operator, w_k ~ A_sigma^{-1} r_k (an inner solve to a tolerance),
and minimises R over span{w_k, x_k, x_{k-1}} by Rayleigh-Ritz in a
B-orthonormal basis of that span; the minimiser is B-normalised and becomes
x_{k+1}.  The loop runs while ||r_k||_2 > TOL_o and k <= k_max (the printed
test of the loop is inverted; this is the intended reading).

Readings (the paper gives no details of these steps):
- orthogonalised Rayleigh-Ritz: span{w_k, x_k, x_{k-1}} = span{x_k, w~, p~}
  with p = x_k - x_{k-1} and w~, p~ the parts of w_k and p that are
  B-orthogonal to the B-normalised x_k (formed on the vectors, so that the
  small differences near convergence keep their digits); with S = [x_k, w~,
  p~] scaled to unit B-norm columns, the eigenvectors of G_B = S^T B S with
  eigenvalue above 1e-10 times its largest give a B-orthonormal basis S T
  of the directions S represents numerically, and the smallest eigenpair of
  T^T (S^T A S) T gives the coefficients;
- the Ritz vector's sign is fixed so that 1^T B x > 0 (as in ipm.py);
- inner solves: from a zero guess with a relative tolerance, either fixed or
  adaptive, rtol_k = min(0.1, ||r_k||_2) (§4.3), by PCG or by any other solver
  of A_sigma w = r_k passed in (GMRES+RAS2 or the stationary RAS iterations of
  §4.2, from ras.py); the fused variant skips the inner solve and applies the
  preconditioner once, w_k = M^{-1} r_k (§4.3, with M_RAS,2 there).
"""
import numpy as np
import scipy.linalg as sla

from .pcg import pcg

DROP = 1e-10


def rayleigh_ritz(S, AS, BS):
    """Coefficients c of the Ritz vector S c minimising R over span(S), and its Ritz value.

    Columns of S with zero B-norm are ignored; the others are scaled to unit
    B-norm before the directions S represents numerically are selected."""
    GB = S.T @ BS
    GA = S.T @ AS
    GB = 0.5 * (GB + GB.T)
    GA = 0.5 * (GA + GA.T)
    d = np.sqrt(np.maximum(np.diag(GB), 0.0))
    sc = np.where(d > 0.0, 1.0 / np.where(d > 0.0, d, 1.0), 0.0)
    GB = GB * np.outer(sc, sc)
    GA = GA * np.outer(sc, sc)
    ev, V = np.linalg.eigh(GB)
    keep = ev > DROP * ev.max()
    T = V[:, keep] / np.sqrt(ev[keep])
    H = T.T @ GA @ T
    mu, Y = np.linalg.eigh(0.5 * (H + H.T))
    return sc * (T @ Y[:, 0]), float(mu[0])


def si_lopcg(A, B, sigma, x0, x1, tol_o=1e-8, kmax=200, mode="fixed", rtol_i=1e-8,
             maxit_i=10000, precond=None, inner_solve=None):
    """Returns dict(lam, x, its, inner (per outer step), res_hist).

    mode: "fixed" (inner solve to rtol_i), "adaptive" (to min(0.1, ||r||_2)),
    "fused" (w = precond(r)).  precond(v) applies the preconditioner M^{-1}.
    inner_solve(rhs, rtol, maxit) -> (w, iterations) replaces the default PCG
    with precond.
    """
    A_sigma = (A - sigma * B).tocsr()

    def bnorm(v):
        return float(np.sqrt(v @ (B @ v)))

    x_prev = np.array(x0, dtype=np.float64) / bnorm(x0)
    x = np.array(x1, dtype=np.float64) / bnorm(x1)
    lam = float(x @ (A @ x))
    r = A @ x - lam * (B @ x)
    res = [float(np.linalg.norm(r))]
    inner = []
    k = 1
    while res[-1] > tol_o and k <= kmax:
        if mode == "fused":
            w = precond(r)
            inner.append(1)
        else:
            rt = rtol_i if mode == "fixed" else min(0.1, res[-1])
            if inner_solve is None:
                out = pcg(lambda v: A_sigma @ v, r, precond, rtol=rt, maxit=maxit_i)
                w, its = out.x, out.iters
            else:
                w, its = inner_solve(r, rt, maxit_i)
            inner.append(its)
        Bx = B @ x
        wt = w - (Bx @ w) * x
        p = x - x_prev
        pt = p - (Bx @ p) * x
        S = np.column_stack([x, wt, pt])
        c, _ = rayleigh_ritz(S, A @ S, B @ S)
        xn = S @ c
        xn /= bnorm(xn)
        if np.sum(B @ xn) < 0:
            xn = -xn
        x_prev, x = x, xn
        lam = float(x @ (A @ x))
        r = A @ x - lam * (B @ x)
        res.append(float(np.linalg.norm(r)))
        k += 1
    return dict(lam=lam, x=x, its=k - 1, inner=np.array(inner, dtype=int), res_hist=np.array(res))


def unit_first(n):
    """x_0 = e_1 of the experiments of §4.2."""
    e = np.zeros(n)
    e[0] = 1.0
    return e
