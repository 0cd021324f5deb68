"""sigma-shifted inverse iteration (inverse power method) with B-normalisation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

§2 and §2.1: x_{k+1} = A_sigma^{-1} B x_k, then B-normalise, with the
quasi-optimal shift sigma of the cell problem; the eigenvalue is the
Rayleigh quotient R(x) = x^T A x / x^T B x (§2.1), evaluated as
sigma + x^T A_sigma x for a B-normalised x.  B is the mass matrix M here.

Readings: start vector 1/||1||_M (the start vector of the LOPCG experiments
in §4.2); sign fixed so that 1^T M x > 0; stop when ||x_{k+1} - x_k||_M
<= tol (the paper fixes no stopping rule for the plain inverse iteration).

The linear solves are either exact (a direct factorisation of A_sigma:
banded Cholesky with the fixed direction fastest for a 2-D grid passed as
`grid`, SuperLU without a grid) or PCG with a supplied preconditioner.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .pcg import pcg


class DirectSolver:
    """Exact solves with A_sigma (SPD)."""

    def __init__(self, A_sigma, grid=None):
        A = sp.csr_matrix(A_sigma)
        self.n = A.shape[0]
        self.kind = "splu"
        perm = bw = None
        if grid is not None and grid.d == 2:
            # reorder with y fastest: half-bandwidth = number of y unknowns + 1
            nx, ny = grid.ndof_dir
            perm = np.arange(self.n).reshape(ny, nx).T.ravel()
            bw = ny + 1
        elif grid is not None:
            raise ValueError("the banded route is for 2-D grids; pass grid=None for SuperLU")
        if perm is not None:
            Ap = A[perm][:, perm].tocsr()
            ab = np.zeros((bw + 1, self.n))
            coo = Ap.tocoo()
            keep = coo.row >= coo.col
            if np.any(coo.row[keep] - coo.col[keep] > bw):
                raise AssertionError("band estimate too small")
            ab[coo.row[keep] - coo.col[keep], coo.col[keep]] = coo.data[keep]
            del coo, Ap
            self.cb = sla.cholesky_banded(ab, lower=True, overwrite_ab=True)
            self.perm = perm
            self.kind = "banded"
        else:
            self.lu = spla.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A",
                                diag_pivot_thresh=0.0, options={"SymmetricMode": True})

    def solve(self, b):
        if self.kind == "banded":
            y = sla.cho_solve_banded((self.cb, True), b[self.perm])
            x = np.empty_like(y)
            x[self.perm] = y
            return x
        return self.lu.solve(b)


def inverse_iteration(A, M, sigma, solve, x0=None, tol=1e-13, maxit=100):
    """Returns dict(lam, x, its, dx_hist, inner) ; ``solve(b)`` returns (u, inner_iters)."""
    A_sigma = (A - sigma * M).tocsr()
    n = A.shape[0]
    if x0 is None:
        x = np.ones(n)
    else:
        x = np.array(x0, dtype=np.float64)
    x /= np.sqrt(x @ (M @ x))
    dx_hist, inner = [], []
    lam = sigma + x @ (A_sigma @ x)
    for k in range(1, maxit + 1):
        b = M @ x
        u, it = solve(b)
        inner.append(it)
        xn = u / np.sqrt(u @ (M @ u))
        if np.sum(M @ xn) < 0:
            xn = -xn
        d = xn - x
        dxn = float(np.sqrt(d @ (M @ d)))
        dx_hist.append(dxn)
        x = xn
        lam = sigma + x @ (A_sigma @ x)
        if dxn <= tol:
            break
    return dict(lam=float(lam), x=x, its=len(dx_hist), dx_hist=np.array(dx_hist),
                inner=np.array(inner))


def inverse_iteration_direct(A, M, sigma, grid=None, **kw):
    ds = DirectSolver((A - sigma * M), grid)
    return inverse_iteration(A, M, sigma, lambda b: (ds.solve(b), 0), **kw)


def inverse_iteration_pcg(A, M, sigma, precond_apply, rtol=1e-10, maxit_inner=1000, **kw):
    A_sigma = (A - sigma * M).tocsr()

    def solve(b):
        res = pcg(lambda v: A_sigma @ v, b, precond_apply, rtol=rtol, maxit=maxit_inner)
        if res.status == "not_spd":
            raise RuntimeError("PCG breakdown in inverse iteration")
        return res.x, res.iters
    return inverse_iteration(A, M, sigma, solve, **kw)


def spectral_residual(A, M, lam, x):
    """||A x - lambda M x||_2 (§2.1)."""
    return float(np.linalg.norm(A @ x - lam * (M @ x)))
