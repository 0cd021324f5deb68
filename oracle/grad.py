"""Derivatives with respect to the potential parameters (beyond the paper).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

theta = (a_1..a_T, phi_1..phi_T) of a sep_fourier or fourier2 potential.
A(theta) = K + M_{V(theta)} (§2, eq:discrete-weak-form) depends on theta only
through the potential mass matrix, which is linear in V, so
dA/dtheta_j = M_{dV/dtheta_j} with the same quadrature.  Here dV/dtheta_j is
written out directly (the phase derivative as -a_t sin(...)) and the weighted
mass matrix comes from the element-loop assembly.

  eigenvalue (Hellmann-Feynman):  dlambda/dtheta = x^T M_{dV} x / x^T M x
  shift (eq:cell-problem):        dsigma/dtheta  = psi^T M#_{dV} psi / psi^T M# psi
  solve u = A_sigma^{-1} b, l(u): dl/dtheta = -w^T (M_{dV} - dsigma/dtheta M) u,
                                  A_sigma w = dl/du  (A_sigma symmetric)
"""
import numpy as np

from .fem import Grid, assemble_elements

TWO_PI = 2.0 * np.pi


def dv_functions(spec, p, q, ell=1):
    """[dV/da_1, .., dV/da_T, dV/dphi_1, .., dV/dphi_T] as vectorised functions of the coordinates."""
    kind = spec["kind"]
    a = np.asarray(spec["a"], float)
    ph = np.asarray(spec["phi"], float)
    k = np.asarray(spec["k"], float)
    if kind == "sep_fourier":
        cy = float(spec["cy"])

        def envelope(z):
            if q == 0:
                return np.full_like(z[0], 1.0 + cy, dtype=np.float64)
            G = np.ones_like(z[0], dtype=np.float64)
            for j in range(q):
                G = G * np.sin(np.pi * z[p + j] / ell)
            return 1.0 + cy * G

        def arg(z, t):
            return TWO_PI * k[t] * z[0] + ph[t]
    elif kind == "fourier2":
        m = np.asarray(spec["m"], float)

        def envelope(z):
            return np.ones_like(z[0], dtype=np.float64)

        def arg(z, t):
            return TWO_PI * (k[t] * z[0] + m[t] * z[1]) + ph[t]
    else:
        raise ValueError(f"no Fourier parameters in a {kind!r} potential")
    T = a.size
    out = []
    for t in range(T):
        out.append(lambda z, t=t: np.cos(arg(z, t)) * envelope(z))
    for t in range(T):
        out.append(lambda z, t=t: -a[t] * np.sin(arg(z, t)) * envelope(z))
    return out


def weighted_mass(grid, f, nq=2):
    """M_f: the mass matrix weighted by f (element assembly, nq Gauss points per direction)."""
    _, _, Mf = assemble_elements(grid, f, nq=nq, with_kinetic=False)
    return Mf


def derivative_matrices(grid, spec, nq=2):
    return [weighted_mass(grid, f, nq) for f in dv_functions(spec, grid.p, grid.q, grid.ell)]


def eigenvalue_grad(grid, M, x, spec, nq=2):
    """Hellmann-Feynman: dlambda/dtheta_j = x^T M_{dV_j} x / x^T M x."""
    xmx = float(x @ (M @ x))
    return np.array([float(x @ (D @ x)) for D in derivative_matrices(grid, spec, nq)]) / xmx


def shift_grad(cell, spec, nq=2):
    """dsigma/dtheta from the oracle cell problem (dict of cell.cell_problem)."""
    g, M, psi = cell["grid"], cell["M"], cell["psi"]
    return eigenvalue_grad(g, M, psi, spec, nq)


def solve_grad(grid, M, u, w, spec, dsigma, nq=2):
    """dl/dtheta = -w^T (M_{dV} - dsigma M) u for u = A_sigma^{-1} b and A_sigma w = dl/du."""
    wmu = float(w @ (M @ u))
    vals = np.array([float(w @ (D @ u)) for D in derivative_matrices(grid, spec, nq)])
    return -(vals - np.asarray(dsigma) * wmu)


def grid_of(cfg):
    return Grid(cfg["p"], cfg["q"], cfg["L"], cfg["ne"], ell=cfg.get("ell", 1))
