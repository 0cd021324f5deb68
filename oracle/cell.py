"""The periodic cell problem: the shift sigma and the cell eigenfunction psi.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

§1 eq:cell-problem and §2 eq:weak-form-cell-problem: on the unit cell
(0,1)^p x (0,ell)^q, with periodic conditions in every x direction and zero
Dirichlet conditions in y, (psi, sigma) is the lowest eigenpair of
(K# + MV#) psi = sigma M# psi.  psi is taken positive (the ground state of
the periodic problem has one sign) and M#-normalised.  Its periodic
extension to Omega_L is psi_ext(i_x, i_y) = psi(i_x mod n_e, i_y) (§2,
periodic extension of the cell vector).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .fem import Grid, assemble_elements, assemble_kron
from .potential import vfun, kron_terms

DENSE_LIMIT = 6000


def cell_matrices(p, q, ne, spec, ell=1, nq=2, route="elements"):
    g = Grid(p, q, 1, ne, ell=ell, cell=True)
    if route == "elements":
        K, M, MV = assemble_elements(g, vfun(spec, p, q, ell), nq=nq)
    else:
        K, M, MV = assemble_kron(g, kron_terms(spec, p, q, ell), nq=nq)
    return g, K, M, MV


def cell_problem(p, q, ne, spec, ell=1, nq=2, route="elements"):
    """Returns dict(sigma, sigma2, psi (cell vector, canonical cell order), grid)."""
    g, K, M, MV = cell_matrices(p, q, ne, spec, ell, nq, route)
    A = (K + MV).tocsc()
    if g.n <= DENSE_LIMIT:
        w, v = sla.eigh(A.toarray(), M.toarray(), subset_by_index=[0, 1])
    else:
        # all eigenvalues exceed min V (K is PSD and the 2-point rule is exact for
        # the mass matrix, so MV >= min(V at quadrature points) M): shift below it.
        vmin = _vmin(g, spec, nq)
        w, v = spla.eigsh(A, k=2, M=M.tocsc(), sigma=vmin - 1.0, which="LM")
        order = np.argsort(w)
        w, v = w[order], v[:, order]
    psi = v[:, 0].copy()
    if psi.sum() < 0:
        psi = -psi
    psi /= np.sqrt(psi @ (M @ psi))
    return dict(sigma=float(w[0]), sigma2=float(w[1]), psi=psi, grid=g, K=K, M=M, MV=MV)


def _vmin(g, spec, nq):
    from .fem import _element_quad_points
    _, coords, _, _ = _element_quad_points(g, nq)
    return float(np.min(vfun(spec, g.p, g.q, g.ell)(coords)))


def extend_periodic(psi_cell, grid):
    """psi_ext on the interior unknowns of ``grid`` (canonical order)."""
    ne = grid.ne
    axes = []
    for a in range(grid.d):
        i = np.arange(1, grid.nel[a])  # 1-based interior node index
        axes.append(np.mod(i, ne) if a < grid.p else i - 1)
    cell_dims = [ne] * grid.p + [grid.nel[grid.p + j] - 1 for j in range(grid.q)]
    mesh = np.meshgrid(*axes, indexing="ij")
    lin = np.zeros(mesh[0].shape, dtype=np.int64)
    stride = 1
    for a in range(grid.d):
        lin += mesh[a] * stride
        stride *= cell_dims[a]
    return psi_cell[lin.ravel(order="F")]
