"""Q1 finite elements for -Laplace(phi) + V phi = lambda phi on (0,L)^p x (0,ell)^q.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain FP64 CPU oracle
that the GPU library is checked against.  Only ``tests/``, the smoke check
and the CPU-baseline leg of the benchmark may import it; the library never
does, and the two share no code.

Follows §2 of the paper (Galerkin scheme, discrete weak form
eq:discrete-weak-form and its matrix form A x = lambda B x) and §4.1 / §4.3,
which use Q1 elements on Cartesian grids built from translated copies of the
unit-cell mesh.  Notation: K stiffness, M mass (the paper's B), MV the
potential mass, so the paper's A is K + MV.

Ordering of unknowns ("canonical"): interior nodes only (homogeneous
Dirichlet nodes are eliminated), x1 fastest, then x2 (if p = 2), then y1,
then y2.  A node index i runs over 1..(nel-1) in each direction, where nel is
the number of elements along that direction.

Two assembly routes are provided so that each can pin the other:
  * ``assemble_elements``: a vectorised loop over elements into COO/CSR
    (any potential);
  * ``assemble_kron``: Kronecker sums of 1-D matrices, exact for potentials
    that are finite sums of products of 1-D functions (every workload here).

Quadrature of the potential term: tensor Gauss-Legendre with ``nq`` points
per direction and element; V is evaluated at cell-local x coordinates
((element index mod n_e) * h + offset) so that the discrete operator is
exactly periodic, as assumption (A1) of §1 makes the continuous one.
"""
import itertools
import math

import numpy as np
import scipy.sparse as sp

__all__ = ["Grid", "gauss_legendre01", "element_1d", "assemble_elements",
           "assemble_kron", "mass_1d_weighted", "interior_coords"]


def gauss_legendre01(nq):
    """Gauss-Legendre points and weights on [0, 1] (weights sum to 1)."""
    xi, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (xi + 1.0), 0.5 * w


def element_1d(h):
    """1-D linear element stiffness k_e and mass m_e on an element of length h."""
    k = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    m = np.array([[2.0, 1.0], [1.0, 2.0]]) * (h / 6.0)
    return k, m


class Grid:
    """Uniform Cartesian Q1 grid of Omega_L = (0,L)^p x (0,ell)^q (eq:geometry-description).

    ``cell=True`` builds the unit-cell grid (0,1)^p x (0,ell)^q of the cell
    problem eq:cell-problem, periodic in every x direction: x node indices run
    over 0..n_e-1 and node n_e is identified with node 0.
    """

    def __init__(self, p, q, L, ne, ell=1, cell=False):
        if p < 1 or q < 0 or p + q > 3:
            raise ValueError("need p >= 1, q >= 0, p + q <= 3")
        self.p, self.q, self.d = p, q, p + q
        self.ne = int(ne)
        self.h = 1.0 / self.ne
        self.L = 1 if cell else int(L)
        # ell is real (eq:geometry-description); the mesh needs ell n_e elements
        self.ell = float(ell)
        nely = int(round(self.ell * self.ne))
        if abs(nely - self.ell * self.ne) > 1e-9:
            raise ValueError("ell * n_e must be an integer")
        self.cell = cell
        self.nel = [self.L * self.ne] * p + [nely] * q
        self.periodic = [cell] * p + [False] * q
        # number of unknowns per direction
        self.ndof_dir = [self.ne if per else m - 1
                         for m, per in zip(self.nel, self.periodic)]
        self.n = int(np.prod(self.ndof_dir))

    def dof_of_node(self, g, axis):
        """Map grid node index g (0..nel) along ``axis`` to an unknown index, -1 if Dirichlet."""
        g = np.asarray(g)
        if self.periodic[axis]:
            return np.mod(g, self.ne)
        out = g - 1
        return np.where((g >= 1) & (g <= self.nel[axis] - 1), out, -1)

    def linear_index(self, idx):
        """Canonical linear index from per-direction unknown indices (x1 fastest)."""
        lin = np.zeros_like(np.asarray(idx[0]))
        stride = 1
        for a in range(self.d):
            lin = lin + np.asarray(idx[a]) * stride
            stride *= self.ndof_dir[a]
        return lin


def interior_coords(grid):
    """Coordinates (one array per direction) of the unknowns in canonical order."""
    axes = []
    for a in range(grid.d):
        if grid.periodic[a]:
            axes.append(np.arange(grid.ne) * grid.h)
        else:
            axes.append(np.arange(1, grid.nel[a]) * grid.h)
    mesh = np.meshgrid(*axes, indexing="ij")
    # canonical order has axis 0 fastest: ravel in Fortran order
    return [m.ravel(order="F") for m in mesh]


def _element_quad_points(grid, nq):
    """Per element and quadrature point: coordinates used to evaluate V.

    Returns (elem_index arrays per axis, coords per axis with shape
    (nelem, nq^d), weights (nq^d,), reference points per axis (nq^d,)).
    x coordinates are cell-local: (e mod n_e) * h + h * xi.
    """
    xi, w = gauss_legendre01(nq)
    h = grid.h
    e_axes = [np.arange(m) for m in grid.nel]
    E = np.meshgrid(*e_axes, indexing="ij")
    E = [e.ravel(order="F") for e in E]
    Q = list(itertools.product(range(nq), repeat=grid.d))
    qxi = np.array([[xi[qq[a]] for a in range(grid.d)] for qq in Q])  # (nQ, d)
    qw = np.array([np.prod([w[qq[a]] for a in range(grid.d)]) for qq in Q])
    coords = []
    for a in range(grid.d):
        if a < grid.p:
            base = np.mod(E[a], grid.ne) * h
        else:
            base = E[a] * h
        coords.append(base[:, None] + h * qxi[None, :, a])
    return E, coords, qw, qxi


def assemble_elements(grid, vfun, nq=2, with_kinetic=True):
    """Route (i): element loop.  Returns (K, M, MV) as CSR matrices.

    vfun(coords) takes a list of d coordinate arrays (x cell-local) and returns
    V at those points.  Element matrices: stiffness sum over directions of
    k_e (x) m_e (x) ..., mass m_e (x) ... (x) m_e, potential mass by tensor
    Gauss-Legendre quadrature with nq points per direction.
    """
    d, h = grid.d, grid.h
    ke, me = element_1d(h)
    corners = list(itertools.product((0, 1), repeat=d))  # local node a, axis 0 first
    nloc = len(corners)
    # element stiffness and mass (same for every element)
    Ke = np.zeros((nloc, nloc))
    Me = np.zeros((nloc, nloc))
    for ia, a in enumerate(corners):
        for ib, b in enumerate(corners):
            mm = 1.0
            for ax in range(d):
                mm *= me[a[ax], b[ax]]
            Me[ia, ib] = mm
            ss = 0.0
            for dirn in range(d):
                t = 1.0
                for ax in range(d):
                    t *= (ke if ax == dirn else me)[a[ax], b[ax]]
                ss += t
            Ke[ia, ib] = ss
    E, coords, qw, qxi = _element_quad_points(grid, nq)
    nelem = E[0].size
    V = np.asarray(vfun(coords), dtype=np.float64).reshape(nelem, -1)
    # shape functions at the reference quadrature points: N_a(xi) = prod (xi or 1-xi)
    N = np.ones((qxi.shape[0], nloc))
    for ia, a in enumerate(corners):
        for ax in range(d):
            N[:, ia] *= qxi[:, ax] if a[ax] else (1.0 - qxi[:, ax])
    B = (qw[:, None, None] * N[:, :, None] * N[:, None, :]) * h ** d  # (nQ, nloc, nloc)
    MVe = (V @ B.reshape(B.shape[0], -1)).reshape(nelem, nloc, nloc)
    # global unknown index of each element corner
    gidx = np.empty((nelem, nloc), dtype=np.int64)
    valid = np.ones((nelem, nloc), dtype=bool)
    for ia, a in enumerate(corners):
        per_axis = []
        for ax in range(d):
            u = grid.dof_of_node(E[ax] + a[ax], ax)
            valid[:, ia] &= u >= 0
            per_axis.append(np.maximum(u, 0))
        gidx[:, ia] = grid.linear_index(per_axis)
    rows = np.repeat(gidx[:, :, None], nloc, axis=2)
    cols = np.repeat(gidx[:, None, :], nloc, axis=1)
    ok = valid[:, :, None] & valid[:, None, :]
    r, c = rows[ok], cols[ok]
    n = grid.n

    def build(vals):
        return sp.csr_matrix((vals[ok], (r, c)), shape=(n, n))

    MV = build(MVe)
    M = build(np.broadcast_to(Me, MVe.shape))
    K = build(np.broadcast_to(Ke, MVe.shape)) if with_kinetic else None
    for A in (MV, M, K):
        if A is not None:
            A.sum_duplicates()
    return K, M, MV


def mass_1d_weighted(nel, h, f, nq, periodic=False, ne=None, dirichlet=True, cell_local=True):
    """1-D weighted mass matrix int f N_i N_j by nq-point Gauss-Legendre per element.

    ``nel`` elements of length h.  Dirichlet: unknowns are nodes 1..nel-1.
    Periodic: unknowns are nodes 0..nel-1 with node nel == node 0.  With
    ``cell_local`` the element coordinate is (e mod ne) * h (x directions).
    f=None gives the plain mass matrix.
    """
    xi, w = gauss_legendre01(nq)
    e = np.arange(nel)
    base = (np.mod(e, ne) if cell_local else e) * h
    pts = base[:, None] + h * xi[None, :]
    fv = np.ones_like(pts) if f is None else np.asarray(f(pts), dtype=np.float64)
    N0 = 1.0 - xi
    N1 = xi
    m00 = h * (fv * (w * N0 * N0)).sum(axis=1)
    m01 = h * (fv * (w * N0 * N1)).sum(axis=1)
    m11 = h * (fv * (w * N1 * N1)).sum(axis=1)
    return _assemble_1d(nel, m00, m01, m11, periodic)


def stiffness_1d(nel, h, periodic=False):
    v = np.full(nel, 1.0 / h)
    return _assemble_1d(nel, v, -v, v, periodic)


def _assemble_1d(nel, a00, a01, a11, periodic):
    e = np.arange(nel)
    left, right = e, e + 1
    if periodic:
        right = np.mod(right, nel)
        n = nel
        li, ri = left, right
        keep_l = np.ones(nel, bool)
        keep_r = np.ones(nel, bool)
    else:
        n = nel - 1
        li, ri = left - 1, right - 1
        keep_l = li >= 0
        keep_r = ri <= n - 1
    rows, cols, vals = [], [], []
    for (ri_, ci_, v, kr, kc) in ((li, li, a00, keep_l, keep_l), (li, ri, a01, keep_l, keep_r),
                                  (ri, li, a01, keep_r, keep_l), (ri, ri, a11, keep_r, keep_r)):
        ok = kr & kc
        rows.append(ri_[ok]); cols.append(ci_[ok]); vals.append(v[ok])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    A.sum_duplicates()
    return A


def _kron_list(mats):
    """Kronecker product with mats[0] the fastest index (canonical order)."""
    out = mats[0]
    for m in mats[1:]:
        out = sp.kron(m, out, format="csr")
    return out


def assemble_kron(grid, terms, nq=2):
    """Route (ii): Kronecker sums of 1-D matrices.

    ``terms`` is a list of (coef, [f_0, ..., f_{d-1}]) meaning
    V(z) = sum coef * prod_a f_a(z_a), where f_a is a vectorised 1-D function
    or None (constant 1).  With tensor Gauss-Legendre quadrature the potential
    mass of such a V factorises exactly into Kronecker products of 1-D
    weighted mass matrices.  Returns (K, M, MV).
    """
    d, h = grid.d, grid.h
    Mass, Stiff = [], []
    for a in range(d):
        per = grid.periodic[a]
        Mass.append(mass_1d_weighted(grid.nel[a], h, None, nq, periodic=per, ne=grid.ne))
        Stiff.append(stiffness_1d(grid.nel[a], h, periodic=per))
    M = _kron_list(Mass)
    K = None
    for dirn in range(d):
        t = _kron_list([Stiff[a] if a == dirn else Mass[a] for a in range(d)])
        K = t if K is None else K + t
    MV = sp.csr_matrix((grid.n, grid.n))
    for coef, fs in terms:
        mats = []
        for a in range(d):
            f = fs[a]
            if f is None:
                mats.append(Mass[a])
            else:
                mats.append(mass_1d_weighted(grid.nel[a], h, f, nq, periodic=grid.periodic[a],
                                             ne=grid.ne, cell_local=(a < grid.p)))
        MV = MV + coef * _kron_list(mats)
    return K.tocsr(), M.tocsr(), MV.tocsr()
