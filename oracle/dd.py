"""Overlapping decomposition, partitions of unity, PerFact coarse space, AS1/AS2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows §2.2 (restriction matrices R_i, partition of unity D_i with
(D_i)_kk = 1/|M_k|, eq:dd-preconditioners, eq:two-level-preconditioners),
§2.3 (def:algebraic-perfact-coarse-space: column i of R_0^T is D_i R_i psi),
§3 (eq:twoLevelASMPreconditioner: local matrices A_sigma,i = R_i A_sigma R_i^T
and A_sigma,0 = R_0 A_sigma R_0^T) and §4.1.2 (distance-based partition of
unity chi_i = I_h(d_i / sum_j d_j)).

Decomposition (§3 and §4.1): the non-overlapping subdomains are the L^p unit
cells Omega'_c = prod_j (c_j - 1, c_j) x (0, ell)^q, numbered with x1 fastest
(the index map of the periodic cells in §3.2).  Omega_c adds delta element
layers in every expanding direction, clipped to Omega_L; its unknowns are the
interior nodes strictly inside Omega_c, i.e. x_j node index in
[(c_j - 1) n_e - delta + 1, c_j n_e + delta - 1] intersected with [1, L n_e - 1].

Everything here is written with explicit index sets and scipy.sparse
products, without exploiting that interior subdomains share one local matrix.
"""
import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def subdomain_ranges(grid, delta):
    """Per subdomain (x1-fastest numbering) a list of inclusive 1-based node ranges per axis."""
    ne, L = grid.ne, grid.L
    per_axis = []
    for a in range(grid.d):
        if a < grid.p:
            rs = []
            for c in range(1, L + 1):
                lo = max((c - 1) * ne - delta + 1, 1)
                hi = min(c * ne + delta - 1, L * ne - 1)
                rs.append((lo, hi))
            per_axis.append(rs)
        else:
            per_axis.append([(1, grid.nel[a] - 1)])
    out = []
    # x1 fastest: iterate the cell multi-index with axis 0 varying fastest
    for combo in itertools.product(*[range(len(r)) for r in reversed(per_axis)]):
        combo = combo[::-1]
        out.append([per_axis[a][combo[a]] for a in range(grid.d)])
    return out


def subdomain_dofs(grid, delta):
    """Canonical linear indices (sorted) of the unknowns of every subdomain."""
    subs = []
    for rng in subdomain_ranges(grid, delta):
        axes = [np.arange(lo, hi + 1) - 1 for (lo, hi) in rng]  # 0-based unknown index
        mesh = np.meshgrid(*axes, indexing="ij")
        lin = grid.linear_index([m.ravel(order="F") for m in mesh])
        subs.append(np.sort(lin))
    return subs


def restriction(n, dofs):
    """Boolean restriction matrix R_i (|N_i| x n) of §2.2."""
    m = dofs.size
    return sp.csr_matrix((np.ones(m), (np.arange(m), dofs)), shape=(m, n))


def pu_equal(grid, subs):
    """Equal-weight partition of unity of §2.2: (D_i)_kk = 1 / #{subdomains containing k}."""
    count = np.zeros(grid.n)
    for s in subs:
        count[s] += 1.0
    return [1.0 / count[s] for s in subs]


def pu_distance(grid, subs, delta):
    """Distance-based partition of unity of §4.1.2.

    d_i(z) = dist(z, boundary of Omega_i minus boundary of Omega_L) inside
    Omega_i; for a point inside the box Omega_i this is the smallest
    perpendicular distance to one of its faces that is not on the global
    boundary (faces exist only in expanding directions).  chi_i = d_i / sum_j d_j
    at the nodes (nodal interpolation I_h).
    """
    h = grid.h
    L = grid.L
    coords = _node_coords(grid)
    ranges = subdomain_ranges(grid, delta)
    dist = []
    for s, rng in zip(subs, ranges):
        dmin = np.full(s.size, np.inf)
        for a in range(grid.p):
            lo_node, hi_node = rng[a]
            # box extent of Omega_i along axis a (clipped), in coordinates
            lo = (lo_node - 1) * h
            hi = (hi_node + 1) * h
            z = coords[a][s]
            if lo > 0.0 + 1e-12:
                dmin = np.minimum(dmin, z - lo)
            if hi < L - 1e-12:
                dmin = np.minimum(dmin, hi - z)
        dist.append(dmin)
    total = np.zeros(grid.n)
    for s, dd in zip(subs, dist):
        if np.all(np.isinf(dd)):
            continue
        total[s] += dd
    out = []
    for s, dd in zip(subs, dist):
        if np.all(np.isinf(dd)):  # a single subdomain covering everything
            out.append(np.ones(s.size))
        else:
            out.append(dd / total[s])
    return out


def _node_coords(grid):
    axes = [np.arange(1, grid.nel[a]) * grid.h for a in range(grid.d)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return [m.ravel(order="F") for m in mesh]


def coarse_basis(grid, subs, weights, psi_ext):
    """R_0^T of def:algebraic-perfact-coarse-space: column i = R_i^T D_i R_i psi."""
    n, N = grid.n, len(subs)
    rows, cols, vals = [], [], []
    for i, (s, w) in enumerate(zip(subs, weights)):
        rows.append(s)
        cols.append(np.full(s.size, i))
        vals.append(w * psi_ext[s])
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, N))


class AdditiveSchwarz:
    """One- or two-level additive Schwarz preconditioner (eq:dd-preconditioners,
    eq:two-level-preconditioners, eq:twoLevelASMPreconditioner), exact local solves.

    apply(r) = R_0^T A_0^{-1} R_0 r + sum_i R_i^T A_i^{-1} R_i r   (two-level)
    """

    def __init__(self, A_sigma, subs, R0T=None):
        A = sp.csr_matrix(A_sigma)
        self.n = A.shape[0]
        self.subs = subs
        self.R = [restriction(self.n, s) for s in subs]
        self.local = []
        for R in self.R:
            Ai = (R @ A @ R.T).tocsc()
            self.local.append(spla.splu(Ai, permc_spec="MMD_AT_PLUS_A"))
        self.R0T = None
        if R0T is not None:
            self.R0T = sp.csc_matrix(R0T)
            A0 = (self.R0T.T @ A @ self.R0T).toarray()
            self.A0 = 0.5 * (A0 + A0.T)
            self.A0_lu = np.linalg.cholesky(self.A0)  # A0 is SPD (§3)

    def coarse_solve(self, c):
        Lc = self.A0_lu
        y = np.linalg.solve(Lc, c)
        return np.linalg.solve(Lc.T, y)

    def apply(self, r):
        z = np.zeros(self.n)
        for R, lu in zip(self.R, self.local):
            z += R.T @ lu.solve(R @ r)
        if self.R0T is not None:
            z += self.R0T @ self.coarse_solve(self.R0T.T @ r)
        return z

    def dense(self):
        """The preconditioner M^{-1} as a dense matrix (small cases only)."""
        I = np.eye(self.n)
        return np.column_stack([self.apply(I[:, j]) for j in range(self.n)])
