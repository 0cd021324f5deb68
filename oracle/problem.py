"""Convenience assembly of one eigenproblem instance from a workload dict.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Collects the pieces of §2: the Q1 matrices on Omega_L, the cell problem
(sigma, psi), the periodic extension psi_ext, the decomposition into unit
cells with delta overlap layers, a partition of unity and the PerFact coarse
basis.  ``pu`` is "equal" (§2.2) or "distance" (§4.1.2).
"""
from .fem import Grid, assemble_elements, assemble_kron
from .potential import vfun, kron_terms
from .cell import cell_problem, extend_periodic
from .dd import subdomain_dofs, pu_equal, pu_distance, coarse_basis, AdditiveSchwarz


class Problem:
    def __init__(self, cfg, nq=2, route="elements", pu="equal", sigma=None, with_cell=True):
        p, q, L, ne, ell = cfg["p"], cfg["q"], cfg["L"], cfg["ne"], cfg.get("ell", 1)
        self.cfg = cfg
        self.grid = Grid(p, q, L, ne, ell=ell)
        if route == "elements":
            self.K, self.M, self.MV = assemble_elements(self.grid, vfun(cfg["V"], p, q, ell), nq=nq)
        else:
            self.K, self.M, self.MV = assemble_kron(self.grid, kron_terms(cfg["V"], p, q, ell), nq=nq)
        self.A = (self.K + self.MV).tocsr()
        self.delta = cfg["delta"]
        self.subs = subdomain_dofs(self.grid, self.delta)
        if pu == "equal":
            self.D = pu_equal(self.grid, self.subs)
        else:
            self.D = pu_distance(self.grid, self.subs, self.delta)
        self.cell = None
        if with_cell:
            self.cell = cell_problem(p, q, ne, cfg["V"], ell=ell, nq=nq, route=route)
            self.sigma = self.cell["sigma"] if sigma is None else sigma
            self.psi_ext = extend_periodic(self.cell["psi"], self.grid)
            self.R0T = coarse_basis(self.grid, self.subs, self.D, self.psi_ext)
        else:
            self.sigma = sigma
        if self.sigma is not None:
            self.A_sigma = (self.A - self.sigma * self.M).tocsr()

    def preconditioner(self, two_level=True):
        return AdditiveSchwarz(self.A_sigma, self.subs, self.R0T if two_level else None)
