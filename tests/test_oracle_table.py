"""Pins of tabulated potentials (values at the quadrature points of one period
cell) in the oracle.

- a table that samples an analytic potential at the documented points gives
  the analytic potential's matrices exactly (2-D, 3-D with one and with two
  expanding axes, ell != 1): the lookup finds the right element and Gauss point;
- a table with one nonzero value couples exactly the 2^d nodes of that element
  (in every period cell) and weighs most the node nearest the point;
- the truncated Coulomb well and the union-of-disks chain of §4.2: the
  eigenvalue grows with the penalty (V grows pointwise) and the ground state
  concentrates in the disks as the penalty grows.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle.potential import vfun
from oracle.problem import Problem


def _tabulate(spec, p, q, ne, ell):
    z = W.quad_points(p, q, ne, ell)
    return W.quad_table(p, q, ne, ell, vfun(spec, p, q, ell)(z))


@pytest.mark.parametrize("p,q,L,ne,delta,ell,V", [
    (1, 1, 3, 8, 2, 1, W.sep_fourier(1000)),
    (1, 1, 2, 4, 1, 1.5, W.sep_fourier(5)),
    (1, 2, 2, 4, 1, 1, W.sep_fourier(3000)),
    (2, 1, 2, 4, 1, 1, W.fourier2(4000)),
])
def test_table_reproduces_analytic_potential(p, q, L, ne, delta, ell, V):
    Pa = Problem(W.small_config(p, q, L, ne, delta, V, ell=ell), with_cell=False)
    Pt = Problem(W.small_config(p, q, L, ne, delta, _tabulate(V, p, q, ne, ell), ell=ell),
                 with_cell=False)
    scale = abs(Pa.MV).max()
    assert abs(Pa.MV - Pt.MV).max() <= 1e-14 * scale


def test_single_point_table_couples_one_element():
    p, q, L, ne, ell = 1, 1, 2, 4, 1
    z = W.quad_points(p, q, ne, ell)
    n_tab = z[0].size
    e0, e1, qi = 2, 1, 0          # element (2, 1) of the cell, its lower-left Gauss point
    idx = (e0 + ne * e1) * 4 + qi
    tab = np.zeros(n_tab)
    tab[idx] = 1.0
    P = Problem(W.small_config(p, q, L, ne, 1, W.quad_table(p, q, ne, ell, tab)),
                with_cell=False)
    MV = P.MV.tocoo()
    nx = P.grid.nel[0] - 1
    # element (e0 + ne c, e1) has corner nodes (i, j), i in {e0 + ne c, e0 + ne c + 1},
    # j in {e1, e1 + 1} (1-based node indices; unknowns are the interior nodes)
    touched = set()
    for c in range(L):
        for i in (e0 + ne * c, e0 + ne * c + 1):
            for j in (e1, e1 + 1):
                if 1 <= i <= nx and 1 <= j <= P.grid.nel[1] - 1:
                    touched.add((i - 1) + nx * (j - 1))
    nz = {(r, c) for r, c, v in zip(MV.row, MV.col, MV.data) if v != 0.0}
    assert {r for r, _ in nz} == touched and {c for _, c in nz} == touched
    # the lower-left Gauss point lies nearest the lower-left corner (e0, e1)
    diag = P.MV.diagonal()
    ll = (e0 + ne * 0 - 1) + nx * (e1 - 1)
    assert diag[ll] == diag.max()


def test_union_of_disks_penalty():
    ne, L = 8, 4
    lams, outside = [], []
    for a in (10.0, 100.0, 1000.0):
        V = W.union_of_disks(ne, penalty=a)
        P = Problem(W.small_config(1, 1, L, ne, 2, V, ell=V["ell"]), with_cell=False)
        w, v = sla.eigh(P.A.toarray(), P.M.toarray(), subset_by_index=[0, 0])
        x = v[:, 0] / np.sqrt(v[:, 0] @ (P.M @ v[:, 0]))
        # nodes outside every disk (centres (c + 1/2, R))
        h = P.grid.h
        xs = (np.arange(P.grid.nel[0] - 1) + 1) * h
        ys = (np.arange(P.grid.nel[1] - 1) + 1) * h
        X, Y = np.meshgrid(xs, ys, indexing="xy")
        r = np.sqrt((np.mod(X, 1.0) - 0.5) ** 2 + (Y - V["ell"] / 2) ** 2).ravel()
        lams.append(w[0])
        outside.append(np.sum(x[r > 0.75] ** 2) / np.sum(x ** 2))
    assert lams[0] < lams[1] < lams[2]
    assert outside[0] > outside[1] > outside[2]


def test_coulomb_well_is_radial_and_truncated():
    z = W.quad_points(1, 1, 16, 1)
    V = W.coulomb_well(1, 1, 16)
    r = np.sqrt((z[0] - 0.5) ** 2 + (z[1] - 0.5) ** 2)
    np.testing.assert_allclose(V["table"], -1.0 / np.maximum(r, 1e-4), rtol=1e-15)
    assert V["table"].min() >= -1e4
