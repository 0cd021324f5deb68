"""Pins of the oracle's cell problem (eq:cell-problem, eq:weak-form-cell-problem),
decomposition, partition of unity, PerFact coarse space
(def:algebraic-perfact-coarse-space) and additive Schwarz preconditioners
(eq:dd-preconditioners, eq:two-level-preconditioners).
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from oracle.cell import cell_problem, extend_periodic
from oracle.dd import subdomain_dofs, pu_equal, pu_distance, coarse_basis, AdditiveSchwarz
from oracle.fem import Grid, assemble_elements, interior_coords
from oracle.potential import vfun
from oracle.problem import Problem

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def mu(theta, h):
    return (6.0 / h ** 2) * (1.0 - np.cos(theta)) / (2.0 + np.cos(theta))


# ---------------------------------------------------------------- cell problem

@pytest.mark.parametrize("p,q,ne", [(1, 1, 8), (1, 2, 4), (2, 1, 4)])
def test_cell_v0_closed_form(p, q, ne):
    """V = 0: sigma = q mu(pi h / ell) and psi is constant along x and a discrete
    sine along each fixed direction."""
    c = cell_problem(p, q, ne, W.const(0.0))
    h = 1.0 / ne
    assert c["sigma"] == pytest.approx(q * mu(np.pi * h, h), rel=1e-12)
    g = c["grid"]
    z = interior_coords(g)
    shape = np.ones(g.n)
    for j in range(q):
        shape *= np.sin(np.pi * z[p + j])
    psi = c["psi"]
    ratio = psi / shape
    assert np.ptp(ratio) <= 1e-10 * np.abs(ratio).max()


def test_cell_positive_and_normalised():
    c = cell_problem(1, 1, 16, W.sep_fourier(1000))
    assert np.all(c["psi"] > 0)
    assert c["psi"] @ (c["M"] @ c["psi"]) == pytest.approx(1.0, rel=1e-13)


def test_cell_constant_shift():
    s0 = cell_problem(1, 1, 8, W.sep_fourier(3))["sigma"]
    spec = W.sep_fourier(3)
    g = Grid(1, 1, 1, 8, cell=True)
    # V + c through a separate constant term: compare with the eigenvalue of K + MV + c M
    c = cell_problem(1, 1, 8, spec)
    w = sla.eigh((c["K"] + c["MV"] + 2.5 * c["M"]).toarray(), c["M"].toarray(),
                 eigvals_only=True, subset_by_index=[0, 0])[0]
    assert w == pytest.approx(s0 + 2.5, abs=1e-11)


@pytest.mark.parametrize("p,q,spec", [(1, 1, W.sep_fourier(1000)), (2, 1, W.fourier2(4000)),
                                      (1, 2, W.sep_fourier(3000))])
def test_shifted_operator_annihilates_extended_psi(p, q, spec):
    """Periodicity plus the cell equation: (A_sigma psi_ext)_k = 0 at every node
    whose stencil does not reach the x-boundary (kernel lemma of §3.2)."""
    ne = 6
    cfg = W.small_config(p, q, 3, ne, 1, spec)
    P = Problem(cfg)
    r = P.A_sigma @ P.psi_ext
    z = interior_coords(P.grid)
    h = P.grid.h
    inner = np.ones(P.grid.n, bool)
    for a in range(p):
        inner &= (z[a] > 1.5 * h) & (z[a] < P.grid.L - 1.5 * h)
    scale = np.abs(P.A_sigma).max() * np.abs(P.psi_ext).max()
    assert np.abs(r[inner]).max() <= 1e-12 * scale
    assert np.abs(r[~inner]).max() > 1e-6 * scale  # the boundary rows do not vanish


def test_lambda_L_monotone_towards_sigma():
    """sigma < lambda_{L+1} <= lambda_L (nested spaces, min-max) and
    lambda_L - sigma = O(1/L^2) (factorisation eq:factorization-short)."""
    spec = W.sep_fourier(1000)
    ne = 6
    sig = cell_problem(1, 1, ne, spec)["sigma"]
    lams = []
    Ls = [1, 2, 3, 4, 6, 8, 12, 16]
    for L in Ls:
        g = Grid(1, 1, L, ne)
        K, M, MV = assemble_elements(g, vfun(spec, 1, 1))
        lams.append(sla.eigh((K + MV).toarray(), M.toarray(), eigvals_only=True,
                             subset_by_index=[0, 0])[0])
    lams = np.array(lams)
    assert np.all(lams > sig)
    assert np.all(np.diff(lams) <= 1e-10)
    slope = np.polyfit(np.log(Ls[-4:]), np.log(lams[-4:] - sig), 1)[0]
    assert -2.3 < slope < -1.7


@pytest.mark.xfail(strict=True, reason="the shift printed in §4.1 is not reproduced by the "
                   "Q1 / periodic-x / Dirichlet-y reading of eq:weak-form-cell-problem")
def test_printed_sigma_sin4():
    c = cell_problem(1, 1, 30, W.sin4(100.0))
    assert round(c["sigma"], 5) == GOLDEN["sigma_sin4_h30"]["value"]


def test_extension_is_periodic_copy():
    c = cell_problem(1, 1, 4, W.sep_fourier(9))
    g = Grid(1, 1, 3, 4)
    ext = extend_periodic(c["psi"], g)
    nx = g.ndof_dir[0]
    ex = ext.reshape(-1, nx)          # rows: y, columns: x node 1..nx
    cell = c["psi"].reshape(-1, 4)    # rows: y, columns: x node 0..3
    for ix in range(1, nx + 1):
        assert np.array_equal(ex[:, ix - 1], cell[:, ix % 4])


# ------------------------------------------------------------ decomposition

def _geometric_subdomains(grid, delta):
    """Unknowns strictly inside the overlapping boxes, found from node
    coordinates (independent of the index-range arithmetic of the oracle)."""
    z = interior_coords(grid)
    h, L = grid.h, grid.L
    out = []
    cells = list(itertools.product(*[range(1, L + 1)] * grid.p))
    cells = sorted(cells, key=lambda c: tuple(reversed(c)))  # x1 fastest
    for c in cells:
        inside = np.ones(grid.n, bool)
        for a in range(grid.p):
            lo = max(c[a] - 1 - delta * h, 0.0)
            hi = min(c[a] + delta * h, float(L))
            inside &= (z[a] > lo + 1e-12) & (z[a] < hi - 1e-12)
        out.append(np.nonzero(inside)[0])
    return out


@pytest.mark.parametrize("p,q,L,ne,delta", [(1, 1, 4, 4, 1), (1, 1, 4, 6, 2), (2, 1, 3, 4, 1),
                                            (1, 2, 3, 4, 2)])
def test_subdomains_match_geometry(p, q, L, ne, delta):
    g = Grid(p, q, L, ne)
    subs = subdomain_dofs(g, delta)
    geo = _geometric_subdomains(g, delta)
    assert len(subs) == L ** p
    for a, b in zip(subs, geo):
        assert np.array_equal(a, b)
    m_int = (ne + 2 * delta - 1) ** p * (ne - 1) ** q
    assert max(s.size for s in subs) == m_int


@pytest.mark.parametrize("p,q,L,ne,delta", [(1, 1, 4, 6, 2), (2, 1, 3, 4, 1), (1, 1, 5, 6, 3)])
def test_partitions_of_unity(p, q, L, ne, delta):
    g = Grid(p, q, L, ne)
    subs = subdomain_dofs(g, delta)
    for D in (pu_equal(g, subs), pu_distance(g, subs, delta)):
        tot = np.zeros(g.n)
        for s, w in zip(subs, D):
            tot[s] += w
            assert np.all(w > 0)
        assert np.allclose(tot, 1.0, rtol=0, atol=1e-14)


def test_distance_pu_equals_equal_pu_for_delta1():
    g = Grid(2, 1, 3, 4)
    subs = subdomain_dofs(g, 1)
    for a, b in zip(pu_equal(g, subs), pu_distance(g, subs, 1)):
        assert np.allclose(a, b, atol=1e-14)


def test_distance_pu_is_linear_blend():
    """delta = 2, p = 1: across an interface the weights ramp linearly (§4.1.2)."""
    g = Grid(1, 1, 3, 8)
    subs = subdomain_dofs(g, 2)
    D = pu_distance(g, subs, 2)
    z = interior_coords(g)
    s0 = subs[0]
    x = z[0][s0]
    y = z[1][s0]
    sel = y == y.min()
    xs, ws = x[sel], D[0][sel]
    ramp = (xs > 1 - 2 / 8 + 1e-9)
    # inside the overlap (1 - 2h, 1 + 2h) the weight is (1 + 2h - x) / (4h)
    assert np.allclose(ws[ramp], (1 + 2 / 8 - xs[ramp]) / (4 / 8), atol=1e-14)
    assert np.allclose(ws[~ramp], 1.0)


# ------------------------------------------------------------ coarse space / AS

def _problem(p=1, q=1, L=4, ne=6, delta=2, spec=None, pu="equal"):
    spec = spec if spec is not None else (W.sep_fourier(1000) if p == 1 else W.fourier2(4000))
    return Problem(W.small_config(p, q, L, ne, delta, spec), pu=pu)


@pytest.mark.parametrize("pu", ["equal", "distance"])
def test_coarse_columns_sum_to_psi(pu):
    P = _problem(pu=pu)
    s = np.asarray(P.R0T.sum(axis=1)).ravel()
    assert np.allclose(s, P.psi_ext, rtol=0, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2])
def test_coarse_matrix_annihilates_ones_away_from_boundary(p):
    """A_0 1 = R_0 A_sigma psi_ext, which vanishes in rows whose subdomain does
    not touch the x-boundary (derived from the kernel identity above)."""
    P = _problem(p=p, L=4 if p == 1 else 4, ne=4, delta=1)
    A0 = (P.R0T.T @ P.A_sigma @ P.R0T).toarray()
    row = A0 @ np.ones(A0.shape[0])
    L = P.grid.L
    cells = sorted(itertools.product(*[range(1, L + 1)] * p), key=lambda c: tuple(reversed(c)))
    interior = np.array([all(2 <= c[a] <= L - 1 for a in range(p)) for c in cells])
    scale = np.abs(A0).max()
    assert np.abs(row[interior]).max() <= 1e-12 * scale
    np.linalg.cholesky(A0)


def _dense_as(P, two_level, scale=None):
    """M^{-1} from the definition with explicit 0/1 matrices and dense inverses."""
    n = P.grid.n
    A = P.A_sigma.toarray()
    Minv = np.zeros((n, n))
    for s in _geometric_subdomains(P.grid, P.delta):
        R = np.zeros((s.size, n)); R[np.arange(s.size), s] = 1.0
        Minv += R.T @ np.linalg.inv(R @ A @ R.T) @ R
    if two_level:
        R0T = P.R0T.toarray()
        if scale is not None:
            R0T = R0T * scale[None, :]
        Minv += R0T @ np.linalg.inv(R0T.T @ A @ R0T) @ R0T.T
    return Minv


@pytest.mark.parametrize("p,q,L,ne,delta", [(1, 1, 4, 4, 1), (1, 1, 3, 6, 2), (2, 1, 3, 4, 1)])
def test_additive_schwarz_matches_definition(p, q, L, ne, delta):
    P = _problem(p, q, L, ne, delta)
    for two in (False, True):
        ref = _dense_as(P, two)
        got = P.preconditioner(two).dense()
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_preconditioner_symmetric_and_scale_invariant():
    P = _problem(L=4, ne=4, delta=1)
    Mi = P.preconditioner(True).dense()
    assert np.abs(Mi - Mi.T).max() <= 1e-12 * np.abs(Mi).max()
    rng = np.random.default_rng(0)
    scaled = _dense_as(P, True, scale=rng.uniform(0.5, 2.0, P.grid.L))
    assert np.abs(scaled - Mi).max() <= 1e-10 * np.abs(Mi).max()


@pytest.mark.parametrize("p,q,L,ne,delta,key", [(1, 1, 6, 4, 1, "lambda_max_bound_p1"),
                                                (1, 1, 5, 6, 2, "lambda_max_bound_p1"),
                                                (2, 1, 3, 4, 1, "lambda_max_bound_p2")])
def test_lambda_max_bound(p, q, L, ne, delta, key):
    """lambda_max(M_AS,2^{-1} A_sigma) <= N_c + 1 (§3, strengthened triangle inequality)."""
    P = _problem(p, q, L, ne, delta)
    Mi = P.preconditioner(True).dense()
    w = np.linalg.eigvals(Mi @ P.A_sigma.toarray()).real
    assert w.max() <= GOLDEN[key]["value"] + 1e-9
    assert w.min() > 0
