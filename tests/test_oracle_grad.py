"""Pins of the oracle's parameter derivatives (oracle/grad.py).

The Hellmann-Feynman forms are checked against what fixes them independently
of the formula: central finite differences of eigenvalues from a dense
generalized eigensolver (brute force on small grids), the homogeneity of V in
its amplitudes (sum_t a_t dlambda/da_t equals the potential part of the
Rayleigh quotient), finite differences of the cell eigenvalue for the shift
derivative, and finite differences of a shifted solve (with the shift moving
too) for the adjoint form.  Planted mistakes (a dropped envelope, a flipped
phase sign) must break the finite-difference pin.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import workloads as W
from oracle import grad as G
from oracle.cell import cell_problem
from oracle.fem import assemble_elements
from oracle.potential import vfun

CASES = [
    ("2d-sep", dict(p=1, q=1, L=3, ne=8, delta=1), lambda: W.sep_fourier(11)),
    ("3d-fourier2", dict(p=2, q=1, L=2, ne=4, delta=1), lambda: W.fourier2(12, kmax=1)),
    ("3d-sep", dict(p=1, q=2, L=3, ne=4, delta=1), lambda: W.sep_fourier(13)),
]


def _with(spec, th):
    T = len(spec["a"])
    out = dict(spec)
    out["a"], out["phi"] = list(th[:T]), list(th[T:])
    return out


def _dense_ground(cfg, spec):
    g = G.grid_of(cfg)
    K, M, MV = assemble_elements(g, vfun(spec, g.p, g.q, g.ell))
    w, v = sla.eigh((K + MV).toarray(), M.toarray(), subset_by_index=[0, 0])
    return w[0], v[:, 0], g, M, MV


def _fd(f, th0, h):
    out = np.zeros_like(th0)
    for j in range(th0.size):
        tp, tm = th0.copy(), th0.copy()
        tp[j] += h
        tm[j] -= h
        out[j] = (f(tp) - f(tm)) / (2 * h)
    return out


def _theta(spec):
    return np.concatenate([np.asarray(spec["a"], float), np.asarray(spec["phi"], float)])


@pytest.mark.parametrize("name,geo,vgen", CASES, ids=[c[0] for c in CASES])
def test_hellmann_feynman_matches_finite_differences(name, geo, vgen):
    V = vgen()
    cfg = dict(geo, V=V)
    th0 = _theta(V)
    lam, x, g, M, _ = _dense_ground(cfg, V)
    hf = G.eigenvalue_grad(g, M, x, V)
    scale = max(1.0, float(np.max(np.abs(hf))))

    def lam_of(th):
        return _dense_ground(cfg, _with(V, th))[0]
    # step 1e-4: truncation ~h^2, rounding ~eps*lambda/h
    assert np.max(np.abs(_fd(lam_of, th0, 1e-4) - hf)) <= 5e-8 * scale
    # step 1e-6 (the step of the gradient check): rounding dominates
    assert np.max(np.abs(_fd(lam_of, th0, 1e-6) - hf)) <= 2e-6 * scale


@pytest.mark.parametrize("name,geo,vgen", CASES, ids=[c[0] for c in CASES])
def test_amplitude_homogeneity(name, geo, vgen):
    """V is linear in (a_t): sum_t a_t dlambda/da_t = x^T M_V x / x^T M x."""
    V = vgen()
    lam, x, g, M, MV = _dense_ground(dict(geo, V=V), V)
    hf = G.eigenvalue_grad(g, M, x, V)
    T = len(V["a"])
    lhs = float(np.dot(np.asarray(V["a"]), hf[:T]))
    rhs = float(x @ (MV @ x)) / float(x @ (M @ x))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))


@pytest.mark.parametrize("name,geo,vgen", CASES, ids=[c[0] for c in CASES])
def test_shift_derivative_matches_finite_differences(name, geo, vgen):
    V = vgen()
    p, q, ne = geo["p"], geo["q"], geo["ne"]
    sg = G.shift_grad(cell_problem(p, q, ne, V), V)
    fd = _fd(lambda th: cell_problem(p, q, ne, _with(V, th))["sigma"], _theta(V), 1e-5)
    assert np.max(np.abs(fd - sg)) <= 5e-8 * max(1.0, float(np.max(np.abs(sg))))


def _shifted_loss(cfg, spec, b, c):
    """l = c^T A_sigma^{-1} b with sigma the cell shift of spec (direct solve)."""
    g = G.grid_of(cfg)
    K, M, MV = assemble_elements(g, vfun(spec, g.p, g.q, g.ell))
    cell = cell_problem(cfg["p"], cfg["q"], cfg["ne"], spec)
    As = (K + MV - cell["sigma"] * M).tocsc()
    u = spla.spsolve(As, b)
    return float(c @ u), u, As, M, g, cell


@pytest.mark.parametrize("name,geo,vgen", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_adjoint_solve_gradient_matches_finite_differences(name, geo, vgen):
    V = vgen()
    cfg = dict(geo, V=V)
    n = G.grid_of(cfg).n
    b, c = W.random_vector(n, 21), W.random_vector(n, 22)
    _, u, As, M, g, cell = _shifted_loss(cfg, V, b, c)
    w = spla.spsolve(As, c)
    ds = G.shift_grad(cell, V)
    adj = G.solve_grad(g, M, u, w, V, ds)
    fd = _fd(lambda th: _shifted_loss(cfg, _with(V, th), b, c)[0], _theta(V), 1e-5)
    assert np.max(np.abs(fd - adj)) <= 1e-6 * max(1.0, float(np.max(np.abs(adj))))


def test_planted_mistakes_break_the_pin(monkeypatch):
    """A dropped envelope or a flipped phase sign in dV/dtheta fails the FD pin."""
    geo, V = CASES[0][1], CASES[0][2]()
    cfg = dict(geo, V=V)
    th0 = _theta(V)
    lam, x, g, M, _ = _dense_ground(cfg, V)
    fd = _fd(lambda th: _dense_ground(cfg, _with(V, th))[0], th0, 1e-4)
    good = G.dv_functions

    def no_envelope(spec, p, q, ell=1):
        return good(dict(spec, cy=0.0), p, q, ell)

    def flipped_phase(spec, p, q, ell=1):
        fs = good(spec, p, q, ell)
        T = len(spec["a"])
        return fs[:T] + [(lambda z, f=f: -f(z)) for f in fs[T:]]
    for bad in (no_envelope, flipped_phase):
        monkeypatch.setattr(G, "dv_functions", bad)
        wrong = G.eigenvalue_grad(g, M, x, V)
        assert np.max(np.abs(fd - wrong)) > 1e-4
    monkeypatch.setattr(G, "dv_functions", good)
    assert np.max(np.abs(fd - G.eigenvalue_grad(g, M, x, V))) <= 5e-8
