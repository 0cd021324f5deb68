"""Pins of the oracle's restricted additive Schwarz, stationary RAS and GMRES.

- RAS1 on a diagonal operator is its exact inverse (the local solves commute
  with the restrictions and the D_i sum to the identity), while AS1 counts
  overlapped unknowns twice; with the equal partition of unity RAS1 r is
  AS1 r divided by the number of covering subdomains at every node; with one
  subdomain both equal A^{-1};
- the coarse correction is a Galerkin projection: after it R_0^T r = 0, and
  so after every step of the two-level multiplicative stationary RAS;
- stationary RAS1 / RAS2 converge to the sparse direct solution; RAS1 needs
  about 4x the steps when L doubles while RAS2 stays nearly constant (§4.2);
- GMRES: its residuals equal the least-squares minimum over the Krylov space
  of A M^{-1}, computed with a library least-squares solve on a separately
  orthonormalised Krylov basis; with the exact inverse as preconditioner it
  converges in one step; without a preconditioner its residuals never exceed
  CG's; restarts keep the solution; a zero right-hand side returns zero;
- §4.2: GMRES+RAS2 needs no more iterations than CG+ASM2 (fewer with the
  equal partition of unity).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle.pcg import pcg
from oracle.problem import Problem
from oracle.ras import RestrictedAdditiveSchwarz, gmres_right, stationary_ras


def _P(L=6, ne=8, delta=2, seed=1000, pu="equal", p=1):
    V = W.sep_fourier(seed) if p == 1 else W.fourier2(seed)
    return Problem(W.small_config(p, 1, L, ne, delta, V), pu=pu)


def _count(P):
    c = np.zeros(P.grid.n)
    for s in P.subs:
        c[s] += 1.0
    return c


@pytest.mark.parametrize("pu", ["equal", "distance"])
def test_ras1_diagonal_operator_is_exact(pu):
    P = _P(L=5, pu=pu)
    rng = np.random.default_rng(3)
    d = rng.uniform(1.0, 4.0, P.grid.n)
    A = sp.diags(d).tocsr()
    r = rng.standard_normal(P.grid.n)
    ras = RestrictedAdditiveSchwarz(A, P.subs, P.D)
    np.testing.assert_allclose(ras.apply(r), r / d, rtol=1e-14, atol=0)
    as1 = P.preconditioner(False).__class__(A, P.subs)
    np.testing.assert_allclose(as1.apply(r), _count(P) * r / d, rtol=1e-14, atol=0)


def test_ras1_equal_pu_is_as1_over_count():
    P = _P(L=5)
    r = W.random_vector(P.grid.n, 11)
    ras = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D)
    z_as = P.preconditioner(False).apply(r)
    np.testing.assert_allclose(ras.apply(r), z_as / _count(P), rtol=1e-12, atol=1e-14)


def test_single_subdomain_is_exact_inverse():
    P = _P(L=1)
    assert len(P.subs) == 1
    r = W.random_vector(P.grid.n, 12)
    ras = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D)
    x = spla.spsolve(P.A_sigma.tocsc(), r)
    np.testing.assert_allclose(ras.apply(r), x, rtol=1e-10, atol=1e-12 * np.abs(x).max())


@pytest.mark.parametrize("pu", ["equal", "distance"])
def test_coarse_correction_is_galerkin(pu):
    P = _P(L=6, pu=pu)
    ras = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D, P.R0T)
    r = W.random_vector(P.grid.n, 13)
    rn = r - P.A_sigma @ ras.coarse_part(r)
    assert np.abs(P.R0T.T @ rn).max() <= 1e-12 * np.abs(P.R0T.T @ r).max()
    b = W.random_vector(P.grid.n, 14)
    for k in (1, 2, 5):
        out = stationary_ras(P.A_sigma, b, ras, two_level=True, rtol=0.0, maxit=k)
        res = b - P.A_sigma @ out["x"]
        assert np.abs(P.R0T.T @ res).max() <= 1e-11 * np.abs(P.R0T.T @ b).max(), k


@pytest.mark.parametrize("two_level", [False, True])
@pytest.mark.parametrize("pu", ["equal", "distance"])
def test_stationary_converges_to_direct_solution(two_level, pu):
    P = _P(L=4, pu=pu)
    ras = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D, P.R0T if two_level else None)
    b = W.random_vector(P.grid.n, 15)
    out = stationary_ras(P.A_sigma, b, ras, two_level=two_level, rtol=1e-11, maxit=5000)
    assert out["status"] == "ok"
    x = spla.spsolve(P.A_sigma.tocsc(), b)
    assert np.linalg.norm(out["x"] - x) <= 1e-8 * np.linalg.norm(x)
    np.testing.assert_allclose(out["hist"][-1],
                               np.linalg.norm(b - P.A_sigma @ out["x"]) / np.linalg.norm(b),
                               rtol=1e-6)


def test_ras1_not_robust_ras2_robust():
    """§4.2: the one-level stationary RAS degrades with L, the two-level one does not."""
    it1, it2 = {}, {}
    for L in (4, 8, 16):
        P = _P(L=L)
        b = W.random_vector(P.grid.n, 16)
        ras1 = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D)
        ras2 = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D, P.R0T)
        it1[L] = stationary_ras(P.A_sigma, b, ras1, False, rtol=1e-8, maxit=10000)["iters"]
        it2[L] = stationary_ras(P.A_sigma, b, ras2, True, rtol=1e-8, maxit=10000)["iters"]
    assert it1[8] >= 3 * it1[4] and it1[16] >= 3 * it1[8], it1
    assert it2[16] <= 1.3 * it2[4], it2


def _krylov_min_residuals(A, Mdense, b, kmax):
    """min_y ||b - A M K_k y|| / ||b|| for k = 1..kmax with K_k an orthonormal basis
    of span{b, (A M) b, ..., (A M)^{k-1} b}, built by classical Gram-Schmidt applied
    twice and solved with numpy's least squares."""
    AM = A @ Mdense
    Q = np.zeros((b.size, 0))
    v = b / np.linalg.norm(b)
    out = []
    for _ in range(kmax):
        for _ in range(2):
            v = v - Q @ (Q.T @ v)
        v /= np.linalg.norm(v)
        Q = np.column_stack([Q, v])
        B = AM @ Q
        y, *_ = np.linalg.lstsq(B, b, rcond=None)
        out.append(np.linalg.norm(b - B @ y) / np.linalg.norm(b))
        v = AM @ v
    return np.array(out)


@pytest.mark.parametrize("prec", ["none", "ras2"])
def test_gmres_residuals_are_krylov_minimum(prec):
    P = _P(L=3, ne=4, delta=1)
    A = P.A_sigma.toarray()
    n = P.grid.n
    b = W.random_vector(n, 17)
    if prec == "none":
        Md, apply_M = np.eye(n), None
    else:
        ras = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D, P.R0T)
        Md = np.column_stack([ras.apply(e) for e in np.eye(n)])
        apply_M = ras.apply
    out = gmres_right(P.A_sigma, b, apply_M, rtol=1e-10)
    K = min(12, out["iters"])
    ref = _krylov_min_residuals(A, Md, b, K)
    np.testing.assert_allclose(out["hist"][1:K + 1], ref, rtol=1e-6, atol=1e-13)


def test_gmres_exact_preconditioner_one_step():
    P = _P(L=4)
    lu = spla.splu(P.A_sigma.tocsc())
    b = W.random_vector(P.grid.n, 18)
    out = gmres_right(P.A_sigma, b, lu.solve, rtol=1e-10)
    assert out["iters"] == 1
    np.testing.assert_allclose(out["x"], lu.solve(b), rtol=1e-10, atol=1e-13)


def test_gmres_never_worse_than_cg():
    P = _P(L=6)
    b = W.random_vector(P.grid.n, 19)
    g = gmres_right(P.A_sigma, b, None, rtol=1e-9)
    c = pcg(lambda v: P.A_sigma @ v, b, None, rtol=1e-9, maxit=5000)
    k = min(len(g["hist"]), len(c.hist))
    assert np.all(g["hist"][:k] <= c.hist[:k] * (1 + 1e-8))
    assert g["iters"] <= c.iters


@pytest.mark.parametrize("restart", [5, 17])
def test_gmres_restart_and_solution(restart):
    P = _P(L=5)
    ras = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D, P.R0T)
    b = W.random_vector(P.grid.n, 20)
    full = gmres_right(P.A_sigma, b, ras.apply, rtol=1e-10)
    out = gmres_right(P.A_sigma, b, ras.apply, rtol=1e-10, restart=restart, maxit=2000)
    assert out["status"] == "ok" and out["iters"] >= full["iters"]
    x = spla.spsolve(P.A_sigma.tocsc(), b)
    for o in (full, out):
        assert np.linalg.norm(o["x"] - x) <= 1e-7 * np.linalg.norm(x)
        res = np.linalg.norm(b - P.A_sigma @ o["x"]) / np.linalg.norm(b)
        assert res <= 1e-9


def test_zero_rhs():
    P = _P(L=3)
    ras = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D, P.R0T)
    z = np.zeros(P.grid.n)
    for out in (gmres_right(P.A_sigma, z, ras.apply), stationary_ras(P.A_sigma, z, ras)):
        assert out["iters"] == 0 and not out["x"].any()


@pytest.mark.parametrize("case", [(1, 8, 8, 2, "equal", 1000), (1, 16, 8, 2, "equal", 1000),
                                  (2, 3, 4, 1, "equal", 4000), (1, 8, 8, 2, "distance", 1000)])
def test_gmres_ras2_not_more_than_cg_asm2(case):
    """§4.2: the unsymmetric GMRES+RAS2 needs fewer iterations than CG+ASM2."""
    p, L, ne, delta, pu, seed = case
    P = _P(L=L, ne=ne, delta=delta, seed=seed, pu=pu, p=p)
    b = W.random_vector(P.grid.n, 21)
    ras = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D, P.R0T)
    g = gmres_right(P.A_sigma, b, ras.apply, rtol=1e-8)
    c = pcg(lambda v: P.A_sigma @ v, b, P.preconditioner(True).apply, rtol=1e-8, maxit=5000)
    assert g["iters"] <= c.iters
    if pu == "equal":
        assert g["iters"] < c.iters
