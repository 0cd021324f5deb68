"""Pins of the oracle's PCG (eq:cg-energy-norm-error-reduction) and shifted
inverse iteration (§2, §2.1) against direct solvers, dense eigensolvers, the
CG error bound, the contraction rate of inverse iteration and the
L-robustness of the two-level preconditioner (eq:conditionNumberBound, §4.1.1).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import workloads as W
from oracle.ipm import inverse_iteration_direct, inverse_iteration_pcg, spectral_residual
from oracle.pcg import pcg, lanczos_extremes
from oracle.problem import Problem

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _P(L=4, ne=6, delta=2, spec=None, p=1, q=1):
    spec = spec if spec is not None else W.sep_fourier(1000)
    return Problem(W.small_config(p, q, L, ne, delta, spec))


def test_pcg_solves_system():
    P = _P()
    b = W.random_vector(P.grid.n, 3)
    M = P.preconditioner(True)
    res = pcg(lambda v: P.A_sigma @ v, b, M.apply, rtol=1e-12, maxit=500)
    assert res.status == "ok"
    x = spla.spsolve(P.A_sigma.tocsc(), b)
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)
    assert np.linalg.norm(b - P.A_sigma @ res.x) <= 1.01e-12 * np.linalg.norm(b)


def test_pcg_within_cg_bound():
    """Iterations do not exceed what the energy-norm bound predicts from the
    Ritz estimate of kappa(M^{-1} A_sigma), with the residual/energy conversion."""
    P = _P(L=6, ne=6, delta=2)
    b = W.random_vector(P.grid.n, 4)
    M = P.preconditioner(True)
    res = pcg(lambda v: P.A_sigma @ v, b, M.apply, rtol=1e-10, maxit=500)
    lo, hi = lanczos_extremes(res.alphas, res.betas)
    kappa = hi / lo
    rho = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    kappa_A = np.linalg.cond(P.A_sigma.toarray())
    bound = np.log(1e-10 / (2 * np.sqrt(kappa_A) * np.sqrt(kappa))) / np.log(rho)
    assert res.iters <= bound


def test_pcg_detects_indefinite_operator():
    """A shift above lambda_1 makes A_sigma indefinite: CG must report it."""
    P = _P(L=3, ne=4, delta=1)
    lam1 = sla.eigh(P.A.toarray(), P.M.toarray(), eigvals_only=True, subset_by_index=[0, 0])[0]
    A_bad = (P.A - (lam1 + 5.0) * P.M).tocsr()
    res = pcg(lambda v: A_bad @ v, P.M @ np.ones(P.grid.n), None, rtol=1e-12, maxit=500)
    assert res.status == "not_spd"


def test_pcg_detects_indefinite_preconditioner():
    """r.z <= 0 (an indefinite preconditioner, as a rounded local inverse can
    make) is reported as not_spd with the iterations done so far: at once for
    -M^{-1}, after two iterations for a preconditioner whose third application
    flips sign; the SPD preconditioner itself converges."""
    P = _P(L=3, ne=4, delta=1)
    b = P.M @ np.ones(P.grid.n)
    M = P.preconditioner(True)
    A = lambda v: P.A_sigma @ v
    ok = pcg(A, b, M.apply, rtol=1e-10, maxit=500)
    assert ok.status == "ok" and ok.iters > 3
    res = pcg(A, b, lambda r: -M.apply(r), rtol=1e-10, maxit=500)
    assert res.status == "not_spd" and res.iters == 0
    calls = []

    def flip_third(r):
        calls.append(1)
        return -M.apply(r) if len(calls) == 3 else M.apply(r)

    res = pcg(A, b, flip_third, rtol=1e-10, maxit=500)
    assert res.status == "not_spd" and res.iters == 2
    assert np.array_equal(res.alphas, ok.alphas[:2])


def test_as2_iterations_bounded_in_L_and_as1_grows():
    """§4.1.1 and eq:conditionNumberBound: with the PerFact coarse space the
    spectrum of M^{-1} A_sigma (Ritz estimates) and the CG iteration count stop
    depending on L, while the one-level lambda_min falls like 1/L^2."""
    its1, its2, kap1, kap2 = [], [], [], []
    for L in (8, 16, 32):
        P = _P(L=L, ne=6, delta=1, spec=W.sin4())
        b = W.random_vector(P.grid.n, 1)
        for two, its, kap in ((False, its1, kap1), (True, its2, kap2)):
            M = P.preconditioner(two)
            res = pcg(lambda v: P.A_sigma @ v, b, M.apply, rtol=1e-8, maxit=3000)
            assert res.status == "ok"
            its.append(res.iters)
            lo, hi = lanczos_extremes(res.alphas, res.betas)
            kap.append(hi / lo)
    assert abs(its2[2] - its2[1]) <= 3
    assert max(kap2) < 1.2 * min(kap2)
    assert kap1[2] > 3.5 * kap1[1] > 3.5 ** 2 * kap1[0] / 1.1
    assert its1[2] > 1.7 * its1[1]


def _dense_ground(P):
    w, v = sla.eigh(P.A.toarray(), P.M.toarray(), subset_by_index=[0, 1])
    x = v[:, 0] * np.sign(np.sum(P.M @ v[:, 0]))
    return w, x


@pytest.mark.parametrize("p,q,L,ne,delta", [(1, 1, 4, 6, 2), (2, 1, 3, 4, 1), (1, 2, 3, 4, 1)])
def test_inverse_iteration_direct_matches_dense(p, q, L, ne, delta):
    spec = W.sep_fourier(1000) if p == 1 else W.fourier2(4000)
    P = _P(L, ne, delta, spec, p, q)
    w, xr = _dense_ground(P)
    res = inverse_iteration_direct(P.A, P.M, P.sigma, P.grid if P.grid.d == 2 else None)
    assert abs(res["lam"] - w[0]) <= 1e-12 * abs(w[0])
    d = res["x"] - xr
    assert np.sqrt(d @ (P.M @ d)) <= 1e-10
    assert spectral_residual(P.A, P.M, res["lam"], res["x"]) <= 1e-9 * np.abs(P.A).max()


def test_inverse_iteration_contraction_rate():
    """||x_{k+1} - x_k|| shrinks by (lambda_1 - sigma)/(lambda_2 - sigma) per step (§1.2).

    A generic start vector is used: the constant vector is nearly symmetric in
    x and hardly sees the (nearly antisymmetric) second eigenvector."""
    P = _P(L=6, ne=6, delta=2)
    w, _ = _dense_ground(P)
    rho = (w[0] - P.sigma) / (w[1] - P.sigma)
    x0 = 1.0 + W.random_vector(P.grid.n, 8)
    res = inverse_iteration_direct(P.A, P.M, P.sigma, P.grid, x0=x0, tol=1e-14, maxit=60)
    h = res["dx_hist"]
    ratios = h[9:14] / h[8:13]
    assert np.allclose(ratios, rho, rtol=2e-2)


def test_qosi_ratio_tends_to_quarter_for_laplacian():
    """V = 0: (lambda_1 - sigma)/(lambda_2 - sigma) -> 1/4 as L grows (§1.2)."""
    from oracle.fem import Grid, assemble_kron
    from oracle.potential import kron_terms
    from oracle.cell import cell_problem
    ne = 4
    sig = cell_problem(1, 1, ne, W.const(0.0))["sigma"]
    g = Grid(1, 1, 64, ne)
    K, M, _ = assemble_kron(g, kron_terms(W.const(0.0), 1, 1))
    w = spla.eigsh(K.tocsc(), k=2, M=M.tocsc(), sigma=sig, which="LM")[0]
    w = np.sort(w)
    assert (w[0] - sig) / (w[1] - sig) == pytest.approx(GOLDEN["qosi_ratio_limit"]["value"], abs=2e-3)


def test_inverse_iteration_with_pcg_matches_direct():
    P = _P(L=8, ne=6, delta=2)
    M = P.preconditioner(True)
    a = inverse_iteration_direct(P.A, P.M, P.sigma, P.grid)
    b = inverse_iteration_pcg(P.A, P.M, P.sigma, M.apply, rtol=1e-10, tol=1e-9)
    assert abs(a["lam"] - b["lam"]) <= 1e-10 * abs(a["lam"])
    d = a["x"] - b["x"]
    assert np.sqrt(d @ (P.M @ d)) <= 1e-8
