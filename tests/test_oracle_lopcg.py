"""Pins of the oracle's inexact SI-preconditioned LOPCG (alg:si-lopcg).

- it converges to the smallest eigenpair of a dense generalized eigensolver,
  with fixed and adaptive inner tolerances and with the preconditioner
  applied directly (the fused variant of §4.3);
- Rayleigh-Ritz over a span that contains an exact eigenvector returns it;
- the Ritz values never increase (x_k lies in the next search space);
- one step from x_k is at least as good as the shifted inverse-iteration step
  A_sigma^{-1} B x_k from the same x_k, which lies in span{w_k, x_k} when the
  inner solve is exact (w_k = x_k + (sigma - lambda_k) A_sigma^{-1} B x_k);
- the ordering of total inner work reported in §4.3: fused < adaptive < fixed.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import workloads as W
from oracle.lopcg import rayleigh_ritz, si_lopcg, unit_first
from oracle.problem import Problem


def _P(L=6, ne=8, delta=2, seed=1000):
    return Problem(W.small_config(1, 1, L, ne, delta, W.sep_fourier(seed)))


def _dense(P):
    w, v = sla.eigh(P.A.toarray(), P.M.toarray(), subset_by_index=[0, 1])
    x = v[:, 0] / np.sqrt(v[:, 0] @ (P.M @ v[:, 0]))
    return w, x if np.sum(P.M @ x) > 0 else -x


@pytest.mark.parametrize("mode", ["fixed", "adaptive", "fused"])
def test_converges_to_dense_eigenpair(mode):
    P = _P()
    w, xr = _dense(P)
    prec = P.preconditioner(True)
    n = P.grid.n
    out = si_lopcg(P.A, P.M, P.sigma, unit_first(n), np.ones(n), tol_o=1e-10, kmax=500,
                   mode=mode, rtol_i=1e-10, precond=prec.apply)
    assert out["res_hist"][-1] <= 1e-10
    assert abs(out["lam"] - w[0]) <= 1e-12 * abs(w[0])
    d = out["x"] - xr
    assert np.sqrt(d @ (P.M @ d)) <= 1e-8


def test_rayleigh_ritz_recovers_eigenvector():
    P = _P(L=4)
    w, xr = _dense(P)
    rng = np.random.default_rng(3)
    S = np.column_stack([rng.standard_normal(P.grid.n), xr, rng.standard_normal(P.grid.n)])
    c, mu = rayleigh_ritz(S, P.A @ S, P.M @ S)
    assert abs(mu - w[0]) <= 1e-12 * abs(w[0])
    y = S @ c
    y /= np.sqrt(y @ (P.M @ y))
    assert min(np.linalg.norm(y - xr), np.linalg.norm(y + xr)) <= 1e-8 * np.linalg.norm(xr)


def test_ritz_values_do_not_increase():
    P = _P(L=8)
    n = P.grid.n
    prec = P.preconditioner(True)
    out = si_lopcg(P.A, P.M, P.sigma, unit_first(n), np.ones(n), tol_o=1e-11, kmax=200,
                   mode="adaptive", precond=prec.apply)
    lams = []
    # re-run step by step: the Ritz value after k steps
    for k in range(1, out["its"] + 1):
        lams.append(si_lopcg(P.A, P.M, P.sigma, unit_first(n), np.ones(n), tol_o=0.0, kmax=k,
                             mode="adaptive", precond=prec.apply)["lam"])
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(lams, lams[1:]))


def test_step_beats_shifted_inverse_iteration():
    P = _P(L=6)
    n = P.grid.n
    rng = np.random.default_rng(5)
    x1 = np.abs(rng.standard_normal(n)) + 0.1
    x0 = unit_first(n)
    As = P.A_sigma.tocsc()
    lu = spla.splu(As)
    step = si_lopcg(P.A, P.M, P.sigma, x0, x1, tol_o=0.0, kmax=1, mode="fused",
                    precond=lu.solve)
    x = x1 / np.sqrt(x1 @ (P.M @ x1))
    u = lu.solve(P.M @ x)
    r_ipm = float(u @ (P.A @ u)) / float(u @ (P.M @ u))
    assert step["lam"] <= r_ipm + 1e-12 * abs(r_ipm)


def test_inner_work_ordering():
    """§4.3: fused < adaptive < fixed in total inner iterations."""
    P = _P(L=16, ne=8, delta=2, seed=1000)
    n = P.grid.n
    prec = P.preconditioner(True)
    tot = {}
    for mode in ("fixed", "adaptive", "fused"):
        out = si_lopcg(P.A, P.M, P.sigma, unit_first(n), np.ones(n), tol_o=1e-8, kmax=2000,
                       mode=mode, rtol_i=1e-8, precond=prec.apply)
        assert out["res_hist"][-1] <= 1e-8
        tot[mode] = int(out["inner"].sum())
    assert tot["fused"] < tot["adaptive"] < tot["fixed"], tot


def _inner_solvers(P):
    from oracle.ras import RestrictedAdditiveSchwarz, gmres_right, stationary_ras
    As = P.A_sigma
    r1 = RestrictedAdditiveSchwarz(As, P.subs, P.D)
    r2 = RestrictedAdditiveSchwarz(As, P.subs, P.D, P.R0T)

    def wrap(f):
        def solve(b, rt, mi):
            o = f(b, rt, mi)
            return o["x"], o["iters"]
        return solve
    return {
        "ras1": wrap(lambda b, rt, mi: stationary_ras(As, b, r1, False, rtol=rt, maxit=mi)),
        "ras2": wrap(lambda b, rt, mi: stationary_ras(As, b, r2, True, rtol=rt, maxit=mi)),
        "cg+asm2": None,
        "gmres+ras2": wrap(lambda b, rt, mi: gmres_right(As, b, r2.apply, rtol=rt, maxit=mi)),
    }


def test_inner_solvers_of_table2():
    """§4.2 (Table 2): with stationary RAS1 / RAS2, CG+ASM2 or GMRES+RAS2 as the
    inner solver (fixed rTOL_i = TOL_o = 1e-8, zero initial guesses) the outer
    iterations do not change, the total inner work orders as
    GMRES+RAS2 < CG+ASM2 < RAS2 < RAS1, and the worst inner solve of RAS1 grows
    with L while that of RAS2 stays bounded."""
    mx = {}
    for L in (4, 8):
        P = _P(L=L)
        w, xr = _dense(P)
        n = P.grid.n
        prec = P.preconditioner(True)
        its, tot = {}, {}
        for name, solve in _inner_solvers(P).items():
            out = si_lopcg(P.A, P.M, P.sigma, unit_first(n), np.ones(n), tol_o=1e-8, kmax=500,
                           mode="fixed", rtol_i=1e-8, maxit_i=10000, precond=prec.apply,
                           inner_solve=solve)
            assert out["res_hist"][-1] <= 1e-8
            assert abs(out["lam"] - w[0]) <= 1e-10 * abs(w[0]), name
            its[name], tot[name] = out["its"], int(out["inner"].sum())
            mx[name, L] = int(out["inner"].max())
        assert max(its.values()) - min(its.values()) <= 1, its
        assert tot["gmres+ras2"] < tot["cg+asm2"] < tot["ras2"] < tot["ras1"], tot
    assert mx["ras1", 8] >= 3 * mx["ras1", 4], mx
    assert mx["ras2", 8] <= 1.3 * mx["ras2", 4], mx


def test_fused_with_ras2_preconditioner():
    """§4.3 uses M_RAS,2 directly as the LOPCG preconditioner; it converges to
    the dense eigenpair like the M_ASM,2 variant."""
    from oracle.ras import RestrictedAdditiveSchwarz
    P = _P(L=6)
    w, xr = _dense(P)
    n = P.grid.n
    r2 = RestrictedAdditiveSchwarz(P.A_sigma, P.subs, P.D, P.R0T)
    out = si_lopcg(P.A, P.M, P.sigma, unit_first(n), np.ones(n), tol_o=1e-10, kmax=2000,
                   mode="fused", precond=r2.apply)
    assert out["res_hist"][-1] <= 1e-10
    assert abs(out["lam"] - w[0]) <= 1e-11 * abs(w[0])
    d = out["x"] - xr
    assert np.sqrt(d @ (P.M @ d)) <= 1e-8
