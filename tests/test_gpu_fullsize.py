"""GPU parity at the full workload sizes, in the launch configurations that
bench.py times (config 2: bf16 dense local solves; the FP64 path it compares
with) and for the 3-D workloads (config 3: FP32 or FP64 block-chain local
solves, config 4: bf16 dense local solves through the unclipped-box inverse,
or FP64 block-chain ones).

Checks against the oracle at full size:
- the preconditioner z = M_AS,2^{-1} r element by element against the
  oracle's AdditiveSchwarz (exact local solves) on a seeded r: 1e-11
  relative in 2-norm with FP64 local solves, 3e-2 with the single bf16
  inverse (its entries carry 2^-9 relative rounding; the bar of the small
  cases).  For bf16 also node by node against a model of the bf16
  arithmetic written here from the definition: the inverse of the unclipped
  box and the restricted residuals rounded to bf16 as the device rounds them
  (double -> float -> bf16, both to nearest even), their products exact, plus
  the oracle's coarse correction.  On every node covered by interior
  subdomains only, the device must agree with that model to the FP32
  accumulation bound 4 sqrt(m) 2^-24 sum_k |r~_k||B~_ke| (m terms per output),
  which a wrong tile, K split or row order exceeds by orders of magnitude;
- PCG iteration counts of A_sigma u = M 1 from u = 0 to rtol 1e-10 against
  the oracle's count with exact local solves (stored by make_golden.py):
  +-1 (2-D) / +-2 (3-D) with FP64 local solves; with bf16 local solves at
  most 15% + 2 above it (the rounded preconditioner is a perturbation of the
  exact one; a broken tile would cost far more or break CG down);
- config 2: the eigenvector against the oracle's own eigenvector (banded
  Cholesky inverse iteration, recomputed here): ||x - x_ref||_M <= 1e-8 and
  the eigenvalue to 1e-10 relative, for bf16 and FP64 local solves;
- configs 3 and 4: sigma from the oracle's cell problem (1e-12 relative), the
  stored oracle eigenpair (tests/golden/oracle_config<c>.json, written by
  make_golden.py from the oracle alone): lambda to 1e-10 relative and the
  eigenvector at 256 seeded sample nodes to 1e-8; and properties of an
  eigenpair with the oracle's own assembled A and M: the Rayleigh quotient
  x^T A x / x^T M x equals lambda (1e-10 relative), the relative spectral
  residual is small, sigma < lambda, the ground state is positive, and
  sampled rows of A_sigma x match apply_op.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _golden(c):
    path = os.path.join(HERE, "golden", f"oracle_config{c}.json")
    return json.load(open(path)) if os.path.exists(path) else None


_ORACLE = {}


def _oracle_problem(c):
    """The oracle's problem and two-level preconditioner of configuration c (cached)."""
    if c not in _ORACLE:
        from oracle.problem import Problem
        P = Problem(W.config(c), route="kron")
        _ORACLE[c] = (P, P.preconditioner(True))
    return _ORACLE[c]


def _oracle_mats(c):
    from oracle.fem import Grid, assemble_kron
    from oracle.potential import kron_terms
    cfg = W.config(c)
    g = Grid(cfg["p"], cfg["q"], cfg["L"], cfg["ne"])
    K, M, MV = assemble_kron(g, kron_terms(cfg["V"], cfg["p"], cfg["q"]))
    return g, (K + MV).tocsr(), M.tocsr()


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _assemble(c, prec, graphs=True):
    import paper_2311_08757_amd as dd
    cfg = W.config(c)
    return dd.assemble(cfg["p"], cfg["q"], cfg["L"], cfg["ne"], cfg["V"], cfg["delta"],
                       local_prec=prec, graphs=graphs)


def _solve(torch, c, prec):
    import paper_2311_08757_amd as dd
    prob = _assemble(c, prec)
    sigma, _ = dd.cell_shift(prob)
    x = torch.zeros(prob.n_dof, dtype=torch.float64, device="cuda")
    out = dd.inverse_iteration(prob, x, tol_x=1e-9, rtol_inner=1e-10, maxit_inner=3000)
    return prob, sigma, out, x


def _check_eigenpair(torch, c, prec, sigma, out, xd, prob):
    import paper_2311_08757_amd as dd
    g, A, M = _oracle_mats(c)
    x = xd.cpu().numpy()
    lam = out["lam"]
    # Rayleigh quotient and spectral residual with the oracle's matrices
    Ax, Mx = A @ x, M @ x
    rq = float(x @ Ax) / float(x @ Mx)
    assert abs(rq - lam) <= 1e-10 * abs(lam)
    res = np.linalg.norm(Ax - lam * Mx) / np.linalg.norm(lam * Mx)
    assert res <= 1e-6
    assert sigma < lam
    assert abs(float(x @ Mx) - 1.0) <= 1e-10
    assert np.all(x > 0.0)
    # sampled rows of A_sigma x against the device stencil
    y = torch.empty_like(xd)
    dd.apply_op(prob, "A_sigma", xd, y)
    torch.cuda.synchronize()
    idx = np.random.default_rng(11 + c).choice(g.n, size=512, replace=False)
    As = (A[idx] - sigma * M[idx]).tocsr()
    scale = float(abs(As).sum(axis=1).max()) * float(np.max(np.abs(x)))
    assert np.max(np.abs(y.cpu().numpy()[idx] - As @ x)) <= 1e-13 * scale
    gd = _golden(c)
    if gd is not None:
        assert abs(lam - gd["lam"]) <= 1e-10 * abs(gd["lam"])
        xs = x[gd["sample_idx"]]
        assert np.max(np.abs(xs - np.array(gd["sample_x"]))) <= 1e-8


def _bf16(a):
    """Round to bf16 as the device does: double -> float (nearest even), then
    float -> bf16 (nearest even on the upper 16 bits); returned as float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_model_check(P, AS, r, z):
    """Node-by-node agreement of the device's bf16 local solves with the bf16
    model on the nodes that only interior (unclipped) subdomains cover."""
    n = P.grid.n
    m = max(s.size for s in P.subs)
    inter = [i for i, s in enumerate(P.subs) if s.size == m]
    box = P.subs[inter[0]]
    Ab = P.A_sigma[box][:, box].toarray()
    Binv = np.linalg.inv(Ab)
    Bt = _bf16(0.5 * (Binv + Binv.T))
    del Binv, Ab
    R = np.stack([_bf16(r[P.subs[i]]) for i in inter])
    Z, Zabs = R @ Bt, np.abs(R) @ np.abs(Bt)
    zl, za = np.zeros(n), np.zeros(n)
    for row, i in enumerate(inter):
        zl[P.subs[i]] += Z[row]
        za[P.subs[i]] += Zabs[row]
    clipped = np.zeros(n, dtype=bool)
    for i, s in enumerate(P.subs):
        if s.size != m:
            clipped[s] = True
    coarse = AS.R0T @ AS.coarse_solve(AS.R0T.T @ r)
    ze = zl + coarse
    bound = 4.0 * math.sqrt(m) * 2.0 ** -24 * za + 1e-12 * np.max(np.abs(coarse))
    mask = ~clipped
    assert mask.sum() > 0.9 * n
    err = np.abs(z - ze)
    bad = np.flatnonzero(mask & (err > bound))
    assert bad.size == 0, (bad[:10], err[bad[:10]], bound[bad[:10]])
    return np.median(np.abs(zl - (AS.apply(r) - coarse))[mask]), np.median(bound[mask])


def _precond_fullsize(torch, c, prec):
    import paper_2311_08757_amd as dd
    P, AS = _oracle_problem(c)
    prob = _assemble(c, prec)
    assert prob.n_dof == P.grid.n
    dd.set_shift(prob, P.sigma, P.cell["psi"])
    r = W.random_vector(P.grid.n, 7)
    z = torch.empty(P.grid.n, dtype=torch.float64, device="cuda")
    print(f"# config {c} apply_precond {prec} n={P.grid.n}", flush=True)
    dd.apply_precond(prob, _dev(torch, r), z)
    torch.cuda.synchronize()
    zg = z.cpu().numpy()
    zr = AS.apply(r)
    tol = {"fp64": 1e-11, "bf16": 3e-2}[prec]
    assert np.linalg.norm(zg - zr) <= tol * np.linalg.norm(zr)
    if prec == "bf16":
        _bf16_model_check(P, AS, r, zg)


def _pcg_count(torch, c, prec):
    import paper_2311_08757_amd as dd
    gd = _golden(c)
    ref = gd["pcg_iters_M1"]
    prob = _assemble(c, prec)
    dd.cell_shift(prob)
    one = torch.ones(prob.n_dof, dtype=torch.float64, device="cuda")
    b = torch.empty_like(one)
    dd.apply_op(prob, "M", one, b)
    x = torch.zeros_like(one)
    print(f"# config {c} pcg {prec}", flush=True)
    out = dd.pcg_solve(prob, b, x, rtol=1e-10, maxit=3000)
    assert out["true_relres"] <= 1.1e-10
    if prec == "fp64":
        assert abs(out["iters"] - ref) <= (1 if W.config(c)["p"] + W.config(c)["q"] == 2 else 2)
    else:
        assert ref - 2 <= out["iters"] <= math.ceil(1.15 * ref) + 2, (out["iters"], ref)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["bf16", "fp64"])
def test_config2_precond(torch, prec):
    """2-D L = 256, h = 1/64: the bench's preconditioner (ld = 4480, K split 3,
    35 x 2 tiles in XCD-paired order, the clipped-class corrections, the coarse
    right-hand side inside the GEMM launch) against the oracle."""
    _precond_fullsize(torch, 2, prec)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["bf16", "fp64"])
def test_config2_pcg_count(torch, prec):
    _pcg_count(torch, 2, prec)


@pytest.fixture(scope="module")
def oracle2_eig():
    from oracle.ipm import inverse_iteration_direct
    P, _ = _oracle_problem(2)
    return P, inverse_iteration_direct(P.A, P.M, P.sigma, P.grid, tol=1e-13, maxit=200)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["bf16", "fp64"])
def test_config2_eigenpair(torch, prec, oracle2_eig):
    """2-D L = 256, h = 1/64 (1,032,129 unknowns): the bench workload."""
    P, ref = oracle2_eig
    gd = _golden(2)
    prob, sigma, out, x = _solve(torch, 2, prec)
    assert abs(sigma - gd["sigma"]) <= 1e-12 * abs(gd["sigma"])
    _check_eigenpair(torch, 2, prec, sigma, out, x, prob)
    assert abs(out["lam"] - ref["lam"]) <= 1e-10 * abs(ref["lam"])
    d = x.cpu().numpy() - ref["x"]
    assert math.sqrt(float(d @ (P.M @ d))) <= 1e-8


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_config3_eigenpair(torch, prec):
    """3-D p = 1, q = 2, L = 64, h = 1/32 (1,967,167 unknowns), FP32 / FP64 chain local solves."""
    from oracle.cell import cell_problem
    cfg = W.config(3)
    cell = cell_problem(cfg["p"], cfg["q"], cfg["ne"], cfg["V"], route="kron")
    prob, sigma, out, x = _solve(torch, 3, prec)
    assert abs(sigma - cell["sigma"]) <= 1e-12 * abs(cell["sigma"])
    _check_eigenpair(torch, 3, prec, sigma, out, x, prob)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["bf16", "fp64"])
def test_config4_precond(torch, prec):
    """3-D p = 2, q = 1, L = 16, h = 1/16: 196 interior subdomains on the GEMM,
    56 edge and 4 corner subdomains through the clipped-class corrections."""
    _precond_fullsize(torch, 4, prec)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["bf16", "fp64"])
def test_config4_pcg_count(torch, prec):
    _pcg_count(torch, 4, prec)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["bf16", "fp64"])
def test_config4_eigenpair(torch, prec):
    """3-D p = 2, q = 1, L = 16, h = 1/16 (975,375 unknowns)."""
    from oracle.cell import cell_problem
    cfg = W.config(4)
    cell = cell_problem(cfg["p"], cfg["q"], cfg["ne"], cfg["V"], route="kron")
    prob, sigma, out, x = _solve(torch, 4, prec)
    assert abs(sigma - cell["sigma"]) <= 1e-12 * abs(cell["sigma"])
    _check_eigenpair(torch, 4, prec, sigma, out, x, prob)
