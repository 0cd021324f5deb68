"""GPU parity at the full workload sizes, in the launch configurations that
bench.py times (config 2: bf16 dense local solves; the FP64 path it compares
with) and for the 3-D workloads (config 3: FP32 or FP64 block-chain local
solves, config 4: bf16 dense local solves through the unclipped-box inverse,
or FP64 block-chain ones).

Checks against the oracle at full size:
- the preconditioner z = M_AS,2^{-1} r element by element against the
  oracle's AdditiveSchwarz (exact local solves) on a seeded r, also split
  into its local part (AS1) and its coarse part: the local part to 1e-11
  relative in 2-norm with FP64 local solves, 3e-2 with the single bf16
  inverse (its entries carry 2^-9 relative rounding; the bar of the small
  cases); the coarse part to 32 kappa(A_0) u (see _precond_fullsize).  For
  bf16 also node by node against a model of the bf16 arithmetic written here
  from the definition: the inverse of the unclipped box and the restricted
  residuals rounded to bf16 as the device rounds them (correctly rounded from
  FP64), their products exact.  On every node covered by interior subdomains
  only, the device's local part must agree with that model to the FP32
  accumulation bound 4 sqrt(m) 2^-24 sum_k |r~_k||B~_ke| (m terms per output),
  which a wrong tile, K split or row order exceeds by orders of magnitude;
- PCG iteration counts of A_sigma u = M 1 from u = 0 to rtol 1e-10 against
  the oracle's count with exact local solves (stored by make_golden.py):
  +-1 (2-D) / +-2 (3-D) with FP64 local solves; with bf16 local solves at
  most 15% + 2 above it (the rounded preconditioner is a perturbation of the
  exact one; a broken tile would cost far more or break CG down); the true
  residual at most rtol + 1.5 x the oracle's own true residual (the FP64
  residual-update floor, 3.8e-8 relative at config 2);
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
    """Round to bf16 as the device does: the FP64 value correctly rounded to 8
    significant bits (nearest, ties to even), in one step from double.  (The
    device's double -> float -> bf16 conversion compiles to one correctly
    rounded conversion: the float step rounds to odd.)  Returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)
    u = ((u + np.uint64((1 << 44) - 1) + ((u >> np.uint64(45)) & np.uint64(1)))
         >> np.uint64(45)) << np.uint64(45)
    return u.view(np.float64)


def _bf16_model_check(P, zloc):
    """Node-by-node agreement of the device's bf16 local solves (the additive
    Schwarz sum without the coarse part) with the bf16 model on the nodes that
    only interior (unclipped) subdomains cover."""
    n = P.grid.n
    m = max(s.size for s in P.subs)
    inter = [i for i, s in enumerate(P.subs) if s.size == m]
    box = P.subs[inter[0]]
    Ab = P.A_sigma[box][:, box].toarray()
    Binv = np.linalg.inv(Ab)
    Bt = _bf16(0.5 * (Binv + Binv.T))
    del Binv, Ab
    r = _RVEC[P.grid.n]
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
    # FP32 accumulation of m products; 1e-13 max|z| for forming zloc on the host
    bound = 4.0 * math.sqrt(m) * 2.0 ** -24 * za + 1e-13 * np.max(np.abs(zl))
    mask = ~clipped
    assert mask.sum() > 0.5 * n
    err = np.abs(zloc - zl)
    bad = np.flatnonzero(mask & (err > bound))
    assert bad.size == 0, (bad[:10], err[bad[:10]], bound[bad[:10]])


_RVEC = {}


def _precond_fullsize(torch, c, prec):
    """z = M_AS,2^{-1} r and its two parts (the local solves, ddeig_apply_schwarz
    AS1; the coarse correction, COARSE) against the oracle.  The local part
    meets the bar of the precision; the coarse part R_0^T A_0^{-1} R_0 r is as
    sensitive to rounding as A_0 is ill-conditioned (A_0 annihilates the
    periodic ground state up to lambda_1 - sigma), so it is held to
    32 kappa(A_0) u of its norm: 32 u bounds the relative rounding of the
    assembled A_0 (two summation orders of R_0^T A_sigma R_0 already differ by
    about 22 u at config 2), kappa(A_0) from the oracle's A_0."""
    import paper_2311_08757_amd as dd
    P, AS = _oracle_problem(c)
    prob = _assemble(c, prec)
    assert prob.n_dof == P.grid.n
    dd.set_shift(prob, P.sigma, P.cell["psi"])
    r = W.random_vector(P.grid.n, 7)
    _RVEC[P.grid.n] = r
    rd = _dev(torch, r)
    z, zl, zc = (torch.empty(P.grid.n, dtype=torch.float64, device="cuda") for _ in range(3))
    print(f"# config {c} apply_precond {prec} n={P.grid.n}", flush=True)
    dd.apply_precond(prob, rd, z)
    dd.apply_schwarz(prob, "as1", rd, zl)
    dd.apply_schwarz(prob, "coarse", rd, zc)
    torch.cuda.synchronize()
    zg, zlg, zcg = z.cpu().numpy(), zl.cpu().numpy(), zc.cpu().numpy()
    cref = AS.R0T @ AS.coarse_solve(AS.R0T.T @ r)
    zr = AS.apply(r)
    lref = zr - cref
    ev = np.linalg.eigvalsh(AS.A0)
    bar_c = 32.0 * (ev[-1] / ev[0]) * 2.0 ** -53 * np.linalg.norm(cref)
    assert np.linalg.norm(zcg - cref) <= bar_c
    tol = {"fp64": 1e-11, "bf16": 3e-2}[prec]
    assert np.linalg.norm(zlg - lref) <= tol * np.linalg.norm(lref)
    assert np.linalg.norm(zg - zr) <= tol * np.linalg.norm(zr) + bar_c
    # the bench's fused launch (coarse space riding in the dense launches)
    # against the separate parts: the same arithmetic, bitwise up to the final sum
    assert np.max(np.abs(zg - (zlg + zcg))) <= 1e-13 * np.max(np.abs(zg))
    if prec == "bf16":
        _bf16_model_check(P, zg - zcg)


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
    # the recursively updated residual drifts from b - A_sigma x by the rounding
    # of the updates (u ||A|| ||x|| with ||x|| ~ ||b|| / (lambda_1 - sigma)); the
    # oracle's own FP64 PCG ends at the same floor, so the true residual is held
    # to rtol or to that floor
    assert out["true_relres"] <= 1.1e-10 + 1.5 * gd["pcg_true_relres_M1"]
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
