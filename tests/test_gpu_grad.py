"""GPU parity of the parameter derivatives (paper_2311_08757_amd.autograd,
ddeig_potential_form) against the oracle's own derivative forms.

- ddeig_potential_form against x^T M_W y with the oracle's element-loop
  M_W, on seeded vectors, on the global grid and on the periodic cell:
  1e-12 of |x|^T |M_W| |y| (FP64 sums in a different order).
- EigenvalueFn backward (Hellmann-Feynman on the GPU eigenvector) against
  the oracle's Hellmann-Feynman form on its exactly solved eigenvector:
  1e-9 relative (of max |grad|); and against central finite differences of
  the GPU eigenvalue with step 1e-6: 2e-6 of max(1, max |grad|) (rounding of
  lambda / step dominates).
- ShiftedSolveFn backward (adjoint PCG + shift derivative) against the
  oracle's adjoint form with direct solves: 1e-9 relative.
- instances of the batched workload (2-D, L_j in 16..256, n_e = 32,
  delta = 2, bf16 local solves): lambda_j and dlambda_j/dtheta one by one,
  and all 64 as one batch (BatchEigenvaluesFn: grouped inverse iteration and
  one grouped launch of the Hellmann-Feynman forms) against the oracle's
  Hellmann-Feynman derivative stored by make_golden.py (1e-9 relative), two
  of them against central differences of the batched eigenvalue (step 1e-6);
  the batched shifted solve and its adjoint (BatchShiftedSolveFn) against
  the oracle's adjoint form with direct solves (1e-9 relative).
- ddeig_shift_grad against the oracle's cell Hellmann-Feynman form.
"""
import json
import os
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

CASES = [
    # p, q, L, ne, delta, potential
    (1, 1, 4, 8, 2, W.sep_fourier(1000)),
    (1, 2, 3, 4, 1, W.sep_fourier(3000)),
    (2, 1, 3, 4, 1, W.fourier2(4000)),
]
IDS = [f"p{c[0]}q{c[1]}-L{c[2]}-ne{c[3]}-{c[5]['kind']}" for c in CASES]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _geom(case):
    p, q, L, ne, delta, V = case
    return dict(p=p, q=q, L=L, ne=ne, delta=delta, V=V)


def _scale(g):
    return max(1.0, float(np.max(np.abs(g))))


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("space", ["global", "cell"])
def test_potential_form(torch, case, space):
    import paper_2311_08757_amd as dd
    from paper_2311_08757_amd import autograd as AG
    from oracle.fem import Grid, assemble_elements
    from oracle.potential import vfun
    p, q, L, ne, delta, V = case
    prob = dd.assemble(p, q, L, ne, V, delta)
    g = Grid(p, q, L, ne) if space == "global" else Grid(p, q, 1, ne, cell=True)
    n = g.n
    assert n == (prob.n_dof if space == "global" else prob.n_cell)
    x, y = W.random_vector(n, 31), W.random_vector(n, 32)
    T = len(V["a"])
    Ws = [AG.dpotential(V, 0), AG.dpotential(V, T - 1), AG.dpotential(V, T),
          AG.dpotential(V, 2 * T - 1), V, W.const(1.0), W.const(-2.5)]
    for Wp in Ws:
        got = dd.potential_form(prob, Wp, _dev(torch, x), _dev(torch, y), space)
        _, _, MW = assemble_elements(g, vfun(Wp, p, q), with_kinetic=False)
        ref = float(x @ (MW @ y))
        bound = float(np.abs(x) @ (abs(MW) @ np.abs(y)))
        assert abs(got - ref) <= 1e-12 * bound, (Wp, got, ref)


def test_potential_form_errors(torch):
    import paper_2311_08757_amd as dd
    p, q, L, ne, delta, V = CASES[0]
    prob = dd.assemble(p, q, L, ne, V, delta)
    x = torch.zeros(prob.n_dof, dtype=torch.float64, device="cuda")
    with pytest.raises(dd.DdeigError):
        dd.potential_form(prob, V, x, x, space=2)
    with pytest.raises(dd.DdeigError):
        dd.potential_form(prob, W.fourier2(1), x, x)      # FOURIER2 needs p = 2
    bad = dict(V, a=[float("nan")] + list(V["a"][1:]))
    with pytest.raises(dd.DdeigError):
        dd.potential_form(prob, bad, x, x)
    with pytest.raises(ValueError):
        dd.potential_form(prob, V, x[:-1], x)


def _oracle_eig(case):
    from oracle import grad as G
    from oracle.fem import assemble_kron
    from oracle.potential import kron_terms
    from oracle.cell import cell_problem
    from oracle.ipm import inverse_iteration_direct
    p, q, L, ne, delta, V = case
    g = G.grid_of(dict(p=p, q=q, L=L, ne=ne))
    K, M, MV = assemble_kron(g, kron_terms(V, p, q))
    cell = cell_problem(p, q, ne, V, route="kron")
    res = inverse_iteration_direct((K + MV).tocsr(), M, cell["sigma"], g if g.d == 2 else None,
                                   tol=1e-13, maxit=300)
    return res["lam"], G.eigenvalue_grad(g, M, res["x"], V)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_eigenvalue_grad(torch, case):
    from paper_2311_08757_amd import autograd as AG
    V = case[5]
    theta = torch.tensor(AG.param_vector(V), dtype=torch.float64, requires_grad=True)
    lam = AG.EigenvalueFn.apply(theta, _geom(case), {"tol_x": 1e-12})
    lam.backward()
    lam_ref, g_ref = _oracle_eig(case)
    assert abs(lam.item() - lam_ref) <= 1e-11 * abs(lam_ref)
    g = theta.grad.numpy()
    assert np.max(np.abs(g - g_ref)) <= 1e-9 * np.max(np.abs(g_ref))


def test_eigenvalue_grad_finite_differences(torch):
    """Central differences of the GPU eigenvalue, step 1e-6."""
    from paper_2311_08757_amd import autograd as AG
    case = CASES[0]
    V = case[5]
    th0 = AG.param_vector(V)
    opts = {"tol_x": 1e-12}
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    AG.EigenvalueFn.apply(theta, _geom(case), opts).backward()
    g = theta.grad.numpy()
    h = 1e-6
    fd = np.zeros_like(th0)
    for j in range(th0.size):
        tp, tm = th0.copy(), th0.copy()
        tp[j] += h
        tm[j] -= h
        lp = AG.EigenvalueFn.apply(torch.tensor(tp), _geom(case), opts).item()
        lm = AG.EigenvalueFn.apply(torch.tensor(tm), _geom(case), opts).item()
        fd[j] = (lp - lm) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 2e-6 * _scale(g)


@pytest.mark.parametrize("case", CASES[:2], ids=IDS[:2])
def test_shifted_solve_grad(torch, case):
    import scipy.sparse.linalg as spla
    from paper_2311_08757_amd import autograd as AG
    from oracle import grad as G
    from oracle.cell import cell_problem
    from oracle.fem import assemble_elements
    from oracle.potential import vfun
    p, q, L, ne, delta, V = case
    g = G.grid_of(dict(p=p, q=q, L=L, ne=ne))
    b, c = W.random_vector(g.n, 41), W.random_vector(g.n, 42)
    theta = torch.tensor(AG.param_vector(V), dtype=torch.float64, requires_grad=True)
    bd = _dev(torch, b).requires_grad_(True)
    u = AG.ShiftedSolveFn.apply(theta, bd, _geom(case), {"rtol": 1e-13})
    (u * _dev(torch, c)).sum().backward()
    # oracle: direct solves, its own shift derivative and adjoint form
    K, M, MV = assemble_elements(g, vfun(V, p, q))
    cell = cell_problem(p, q, ne, V)
    As = (K + MV - cell["sigma"] * M).tocsc()
    uo, wo = spla.spsolve(As, b), spla.spsolve(As, c)
    assert np.max(np.abs(u.detach().cpu().numpy() - uo)) <= 1e-8 * np.max(np.abs(uo))
    ref = G.solve_grad(g, M, uo, wo, V, G.shift_grad(cell, V))
    assert np.max(np.abs(theta.grad.numpy() - ref)) <= 1e-9 * np.max(np.abs(ref))
    assert np.max(np.abs(bd.grad.cpu().numpy() - wo)) <= 1e-8 * np.max(np.abs(wo))


def _batch_pick():
    inst = W.batch_config()
    Ls = [c["L"] for c in inst]
    pick = sorted({int(np.argmin(Ls)), int(np.argmax(Ls)), 7, 40})
    return [inst[j] for j in pick]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("inst", _batch_pick(), ids=lambda c: f"{c['name']}-L{c['L']}")
def test_batch_instance_grad(torch, inst):
    """Instances of the batched workload with bf16 local solves."""
    from paper_2311_08757_amd import autograd as AG
    case = (inst["p"], inst["q"], inst["L"], inst["ne"], inst["delta"], inst["V"])
    theta = torch.tensor(AG.param_vector(inst["V"]), dtype=torch.float64, requires_grad=True)
    lam = AG.EigenvalueFn.apply(theta, _geom(case), {"tol_x": 1e-12, "local_prec": "bf16"})
    lam.backward()
    lam_ref, g_ref = _oracle_eig(case)
    assert abs(lam.item() - lam_ref) <= 1e-11 * abs(lam_ref)
    assert np.max(np.abs(theta.grad.numpy() - g_ref)) <= 1e-9 * np.max(np.abs(g_ref))


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_shift_grad(torch, case):
    import paper_2311_08757_amd as dd
    from oracle import grad as G
    from oracle.cell import cell_problem
    p, q, L, ne, delta, V = case
    prob = dd.assemble(p, q, L, ne, V, delta)
    dd.cell_shift(prob)
    g = dd.shift_grad(prob)
    ref = G.shift_grad(cell_problem(p, q, ne, V), V)
    assert np.max(np.abs(g - ref)) <= 1e-9 * np.max(np.abs(ref))


def _geom_of(inst):
    return dict(p=inst["p"], q=inst["q"], L=inst["L"], ne=inst["ne"], delta=inst["delta"],
                V=inst["V"])


@pytest.mark.timeout(900)
def test_batch_eig_grad_all_instances(torch):
    """All 64 instances of the batched workload as one batch, bf16 local solves."""
    from paper_2311_08757_amd import autograd as AG
    inst = W.batch_config()
    gold = json.load(open(os.path.join(HERE, "golden", "oracle_batch.json")))
    thetas = torch.tensor(np.stack([AG.param_vector(c["V"]) for c in inst]), dtype=torch.float64,
                          requires_grad=True)
    print("# batch of 64: forward", flush=True)
    lam = AG.BatchEigenvaluesFn.apply(thetas, [_geom_of(c) for c in inst],
                                      {"tol_x": 1e-12, "local_prec": "bf16"})
    lam.sum().backward()
    g = thetas.grad.numpy()
    for j, gd in enumerate(gold):
        assert abs(lam[j].item() - gd["lam"]) <= 1e-10 * abs(gd["lam"]), j
        ref = np.array(gd["grad"])
        assert np.max(np.abs(g[j] - ref)) <= 1e-9 * np.max(np.abs(ref)), (j, g[j], ref)


@pytest.mark.timeout(900)
def test_batch_eig_grad_finite_differences(torch):
    """Central differences (step 1e-6) of the batched eigenvalues of two
    instances of the batched workload (bf16 local solves) against the batched
    Hellmann-Feynman gradient."""
    from paper_2311_08757_amd import autograd as AG
    inst = W.batch_config()
    Ls = [c["L"] for c in inst]
    pick = [inst[int(np.argmin(Ls))], inst[7]]
    geoms = [_geom_of(c) for c in pick]
    th0 = np.stack([AG.param_vector(c["V"]) for c in pick])
    opts = {"tol_x": 1e-12, "local_prec": "bf16"}
    thetas = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    AG.BatchEigenvaluesFn.apply(thetas, geoms, opts).sum().backward()
    g = thetas.grad.numpy()
    h = 1e-6
    fd = np.zeros_like(th0)
    for k in range(th0.shape[1]):
        tp, tm = th0.copy(), th0.copy()
        tp[:, k] += h
        tm[:, k] -= h
        lp = AG.BatchEigenvaluesFn.apply(torch.tensor(tp), geoms, opts).numpy()
        lm = AG.BatchEigenvaluesFn.apply(torch.tensor(tm), geoms, opts).numpy()
        fd[:, k] = (lp - lm) / (2 * h)
    for j in range(2):
        assert np.max(np.abs(fd[j] - g[j])) <= 2e-6 * _scale(g[j]), (j, fd[j], g[j])


@pytest.mark.timeout(600)
def test_batch_solve_grad(torch):
    """Batched shifted solves and their adjoint against the oracle (direct solves)."""
    import scipy.sparse.linalg as spla
    from paper_2311_08757_amd import autograd as AG
    from oracle import grad as G
    from oracle.cell import cell_problem
    from oracle.fem import assemble_elements
    from oracle.potential import vfun
    cases = [(1, 1, L, 8, 2, W.sep_fourier(600 + L)) for L in (5, 6, 8)]
    geoms = [_geom(c) for c in cases]
    thetas = torch.tensor(np.stack([AG.param_vector(c[5]) for c in cases]), dtype=torch.float64,
                          requires_grad=True)
    grids = [G.grid_of(dict(p=c[0], q=c[1], L=c[2], ne=c[3])) for c in cases]
    bs = [W.random_vector(gr.n, 50 + j) for j, gr in enumerate(grids)]
    cs = [W.random_vector(gr.n, 60 + j) for j, gr in enumerate(grids)]
    bd = [_dev(torch, b).requires_grad_(True) for b in bs]
    u = AG.BatchShiftedSolveFn.apply(thetas, geoms, {"rtol": 1e-13, "local_prec": "bf16"}, *bd)
    (u * _dev(torch, np.concatenate(cs))).sum().backward()
    off = 0
    for j, (c, gr) in enumerate(zip(cases, grids)):
        p, q, L, ne, delta, V = c
        K, M, MV = assemble_elements(gr, vfun(V, p, q))
        cell = cell_problem(p, q, ne, V)
        As = (K + MV - cell["sigma"] * M).tocsc()
        uo, wo = spla.spsolve(As, bs[j]), spla.spsolve(As, cs[j])
        uj = u.detach()[off:off + gr.n].cpu().numpy()
        off += gr.n
        assert np.max(np.abs(uj - uo)) <= 1e-8 * np.max(np.abs(uo))
        ref = G.solve_grad(gr, M, uo, wo, V, G.shift_grad(cell, V))
        assert np.max(np.abs(thetas.grad.numpy()[j] - ref)) <= 1e-9 * np.max(np.abs(ref)), j
        assert np.max(np.abs(bd[j].grad.cpu().numpy() - wo)) <= 1e-8 * np.max(np.abs(wo))
