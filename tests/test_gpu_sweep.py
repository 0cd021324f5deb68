"""The march A_sigma sweeps of wide grids (the 2-D row march and the 3-D
plane march; ddeig_options.sweep 2, and the size-based choice) against the
tile sweep and the oracle.

- A_sigma x, A x, M x and K x from the march equal the tile sweep's bit for bit
  (every output takes its taps in the same order from the same values), on
  grids of one ragged workgroup, of several workgroups with a ragged last one,
  and at the 66,060,225-unknown HBM-scale grid (sweep chosen by size) over the
  whole vector; also with x and y at element offsets within a 128-byte line,
  writing nothing outside y;
- at that size, sampled rows of A_sigma x against the oracle: the operator is
  periodic in x with the period cell's coefficients, so the row of node (i, j)
  is the row of the node with the same cell-local position in a small oracle
  problem on the same cell (the Dirichlet end nodes map to the small
  problem's end nodes); 1e-13 of the row's absolute sum times max |x|; the
  same for the 3-D plane march (p = 1, q = 2, L = 2048, h = 1/32, 62,979,135
  unknowns) and on small 3-D grids (one expanding axis and two);
- the fused direction-update sweep inside PCG: iteration counts within +-1 of
  the oracle's PCG, the true residual below 1.1 rtol, residual histories to
  1e-6, and the eigenpair of inverse iteration to 1e-10 / 1e-8 (M-norm).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CASES = [
    # p, q, L, ne, delta, potential
    (1, 1, 4, 8, 2, W.sep_fourier(1000)),    # 31 columns: one ragged workgroup
    (1, 1, 130, 8, 2, W.sep_fourier(17)),    # 1039 columns: 512 + 512 + 15
    (1, 1, 67, 16, 4, W.sin4()),             # 1071 columns, 15 rows
    (1, 2, 3, 4, 1, W.sep_fourier(3000)),    # 3-D: one ragged 256 x 8 block
    (1, 2, 70, 8, 2, W.sep_fourier(7)),      # 3-D: 559 columns in 3 blocks, 7 x 7 lines
    (2, 1, 3, 4, 1, W.fourier2(4000)),       # 3-D, two expanding axes (y periodic table)
]
IDS = [f"p{c[0]}q{c[1]}-L{c[2]}-ne{c[3]}-d{c[4]}-{c[5]['kind']}" for c in CASES]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _oracle(case):
    from oracle.problem import Problem
    p, q, L, ne, delta, V = case
    return Problem(W.small_config(p, q, L, ne, delta, V))


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _assemble(case, sweep, **kw):
    import paper_2311_08757_amd as dd
    p, q, L, ne, delta, V = case
    return dd.assemble(p, q, L, ne, V, delta, sweep=sweep, **kw)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_march_equals_tiles(torch, case):
    import paper_2311_08757_amd as dd
    pm, pt = _assemble(case, "march"), _assemble(case, "tiles")
    sig, psi = dd.cell_shift(pt)
    dd.set_shift(pm, sig, psi)
    x = _dev(torch, W.random_vector(pm.n_dof, 5))
    for op in ("A_sigma", "A", "M", "K"):
        ym, yt = torch.empty_like(x), torch.empty_like(x)
        dd.apply_op(pm, op, x, ym)
        dd.apply_op(pt, op, x, yt)
        torch.cuda.synchronize()
        assert torch.equal(ym, yt), op


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_march_unaligned_vectors(torch, case):
    """x and y at element offsets within a 128-byte line (views into larger
    buffers): the march gives the tile sweep's bits at every offset and writes
    nothing outside y."""
    import paper_2311_08757_amd as dd
    pm, pt = _assemble(case, "march"), _assemble(case, "tiles")
    sig, psi = dd.cell_shift(pt)
    dd.set_shift(pm, sig, psi)
    n = pm.n_dof
    xb = _dev(torch, W.random_vector(n + 16, 6))
    yt = torch.empty(n, dtype=torch.float64, device="cuda")
    for ox, oy in [(0, 1), (1, 0), (3, 7), (5, 15), (15, 9)]:
        x = xb[ox:ox + n]
        yb = torch.full((n + 16,), float("nan"), dtype=torch.float64, device="cuda")
        y = yb[oy:oy + n]
        dd.apply_op(pt, "A_sigma", x, yt)
        dd.apply_op(pm, "A_sigma", x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, yt), (ox, oy)
        # nothing written outside y
        assert torch.isnan(yb[:oy]).all() and torch.isnan(yb[oy + n:]).all(), (ox, oy)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_march_pcg_and_eigenpair(torch, case):
    import paper_2311_08757_amd as dd
    from oracle.pcg import pcg
    from oracle.ipm import inverse_iteration_direct
    P = _oracle(case)
    prob = _assemble(case, "march")
    dd.set_shift(prob, P.sigma, P.cell["psi"])
    b = W.random_vector(P.grid.n, 8)
    x = torch.zeros(P.grid.n, dtype=torch.float64, device="cuda")
    out = dd.pcg_solve(prob, _dev(torch, b), x, rtol=1e-10, maxit=500, hist_cap=501)
    ref = pcg(lambda v: P.A_sigma @ v, b, P.preconditioner(True).apply, rtol=1e-10, maxit=500)
    assert abs(out["iters"] - ref.iters) <= (1 if P.grid.d == 2 else 2)
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - P.A_sigma @ xs) <= 1.1e-10 * np.linalg.norm(b)
    k = min(out["iters"], ref.iters)
    assert np.allclose(out["hist"][:k + 1], ref.hist[:k + 1], rtol=1e-6, atol=1e-13)
    prob = _assemble(case, "march")
    dd.cell_shift(prob)
    u = torch.zeros(P.grid.n, dtype=torch.float64, device="cuda")
    eo = dd.inverse_iteration(prob, u, tol_x=1e-9, rtol_inner=1e-10)
    er = inverse_iteration_direct(P.A, P.M, P.sigma, P.grid if P.grid.d == 2 else None)
    assert abs(eo["lam"] - er["lam"]) <= 1e-10 * abs(er["lam"])
    d = u.cpu().numpy() - er["x"]
    assert np.sqrt(d @ (P.M @ d)) <= 1e-8


def _hbm_scale(torch, p, q, L, ne, delta, V, Ls):
    """Whole-vector equality of the size-chosen sweep (the march) with the tile
    sweep, and sampled rows against a small oracle problem (L = Ls) on the same
    period cell."""
    import paper_2311_08757_amd as dd
    from oracle.problem import Problem
    case = (p, q, L, ne, delta, V)
    pa = _assemble(case, "auto", coarse=False)
    sig, psi = dd.cell_shift(pa)
    n = pa.n_dof
    N0 = L * ne - 1
    x = torch.randn(n, dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(3))
    ya = torch.empty_like(x)
    dd.apply_op(pa, "A_sigma", x, ya)
    torch.cuda.synchronize()
    ys = ya.cpu().numpy()
    xh = x.cpu().numpy()
    del pa
    pt = _assemble(case, "tiles", coarse=False)
    dd.set_shift(pt, sig, psi)
    yt = torch.empty_like(x)
    dd.apply_op(pt, "A_sigma", x, yt)
    torch.cuda.synchronize()
    assert torch.equal(ya, yt)
    del pt, yt
    Ps = Problem(W.small_config(p, q, Ls, ne, delta, V))
    N0s = Ls * ne - 1
    rest = n // N0          # the other axes, unchanged in the small problem
    assert Ps.grid.n == N0s * rest
    As = (Ps.A - sig * Ps.M).tocsr()
    rng = np.random.default_rng(21)
    ii = np.concatenate([[0, 1, N0 - 2, N0 - 1], rng.integers(0, N0, size=1020)])
    jj = np.concatenate([[0, rest - 1, 0, rest - 1], rng.integers(0, rest, size=1020)])
    xmax = float(np.max(np.abs(xh)))
    for i, j in zip(ii, jj):
        if i == 0:
            i_s = 0
        elif i == N0 - 1:
            i_s = N0s - 1
        else:
            i_s = ne + (i + 1) % ne - 1
        row = As.getrow(i_s + N0s * j)
        cols = row.indices
        d0 = cols % N0s - i_s
        big = (i + d0) + N0 * (cols // N0s)
        expect = float(row.data @ xh[big])
        bar = 1e-13 * float(np.abs(row.data).sum()) * xmax
        assert abs(ys[i + N0 * j] - expect) <= bar, (i, j)


def test_march_hbm_scale_2d(torch):
    """2-D, L = 16384, h = 1/64: 1,048,575 x 63 unknowns (row march)."""
    _hbm_scale(torch, 1, 1, 16384, 64, 4, W.config(2)["V"], 4)


def test_march_hbm_scale_3d(torch):
    """3-D p = 1, q = 2, L = 2048, h = 1/32: 65,535 x 31 x 31 unknowns (plane march)."""
    _hbm_scale(torch, 1, 2, 2048, 32, 2, W.config(3)["V"], 3)
