"""Pins of the oracle's Q1 discretisation (§2, eq:discrete-weak-form; Q1 on
Cartesian grids as in §4.1 and §4.3).

Each pin is something other than the oracle itself: hand-derived stencil
constants, a brute-force route through global hat functions, the closed-form
spectrum of the V = 0 operator, the exact shift of the spectrum under a
constant potential (§1), and the reduction of a separable potential (§4.3) to
one-dimensional problems.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle.fem import Grid, assemble_elements, assemble_kron
from oracle.potential import vfun, kron_terms


def mu(theta, h):
    """Generalised eigenvalue of the 1-D linear-element pair (K1, M1) on the
    mode with phase theta: K1 has symbol (2/h)(1 - cos), M1 has (h/3)(2 + cos)."""
    return (6.0 / h ** 2) * (1.0 - np.cos(theta)) / (2.0 + np.cos(theta))


def interior_index(grid, node):
    """Canonical index of an interior node given by 1-based indices."""
    idx = [node[a] - 1 for a in range(grid.d)]
    return int(grid.linear_index([np.array(i) for i in idx]))


def test_2d_stencils_v0():
    # Q1 on squares: stiffness stencil (1/3)[[-1,-1,-1],[-1,8,-1],[-1,-1,-1]]
    # (independent of h in 2-D) and mass stencil h^2/36 [[1,4,1],[4,16,4],[1,4,1]].
    g = Grid(1, 1, 2, 4)
    K, M, MV = assemble_elements(g, vfun(W.const(0.0), 1, 1))
    h = g.h
    kst = np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]]) / 3.0
    mst = np.array([[1, 4, 1], [4, 16, 4], [1, 4, 1]]) * h * h / 36.0
    c = interior_index(g, (3, 2))
    for dx, dy in itertools.product((-1, 0, 1), repeat=2):
        j = interior_index(g, (3 + dx, 2 + dy))
        assert K[c, j] == pytest.approx(kst[dy + 1, dx + 1], abs=1e-14)
        assert M[c, j] == pytest.approx(mst[dy + 1, dx + 1], abs=1e-16)
    assert abs(MV).max() == 0.0


def _hat(z, node, h):
    return np.prod([np.maximum(0.0, 1.0 - np.abs(z[a] - node[a]) / h) for a in range(len(node))], axis=0)


def _grad_hat(z, node, h, a):
    d = len(node)
    out = np.ones_like(z[0])
    for b in range(d):
        if b == a:
            s = np.where(np.abs(z[b] - node[b]) < h, -np.sign(z[b] - node[b]) / h, 0.0)
            out = out * s
        else:
            out = out * np.maximum(0.0, 1.0 - np.abs(z[b] - node[b]) / h)
    return out


@pytest.mark.parametrize("p,q,L,ne", [(1, 1, 2, 3), (1, 2, 2, 2), (2, 1, 2, 2)])
def test_bruteforce_hat_functions(p, q, L, ne):
    """Route (iii): integrate products of global hat functions element by
    element (gradients with a 3-point rule, exact for these polynomials; V with
    the 2-point Gauss rule at cell-local x) and compare with both routes."""
    spec = W.sep_fourier(11) if p == 1 else W.fourier2(12)
    g = Grid(p, q, L, ne)
    h, d = g.h, g.d
    V = vfun(spec, p, q)
    nodes = list(itertools.product(*[range(1, m) for m in g.nel]))
    idx = [interior_index(g, nd) for nd in nodes]
    n = g.n
    Kb = np.zeros((n, n)); Mb = np.zeros((n, n)); Vb = np.zeros((n, n))
    x3, w3 = np.polynomial.legendre.leggauss(3)
    x2, w2 = np.polynomial.legendre.leggauss(2)
    for e in itertools.product(*[range(m) for m in g.nel]):
        lo = np.array(e) * h
        P3 = np.array(list(itertools.product(*[0.5 * h * (x3 + 1)] * d))) + lo
        W3 = np.array([np.prod(t) for t in itertools.product(*[0.5 * h * w3] * d)])
        P2 = np.array(list(itertools.product(*[0.5 * h * (x2 + 1)] * d))) + lo
        W2 = np.array([np.prod(t) for t in itertools.product(*[0.5 * h * w2] * d)])
        z3 = [P3[:, a] for a in range(d)]
        z2 = [P2[:, a] for a in range(d)]
        zc = [np.mod(z2[a], 1.0) if a < p else z2[a] for a in range(d)]
        # cell-local x: element index mod n_e times h plus the offset inside the element
        for a in range(p):
            zc[a] = (e[a] % ne) * h + (z2[a] - lo[a])
        Vq = V(zc)
        near = [k for k, nd in enumerate(nodes)
                if all(e[a] <= nd[a] * 1 <= e[a] + 1 for a in range(d))]
        for i in near:
            ni = np.array(nodes[i]) * h
            for j in near:
                nj = np.array(nodes[j]) * h
                Kb[idx[i], idx[j]] += sum(np.sum(W3 * _grad_hat(z3, ni, h, a) * _grad_hat(z3, nj, h, a))
                                          for a in range(d))
                Mb[idx[i], idx[j]] += np.sum(W3 * _hat(z3, ni, h) * _hat(z3, nj, h))
                Vb[idx[i], idx[j]] += np.sum(W2 * Vq * _hat(z2, ni, h) * _hat(z2, nj, h))
    for route in ("elements", "kron"):
        if route == "elements":
            K, M, MV = assemble_elements(g, V)
        else:
            K, M, MV = assemble_kron(g, kron_terms(spec, p, q))
        assert np.abs(K.toarray() - Kb).max() <= 1e-12 * np.abs(Kb).max()
        assert np.abs(M.toarray() - Mb).max() <= 1e-12 * np.abs(Mb).max()
        assert np.abs(MV.toarray() - Vb).max() <= 1e-12 * np.abs(Vb).max()


@pytest.mark.parametrize("p,q,spec", [
    (1, 1, W.sep_fourier(1000)), (1, 2, W.sep_fourier(3000)), (2, 1, W.fourier2(4000)),
    (1, 1, W.sin4()), (2, 1, W.sep_sum_43())])
def test_routes_agree(p, q, spec):
    g = Grid(p, q, 3, 6)
    K1, M1, V1 = assemble_elements(g, vfun(spec, p, q))
    K2, M2, V2 = assemble_kron(g, kron_terms(spec, p, q))
    for a, b in ((K1, K2), (M1, M2), (V1, V2)):
        assert abs(a - b).max() <= 1e-13 * max(abs(a).max(), 1e-300)


@pytest.mark.parametrize("p,q,L,ne", [(1, 1, 3, 5), (1, 2, 2, 3), (2, 1, 2, 3)])
def test_v0_spectrum_closed_form(p, q, L, ne):
    """V = 0: the Q1 generalised eigenvalues are sums of mu(j pi h / (L or ell))."""
    g = Grid(p, q, L, ne)
    K, M, _ = assemble_elements(g, vfun(W.const(0.0), p, q))
    w = sla.eigh(K.toarray(), M.toarray(), eigvals_only=True)
    h = g.h
    sets = [[mu(j * np.pi / m, h) for j in range(1, m)] for m in g.nel]
    ref = np.sort([sum(t) for t in itertools.product(*sets)])
    assert np.allclose(w, ref, rtol=1e-11, atol=1e-9)


def test_constant_potential_shifts_spectrum():
    """A constant shift of V shifts every eigenvalue by the same constant (§1)."""
    g = Grid(1, 1, 2, 4)
    K, M, V0 = assemble_elements(g, vfun(W.sep_fourier(5), 1, 1))
    _, _, Vc = assemble_elements(g, vfun(W.const(3.25), 1, 1))
    w0 = sla.eigh((K + V0).toarray(), M.toarray(), eigvals_only=True)
    w1 = sla.eigh((K + V0 + Vc).toarray(), M.toarray(), eigvals_only=True)
    assert np.allclose(w1 - w0, 3.25, rtol=0, atol=1e-10)


def _eig1d_dirichlet(nel, h, f, per_ne=None):
    """Smallest generalised eigenvalue of the 1-D problem -u'' + f u with zero
    Dirichlet ends, built here by a plain element loop with 2-point Gauss."""
    n = nel - 1
    A = np.zeros((nel + 1, nel + 1)); B = np.zeros((nel + 1, nel + 1))
    xg, wg = np.polynomial.legendre.leggauss(2)
    for e in range(nel):
        base = ((e % per_ne) if per_ne else e) * h
        for xi, wi in zip(0.5 * (xg + 1), 0.5 * wg):
            z = base + h * xi
            N = np.array([1 - xi, xi])
            A[e:e + 2, e:e + 2] += h * wi * f(z) * np.outer(N, N)
        A[e:e + 2, e:e + 2] += np.array([[1, -1], [-1, 1]]) / h
        B[e:e + 2, e:e + 2] += np.array([[2, 1], [1, 2]]) * h / 6
    return sla.eigh(A[1:n + 1, 1:n + 1], B[1:n + 1, 1:n + 1], eigvals_only=True)[0]


def test_separable_sum_reduces_to_1d():
    """The §4.3 potential is a sum of one-variable functions, so with tensor
    Q1 and tensor Gauss quadrature the 3-D lambda_1 is the sum of three 1-D ones."""
    spec = W.sep_sum_43()
    L, ne = 2, 5
    g = Grid(2, 1, L, ne)
    K, M, MV = assemble_elements(g, vfun(spec, 2, 1))
    lam = sla.eigh((K + MV).toarray(), M.toarray(), eigvals_only=True, subset_by_index=[0, 0])[0]
    h = g.h
    fx = lambda x: 10 * np.sin(2 * np.pi * x) + 10 * np.sin(4 * np.pi * x)
    fy = lambda x: 20 * np.sin(2 * np.pi * x) + 20 * np.sin(4 * np.pi * x)
    fz = lambda z: 10 * z
    ref = 40.0 + _eig1d_dirichlet(L * ne, h, fx, ne) + _eig1d_dirichlet(L * ne, h, fy, ne) \
        + _eig1d_dirichlet(ne, h, fz)
    assert lam == pytest.approx(ref, rel=1e-12)


def test_shifted_operator_spd():
    """A_sigma = A - sigma M is SPD for sigma below lambda_1 (§3)."""
    from oracle.cell import cell_problem
    cfg = W.small_config(1, 1, 3, 6, 2, W.sep_fourier(21))
    g = Grid(1, 1, 3, 6)
    K, M, MV = assemble_elements(g, vfun(cfg["V"], 1, 1))
    sig = cell_problem(1, 1, 6, cfg["V"])["sigma"]
    As = (K + MV - sig * M).toarray()
    assert np.abs(As - As.T).max() == 0.0
    np.linalg.cholesky(As)
