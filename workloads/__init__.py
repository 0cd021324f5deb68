"""Seeded synthetic workloads shared by the oracle and the GPU library.

This module holds configuration data and random draws only -- none of the
method's arithmetic.  Both sides read their inputs from here; neither imports
the other.

Every workload is an analytic potential on a box (0,L)^p x (0,ell)^q, as in
the paper's experiments (§4); no dataset is involved.  Random coefficients
come from ``numpy.random.default_rng(seed)``: amplitudes are drawn first,
then phases.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def sep_fourier(seed, nterms=4, amax=10.0, cy=0.5):
    """V = sum_k a_k cos(2 pi k x1 + phi_k) (1 + cy prod_j sin(pi y_j))."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, amax, nterms)
    phi = rng.uniform(0.0, TWO_PI, nterms)
    return {"kind": "sep_fourier", "a": a.tolist(), "phi": phi.tolist(),
            "k": list(range(1, nterms + 1)), "cy": float(cy)}


def fourier2(seed, kmax=3, amax=5.0):
    """V = sum_{(k,m) in {0..kmax}^2 \\ (0,0)} a_km cos(2 pi (k x1 + m x2) + phi_km)."""
    km = [(k, m) for m in range(kmax + 1) for k in range(kmax + 1) if (k, m) != (0, 0)]
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, amax, len(km))
    phi = rng.uniform(0.0, TWO_PI, len(km))
    return {"kind": "fourier2", "a": a.tolist(), "phi": phi.tolist(),
            "k": [k for k, _ in km], "m": [m for _, m in km]}


def sin4(amp=100.0):
    """The §4.1 potential amp * sin^4(pi x) sin^4(pi y)."""
    return {"kind": "sin4", "amp": float(amp)}


def sep_sum_43():
    """The §4.3 potential 10 (4 + sin 2pi x + sin 4pi x + 2 sin 2pi y + 2 sin 4pi y + z).

    Here (x, y) are the two expanding directions x1, x2 and z is the fixed one.
    """
    return {"kind": "sep_sum", "c0": 40.0,
            "terms": [[10.0, 0, 1], [10.0, 0, 2], [20.0, 1, 1], [20.0, 1, 2]],
            "g": [10.0]}


def const(c):
    return {"kind": "const", "c": float(c)}


def config(cfg):
    """The five configurations: geometry, mesh, overlap and potential."""
    if cfg == 1:
        return dict(name="2d-L8-ne32", p=1, q=1, L=8, ell=1, ne=32, delta=2, V=sep_fourier(1000))
    if cfg == 2:
        return dict(name="2d-L256-ne64", p=1, q=1, L=256, ell=1, ne=64, delta=4, V=sep_fourier(2000))
    if cfg == 3:
        return dict(name="3d-p1q2-L64-ne32", p=1, q=2, L=64, ell=1, ne=32, delta=2, V=sep_fourier(3000))
    if cfg == 4:
        return dict(name="3d-p2q1-L16-ne16", p=2, q=1, L=16, ell=1, ne=16, delta=1, V=fourier2(4000))
    raise ValueError(cfg)


def batch_config(n_instances=64, seed=5000):
    """Config 5: independent 2-D instances with L_j uniform in 16..256, n_e=32, delta=2."""
    Ls = np.random.default_rng(seed).integers(16, 257, size=n_instances)
    return [dict(name=f"2d-batch-{j}", p=1, q=1, L=int(Ls[j]), ell=1, ne=32, delta=2,
                 V=sep_fourier(seed + 1 + j)) for j in range(n_instances)]


def quad_points(p, q, ne, ell=1):
    """Coordinates (one array per axis) of the quadrature points of one period
    cell, in the order of a tabulated potential: the cell's elements (n_e per
    expanding, ell n_e per fixed direction) lexicographically with axis 0
    fastest, in each element its 2^(p+q) tensor 2-point Gauss points with point
    index sum_a b_a 2^a, b_a = 0 at (e_a + (1 - 1/sqrt 3) / 2) h."""
    d = p + q
    h = 1.0 / ne
    nel = [ne] * p + [int(round(ell * ne))] * q
    off = (0.5 * (1.0 - 1.0 / np.sqrt(3.0)), 0.5 * (1.0 + 1.0 / np.sqrt(3.0)))
    E = np.meshgrid(*[np.arange(m) for m in nel], indexing="ij")
    E = [e.ravel(order="F") for e in E]
    out = []
    for a in range(d):
        pts = np.array([off[(qi >> a) & 1] for qi in range(2 ** d)])
        out.append(((E[a][:, None] + pts[None, :]) * h).ravel())
    return out


def quad_table(p, q, ne, ell, values):
    """A tabulated potential dict from values at quad_points(p, q, ne, ell)."""
    values = np.ascontiguousarray(values, dtype=np.float64)
    return {"kind": "quad_table", "p": p, "q": q, "ne": ne, "ell": ell, "table": values}


def coulomb_well(p, q, ne, ell=1, Z=1.0, b=1e-4):
    """A truncated Coulomb well at the centre c of every period cell,
    V = -Z / max(|z - c|, b) (the radial potential of §4.2, Z = 1, b = 1e-4)."""
    z = quad_points(p, q, ne, ell)
    r2 = sum((z[a] - 0.5) ** 2 for a in range(p)) + sum((z[p + j] - 0.5 * ell) ** 2
                                                        for j in range(q))
    return quad_table(p, q, ne, ell, -Z / np.maximum(np.sqrt(r2), b))


def union_of_disks(ne, R=0.75, Z=1.0, b=1e-4, penalty=1.0e3):
    """The linear chain of §4.2 on the box (0, L) x (0, 2R): disks of radius R
    around the cell centres (i - 1/2, R) carry the truncated Coulomb potential
    -Z / max(r, b), the rest of the box the penalty a (the penalised potential
    of §4.2 that confines the eigenfunctions to the union of disks as a grows).
    Adjacent disks overlap for R > 1/2.  ell = 2R must be a multiple of h."""
    ell = 2.0 * R
    z = quad_points(1, 1, ne, ell)
    r = np.sqrt((z[0] - 0.5) ** 2 + (z[1] - R) ** 2)
    return quad_table(1, 1, ne, ell, np.where(r <= R, -Z / np.maximum(r, b), penalty))


def small_config(p, q, L, ne, delta, V, ell=1):
    return dict(name=f"p{p}q{q}-L{L}-ne{ne}-d{delta}", p=p, q=q, L=L, ell=ell, ne=ne,
                delta=delta, V=V)


def random_vector(n, seed):
    """A seeded standard-normal vector (test right-hand sides)."""
    return np.random.default_rng(seed).standard_normal(n)
