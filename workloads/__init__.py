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


def small_config(p, q, L, ne, delta, V, ell=1):
    return dict(name=f"p{p}q{q}-L{L}-ne{ne}-d{delta}", p=p, q=q, L=L, ell=ell, ne=ne,
                delta=delta, V=V)


def random_vector(n, seed):
    """A seeded standard-normal vector (test right-hand sides)."""
    return np.random.default_rng(seed).standard_normal(n)
