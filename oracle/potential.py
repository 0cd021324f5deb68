"""Evaluation of the periodic potentials V used by the workloads.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Assumption (A1) of §1: V has period 1 in every expanding direction x_i;
(A2): V is bounded.  A potential is described by a plain dict ("spec"),
produced by the seeded input generators in ``workloads``:

  const        V = c
  sep_fourier  V = sum_t a_t cos(2 pi k_t x1 + phi_t) * (1 + cy * prod_j sin(pi y_j / ell))
  fourier2     V = sum_t a_t cos(2 pi (k_t x1 + m_t x2) + phi_t)          (p = 2)
  sin4         V = amp * prod_i sin^4(pi x_i) * prod_j sin^4(pi y_j / ell)   (§4.1)
  sep_sum      V = c0 + sum_t a_t sin(2 pi k_t z_{axis_t}) + sum_j g_j y_j (§4.3)

``vfun`` returns a vectorised V(coords) for the element assembly route;
``kron_terms`` returns the same V as a finite sum of products of 1-D
functions for the Kronecker route.  The two are written independently so
that the assembly-route test pins both.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def vfun(spec, p, q, ell=1):
    kind = spec["kind"]
    if kind == "const":
        c = float(spec["c"])
        return lambda z: np.full_like(z[0], c, dtype=np.float64)
    if kind == "sep_fourier":
        a = np.asarray(spec["a"], float); ph = np.asarray(spec["phi"], float)
        k = np.asarray(spec["k"], float); cy = float(spec["cy"])

        def f(z):
            x = z[0]
            F = np.zeros_like(x, dtype=np.float64)
            for t in range(a.size):
                F += a[t] * np.cos(TWO_PI * k[t] * x + ph[t])
            G = np.ones_like(x, dtype=np.float64)
            for j in range(q):
                G = G * np.sin(np.pi * z[p + j] / ell)
            return F * (1.0 + cy * G) if q > 0 else F * (1.0 + cy)
        return f
    if kind == "fourier2":
        a = np.asarray(spec["a"], float); ph = np.asarray(spec["phi"], float)
        k = np.asarray(spec["k"], float); m = np.asarray(spec["m"], float)

        def f(z):
            out = np.zeros_like(z[0], dtype=np.float64)
            for t in range(a.size):
                out += a[t] * np.cos(TWO_PI * (k[t] * z[0] + m[t] * z[1]) + ph[t])
            return out
        return f
    if kind == "sin4":
        amp = float(spec["amp"])

        def f(z):
            out = np.full_like(z[0], amp, dtype=np.float64)
            for i in range(p):
                out = out * np.sin(np.pi * z[i]) ** 4
            for j in range(q):
                out = out * np.sin(np.pi * z[p + j] / ell) ** 4
            return out
        return f
    if kind == "sep_sum":
        c0 = float(spec["c0"])
        terms = spec["terms"]
        g = list(spec.get("g", []))

        def f(z):
            out = np.full_like(z[0], c0, dtype=np.float64)
            for (amp, axis, kk) in terms:
                out = out + amp * np.sin(TWO_PI * kk * z[int(axis)])
            for j, gj in enumerate(g):
                out = out + gj * z[p + j]
            return out
        return f
    if kind == "quad_table":
        # V known only at the quadrature points of the period cell: a point's
        # element is floor(z / h) (x cell-local), its Gauss point along each axis
        # the lower or upper one of that element
        ne = int(spec["ne"])
        h = 1.0 / ne
        tab = np.asarray(spec["table"], dtype=np.float64)
        nel = [ne] * p + [int(round(ell * ne))] * q

        def f(z):
            d = p + q
            elem = np.zeros(np.shape(z[0]), dtype=np.int64)
            pt = np.zeros(np.shape(z[0]), dtype=np.int64)
            stride = 1
            for a in range(d):
                u = np.asarray(z[a]) / h
                e = np.floor(u).astype(np.int64)
                upper = (u - e) > 0.5
                elem += stride * e
                pt += upper.astype(np.int64) << a
                stride *= nel[a]
            return tab[elem * (1 << d) + pt]
        return f
    raise ValueError(f"unknown potential kind {kind!r}")


def kron_terms(spec, p, q, ell=1):
    """V as a list of (coef, [f_0..f_{d-1}]) products; None means the constant 1."""
    d = p + q
    kind = spec["kind"]
    none = [None] * d
    if kind == "const":
        return [(float(spec["c"]), list(none))]
    if kind == "sep_fourier":
        a = np.asarray(spec["a"], float); ph = np.asarray(spec["phi"], float)
        k = np.asarray(spec["k"], float); cy = float(spec["cy"])

        def F(x):
            s = np.zeros_like(x, dtype=np.float64)
            for t in range(a.size):
                s += a[t] * np.cos(TWO_PI * k[t] * x + ph[t])
            return s
        t1 = list(none); t1[0] = F
        if q == 0:
            return [(1.0 + cy, t1)]
        t2 = list(none); t2[0] = F
        for j in range(q):
            t2[p + j] = (lambda y: np.sin(np.pi * y / ell))
        return [(1.0, t1), (cy, t2)]
    if kind == "fourier2":
        out = []
        for amp, kk, mm, phi in zip(spec["a"], spec["k"], spec["m"], spec["phi"]):
            # cos(u + v) = cos u cos v - sin u sin v with u = 2 pi k x1, v = 2 pi m x2 + phi
            c1 = list(none); c1[0] = (lambda x, kk=kk: np.cos(TWO_PI * kk * x))
            c1[1] = (lambda x, mm=mm, phi=phi: np.cos(TWO_PI * mm * x + phi))
            s1 = list(none); s1[0] = (lambda x, kk=kk: np.sin(TWO_PI * kk * x))
            s1[1] = (lambda x, mm=mm, phi=phi: np.sin(TWO_PI * mm * x + phi))
            out.append((float(amp), c1))
            out.append((-float(amp), s1))
        return out
    if kind == "sin4":
        fs = [(lambda x: np.sin(np.pi * x) ** 4)] * p + \
             [(lambda y: np.sin(np.pi * y / ell) ** 4)] * q
        return [(float(spec["amp"]), fs)]
    if kind == "sep_sum":
        out = [(float(spec["c0"]), list(none))]
        for (amp, axis, kk) in spec["terms"]:
            t = list(none); t[int(axis)] = (lambda x, kk=kk: np.sin(TWO_PI * kk * x))
            out.append((float(amp), t))
        for j, gj in enumerate(spec.get("g", [])):
            t = list(none); t[p + j] = (lambda y: y)
            out.append((float(gj), t))
        return out
    raise ValueError(f"unknown potential kind {kind!r}")
