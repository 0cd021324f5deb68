"""Derivatives with respect to the parameters of the potential.

The paper does not differentiate; this module adds gradients on top of the
same solver.  Parameters theta = (a_1..a_T, phi_1..phi_T) of a SEP_FOURIER or
FOURIER2 potential (the seeded periodic families of the workloads).

A = K + M_V (§2, eq:discrete-weak-form) depends on theta only through V and
is linear in V, so dA/dtheta_j is the mass matrix weighted by dV/dtheta_j,
assembled with the same quadrature.  With that:

* ground-state eigenvalue (Hellmann-Feynman, x the eigenvector):
      dlambda/dtheta_j = x^T M_{dV_j} x / x^T M x;
* the shift sigma is the lowest eigenvalue of the cell problem
  (eq:cell-problem), so likewise
      dsigma/dtheta_j = psi^T M#_{dV_j} psi / psi^T M# psi;
* a shifted solve u = A_sigma^{-1} b with b independent of theta and an
  upstream gradient g = dl/du: A_sigma is symmetric, so the adjoint system
  A_sigma w = g is solved by the same PCG with the same two-level
  preconditioner, and
      dl/dtheta_j = -w^T (M_{dV_j} - dsigma/dtheta_j M) u,   dl/db = w.

Derivative potentials need no new kernel: dV/da_t is term t alone with unit
amplitude, and dV/dphi_t = -a_t sin(...) is term t with its phase advanced by
pi/2.  Every form x^T M_W y runs in ddeig_potential_form.
"""
import math

import numpy as np
import torch

from . import ddeig as _dd

PARAM_KINDS = ("sep_fourier", "fourier2")


def param_vector(spec):
    """theta = (a_1..a_T, phi_1..phi_T) of a SEP_FOURIER / FOURIER2 potential dict."""
    if spec["kind"] not in PARAM_KINDS:
        raise ValueError(f"potential kind {spec['kind']!r} has no Fourier parameters")
    return np.concatenate([np.asarray(spec["a"], float), np.asarray(spec["phi"], float)])


def with_params(spec, theta):
    """The potential dict with its amplitudes and phases replaced by theta."""
    theta = np.asarray(theta, dtype=np.float64).ravel()
    T = len(spec["a"])
    if theta.size != 2 * T:
        raise ValueError(f"theta has {theta.size} entries, expected {2 * T}")
    out = dict(spec)
    out["a"] = theta[:T].tolist()
    out["phi"] = theta[T:].tolist()
    return out


def dpotential(spec, j):
    """dV/dtheta_j as a one-term potential dict of the same kind."""
    T = len(spec["a"])
    t = j % T
    one = dict(spec)
    for key in ("k", "m"):
        if key in spec:
            one[key] = [spec[key][t]]
    if j < T:   # amplitude: the term itself with a = 1
        one["a"], one["phi"] = [1.0], [float(spec["phi"][t])]
    else:       # phase: -a sin(u) = a cos(u + pi/2)
        one["a"], one["phi"] = [float(spec["a"][t])], [float(spec["phi"][t]) + 0.5 * math.pi]
    return one


def _mass_spec():
    return {"kind": "const", "c": 1.0}


def forms(prob, spec, x, y, space="global"):
    """(x^T M_{dV_j} y for every parameter j, x^T M y)."""
    T = len(spec["a"])
    vals = np.array([_dd.potential_form(prob, dpotential(spec, j), x, y, space)
                     for j in range(2 * T)])
    return vals, _dd.potential_form(prob, _mass_spec(), x, y, space)


def eigenvalue_grad(prob, spec, x):
    """dlambda/dtheta for the ground state x (any scaling) of the problem."""
    vals, xmx = forms(prob, spec, x, x)
    return vals / xmx


def shift_grad(prob, spec, psi):
    """dsigma/dtheta from the cell eigenvector psi (n_cell values, cell order)."""
    if not isinstance(psi, torch.Tensor):
        psi = torch.as_tensor(np.ascontiguousarray(psi, dtype=np.float64), device="cuda")
    vals, pmp = forms(prob, spec, psi, psi, space="cell")
    return vals / pmp


def solve_grad(prob, spec, u, w, dsigma):
    """dl/dtheta = -(w^T M_{dV} u - dsigma w^T M u) for u = A_sigma^{-1} b, A_sigma w = dl/du."""
    vals, wmu = forms(prob, spec, w, u)
    return -(vals - np.asarray(dsigma) * wmu)


def _assemble(geom, spec, opts):
    prob = _dd.assemble(geom["p"], geom["q"], geom["L"], geom["ne"], spec, geom["delta"],
                        ell=geom.get("ell", 1), local_prec=opts.get("local_prec", "fp64"))
    _, psi = _dd.cell_shift(prob)
    return prob, psi


def _theta_in(theta):
    if not isinstance(theta, torch.Tensor) or theta.dim() != 1:
        raise TypeError("theta must be a 1-D tensor (a_1..a_T, phi_1..phi_T)")
    return theta.detach().to("cpu", torch.float64).numpy()


class EigenvalueFn(torch.autograd.Function):
    """lambda(theta): the smallest eigenvalue of K + M_V(theta) on the box of geom.

    geom: dict(p, q, L, ne, delta[, ell], V) with V the base potential dict
    (its kind, wave numbers and cy; theta supplies a and phi).  opts:
    local_prec, tol_x, rtol_inner, maxit_inner.  Forward: cell shift and the
    shifted inverse iteration; backward: Hellmann-Feynman forms on the
    converged eigenvector.  Returns a 0-d float64 tensor on theta's device.
    """

    @staticmethod
    def forward(ctx, theta, geom, opts=None):
        opts = opts or {}
        spec = with_params(geom["V"], _theta_in(theta))
        prob, _ = _assemble(geom, spec, opts)
        x = torch.zeros(prob.n_dof, dtype=torch.float64, device="cuda")
        out = _dd.inverse_iteration(prob, x, tol_x=opts.get("tol_x", 1e-11),
                                    maxit_outer=opts.get("maxit_outer", 200),
                                    rtol_inner=opts.get("rtol_inner", 1e-12),
                                    maxit_inner=opts.get("maxit_inner", 3000))
        ctx.prob, ctx.spec, ctx.x = prob, spec, x
        ctx.info = out
        return torch.tensor(out["lam"], dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, g):
        grad = eigenvalue_grad(ctx.prob, ctx.spec, ctx.x)
        gt = torch.as_tensor(grad, dtype=torch.float64, device=g.device)
        return g * gt, None, None


class ShiftedSolveFn(torch.autograd.Function):
    """u(theta, b) = A_sigma(theta)^{-1} b with sigma(theta) the cell shift.

    b is an n_dof CUDA float64 vector.  Forward: one PCG solve with the two-level
    preconditioner; backward: the adjoint PCG solve A_sigma w = dl/du (the same
    operator and preconditioner), then the potential forms for dl/dtheta and
    dl/db = w.  opts: local_prec, rtol, maxit.
    """

    @staticmethod
    def forward(ctx, theta, b, geom, opts=None):
        opts = opts or {}
        spec = with_params(geom["V"], _theta_in(theta))
        prob, psi = _assemble(geom, spec, opts)
        bb = b.detach().contiguous()
        u = torch.zeros_like(bb)
        rtol, maxit = opts.get("rtol", 1e-12), opts.get("maxit", 3000)
        _dd.pcg_solve(prob, bb, u, rtol=rtol, maxit=maxit)
        ctx.prob, ctx.spec, ctx.psi, ctx.u = prob, spec, psi, u
        ctx.rtol, ctx.maxit = rtol, maxit
        ctx.theta_device = theta.device
        return u.clone()

    @staticmethod
    def backward(ctx, gu):
        prob = ctx.prob
        g = gu.detach().to(torch.float64).contiguous()
        w = torch.zeros_like(g)
        _dd.pcg_solve(prob, g, w, rtol=ctx.rtol, maxit=ctx.maxit)
        ds = shift_grad(prob, ctx.spec, ctx.psi)
        grad = solve_grad(prob, ctx.spec, ctx.u, w, ds)
        gtheta = torch.as_tensor(grad, dtype=torch.float64, device=ctx.theta_device)
        return (gtheta if ctx.needs_input_grad[0] else None,
                w if ctx.needs_input_grad[1] else None, None, None)


def eigenvalues(thetas, geoms, opts=None):
    """lambda_j(theta_j) for independent instances (a list of EigenvalueFn applications)."""
    return torch.stack([EigenvalueFn.apply(t, g, opts) for t, g in zip(thetas, geoms)])
