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

All 2T derivative forms (and the mass form) of a vector pair come from one
element-walking kernel of the library (ddeig_eig_grad, ddeig_shift_grad,
ddeig_solve_grad, and their batch versions over all instances of a batch in
one grouped launch); this module only calls them.  dpotential() gives dV/dtheta
as a potential dict (term t with unit amplitude, or with its phase advanced by
pi/2) for ddeig_potential_form.
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


def eigenvalue_grad(prob, spec, x):
    """dlambda/dtheta for the ground state x (any scaling) of the problem
    (ddeig_eig_grad; spec must be the problem's own potential)."""
    return _dd.eig_grad(prob, x)


def shift_grad(prob, spec, psi=None):
    """dsigma/dtheta from the problem's cell eigenvector (ddeig_shift_grad)."""
    return _dd.shift_grad(prob)


def solve_grad(prob, spec, u, w, dsigma=None):
    """dl/dtheta = -(w^T M_{dV} u - dsigma w^T M u) for u = A_sigma^{-1} b,
    A_sigma w = dl/du (ddeig_solve_grad, which forms dsigma itself)."""
    return _dd.solve_grad(prob, u, w)


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
        grad = _dd.eig_grad(ctx.prob, ctx.x)
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
        grad = _dd.solve_grad(prob, ctx.u, w)
        gtheta = torch.as_tensor(grad, dtype=torch.float64, device=ctx.theta_device)
        return (gtheta if ctx.needs_input_grad[0] else None,
                w if ctx.needs_input_grad[1] else None, None, None)


def _batch_problems(thetas, geoms, opts):
    specs = [with_params(g["V"], t) for g, t in zip(geoms, thetas)]
    probs = [_assemble(g, sp, opts)[0] for g, sp in zip(geoms, specs)]
    batch = _dd.batch_create(probs, graphs=opts.get("graphs", True))
    return specs, probs, batch


class BatchEigenvaluesFn(torch.autograd.Function):
    """lambda_j(theta_j) for independent instances solved as one batch.

    thetas: (n, 2T) tensor, row j the parameters of instance j; geoms: list of
    n geometry dicts (as for EigenvalueFn; 2-D with dense local solves, as the
    batch requires).  Forward: every instance's cell shift and set-up, then
    ddeig_batch_inverse_iteration with grouped launches; backward: the
    Hellmann-Feynman forms of all instances in one grouped launch
    (ddeig_batch_eig_grad).  opts: local_prec (default bf16), tol_x,
    rtol_inner, maxit_inner, maxit_outer, graphs.  Returns an (n,) tensor.
    """

    @staticmethod
    def forward(ctx, thetas, geoms, opts=None):
        opts = dict(opts or {})
        opts.setdefault("local_prec", "bf16")
        th = thetas.detach().to("cpu", torch.float64).numpy()
        if th.ndim != 2 or th.shape[0] != len(geoms):
            raise ValueError("thetas must be (n instances, 2T)")
        specs, probs, batch = _batch_problems(th, geoms, opts)
        xs = [torch.zeros(p.n_dof, dtype=torch.float64, device="cuda") for p in probs]
        _, info = _dd.batch_inverse_iteration(batch, xs, tol_x=opts.get("tol_x", 1e-11),
                                              maxit_outer=opts.get("maxit_outer", 200),
                                              rtol_inner=opts.get("rtol_inner", 1e-12),
                                              maxit_inner=opts.get("maxit_inner", 3000))
        ctx.batch, ctx.xs = batch, xs
        ctx.info = info
        return torch.tensor([f["lam"] for f in info], dtype=torch.float64, device=thetas.device)

    @staticmethod
    def backward(ctx, g):
        grad = _dd.batch_eig_grad(ctx.batch, ctx.xs)
        gt = torch.as_tensor(grad, dtype=torch.float64, device=g.device)
        return g[:, None] * gt, None, None


class BatchShiftedSolveFn(torch.autograd.Function):
    """u_j = A_sigma,j(theta_j)^{-1} b_j for independent instances solved as one batch.

    thetas: (n, 2T) tensor; bs: list of n CUDA float64 vectors; geoms as for
    BatchEigenvaluesFn.  Forward: ddeig_batch_pcg_solve; backward: the adjoint
    batch solve A_sigma,j w_j = dl/du_j with the same operators and
    preconditioners, then ddeig_batch_solve_grad (one grouped launch, the
    shifts moving with theta).  Returns the list of solutions as one
    concatenated tensor (instance-major) so that autograd sees one output;
    dl/db_j = w_j.  opts: local_prec (default bf16), rtol, maxit.
    """

    @staticmethod
    def forward(ctx, thetas, geoms, opts, *bs):
        opts = dict(opts or {})
        opts.setdefault("local_prec", "bf16")
        th = thetas.detach().to("cpu", torch.float64).numpy()
        specs, probs, batch = _batch_problems(th, geoms, opts)
        bb = [b.detach().contiguous() for b in bs]
        us = [torch.zeros_like(b) for b in bb]
        rtol, maxit = opts.get("rtol", 1e-12), opts.get("maxit", 3000)
        _dd.batch_pcg_solve(batch, bb, us, rtol=rtol, maxit=maxit)
        ctx.batch, ctx.us, ctx.rtol, ctx.maxit = batch, us, rtol, maxit
        ctx.sizes = [u.numel() for u in us]
        ctx.theta_device = thetas.device
        return torch.cat(us)

    @staticmethod
    def backward(ctx, gu):
        gs = [g.detach().to(torch.float64).contiguous()
              for g in torch.split(gu, ctx.sizes)]
        ws = [torch.zeros_like(g) for g in gs]
        _dd.batch_pcg_solve(ctx.batch, gs, ws, rtol=ctx.rtol, maxit=ctx.maxit)
        grad = _dd.batch_solve_grad(ctx.batch, ctx.us, ws)
        gtheta = torch.as_tensor(grad, dtype=torch.float64, device=ctx.theta_device)
        return (gtheta, None, None) + tuple(ws)


def eigenvalues(thetas, geoms, opts=None):
    """lambda_j(theta_j) for independent instances as one batch (BatchEigenvaluesFn)."""
    if not isinstance(thetas, torch.Tensor):
        thetas = torch.stack(list(thetas))
    return BatchEigenvaluesFn.apply(thetas, geoms, opts)
