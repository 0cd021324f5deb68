"""Thin ctypes binding of libddeig (include/ddeig.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Vectors are torch float64 tensors on the GPU (contiguous); the library works
on the torch stream that is current when ``assemble`` is called.  There is no
CPU fallback: a missing library raises at import of the first call.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddeig.so")

DDEIG_OK = 0
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTSPD", -5: "ENOCONV",
          -6: "ESTATE", -7: "EINTERNAL"}
V_KINDS = {"const": 0, "sep_fourier": 1, "fourier2": 2, "sin4": 3, "sep_sum": 4,
           "quad_table": 5}
OPS = {"A_sigma": 0, "A": 1, "M": 2, "K": 3}
MAX_TERMS = 64


class DdeigError(RuntimeError):
    def __init__(self, status, func, msg):
        self.status = status
        self.code = STATUS.get(status, str(status))
        super().__init__(f"{func}: {self.code}: {msg}")


class Geometry(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("q", ctypes.c_int), ("L", ctypes.c_int),
                ("ell", ctypes.c_double)]


class Potential(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nterms", ctypes.c_int),
                ("a", ctypes.POINTER(ctypes.c_double)), ("phi", ctypes.POINTER(ctypes.c_double)),
                ("k", ctypes.POINTER(ctypes.c_int)), ("m", ctypes.POINTER(ctypes.c_int)),
                ("cy", ctypes.c_double), ("c0", ctypes.c_double),
                ("g", ctypes.POINTER(ctypes.c_double)),
                ("table", ctypes.POINTER(ctypes.c_double)), ("table_len", ctypes.c_long)]


class Options(ctypes.Structure):
    _fields_ = [("pu", ctypes.c_int), ("coarse", ctypes.c_int), ("local_prec", ctypes.c_int),
                ("batch_iters", ctypes.c_int), ("graphs", ctypes.c_int), ("sweep", ctypes.c_int)]


class PcgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("relres", ctypes.c_double), ("breakdown", ctypes.c_int),
                ("hist", ctypes.POINTER(ctypes.c_double)), ("hist_cap", ctypes.c_int),
                ("true_relres", ctypes.c_double), ("fallback", ctypes.c_int)]


class EigInfo(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("dx_M", ctypes.c_double),
                ("outer_its", ctypes.c_int), ("inner_sum", ctypes.c_long),
                ("inner_max", ctypes.c_int), ("t_solve_ms", ctypes.c_double),
                ("spec_res", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("inner_unconverged", ctypes.c_int), ("fallback", ctypes.c_int)]


class LopcgInfo(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("res_norm", ctypes.c_double),
                ("outer_its", ctypes.c_int), ("inner_sum", ctypes.c_long),
                ("inner_max", ctypes.c_int), ("t_solve_ms", ctypes.c_double)]


EXPORTS = ["ddeig_assemble", "ddeig_cell_shift", "ddeig_set_shift", "ddeig_apply_op", "ddeig_debug_force_breakdown",
           "ddeig_apply_precond", "ddeig_apply_schwarz", "ddeig_stationary_ras",
           "ddeig_gmres_solve", "ddeig_pcg_solve", "ddeig_inverse_iteration", "ddeig_lopcg",
           "ddeig_profile_kernel", "ddeig_profile_iteration", "ddeig_potential_form",
           "ddeig_potential_form_noalloc", "ddeig_eig_grad", "ddeig_shift_grad",
           "ddeig_solve_grad", "ddeig_batch_eig_grad", "ddeig_batch_solve_grad", "ddeig_batch_create",
           "ddeig_batch_query", "ddeig_batch_tuning", "ddeig_batch_pcg_solve", "ddeig_batch_inverse_iteration",
           "ddeig_batch_destroy", "ddeig_query", "ddeig_destroy", "ddeig_status_string",
           "ddeig_last_error"]

_lib = None


def load_library(path=LIB_PATH):
    """Loads libddeig.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2311_08757_amd.build_lib.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.ddeig_assemble.argtypes = [ctypes.POINTER(Geometry), ctypes.c_double,
                                   ctypes.POINTER(Potential), ctypes.c_int,
                                   ctypes.POINTER(Options), P, ctypes.POINTER(P)]
    lib.ddeig_cell_shift.argtypes = [P, dp, dp]
    lib.ddeig_set_shift.argtypes = [P, ctypes.c_double, dp]
    lib.ddeig_debug_force_breakdown.argtypes = [P, ctypes.c_int]
    lib.ddeig_apply_op.argtypes = [P, ctypes.c_int, P, P]
    lib.ddeig_apply_precond.argtypes = [P, P, P]
    lib.ddeig_apply_schwarz.argtypes = [P, ctypes.c_int, P, P]
    lib.ddeig_stationary_ras.argtypes = [P, ctypes.c_int, P, P, ctypes.c_double, ctypes.c_int,
                                         ctypes.POINTER(PcgInfo)]
    lib.ddeig_gmres_solve.argtypes = [P, ctypes.c_int, P, P, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(PcgInfo)]
    lib.ddeig_pcg_solve.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(PcgInfo)]
    lib.ddeig_inverse_iteration.argtypes = [P, P, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_int, ctypes.POINTER(EigInfo)]
    lib.ddeig_lopcg.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                ctypes.POINTER(LopcgInfo)]
    lib.ddeig_profile_kernel.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, dp, dp]
    lib.ddeig_profile_iteration.argtypes = [P, P, ctypes.c_int, dp]
    lib.ddeig_potential_form.argtypes = [P, ctypes.c_int, ctypes.POINTER(Potential), P, P, dp]
    lib.ddeig_potential_form_noalloc.argtypes = [P, ctypes.c_int, ctypes.POINTER(Potential), P, P,
                                                 dp]
    lib.ddeig_eig_grad.argtypes = [P, P, dp, ctypes.c_int]
    lib.ddeig_shift_grad.argtypes = [P, dp, ctypes.c_int]
    lib.ddeig_solve_grad.argtypes = [P, P, P, dp, ctypes.c_int]
    lib.ddeig_batch_eig_grad.argtypes = [P, PP, dp, ctypes.c_int]
    lib.ddeig_batch_solve_grad.argtypes = [P, PP, PP, dp, ctypes.c_int]
    lib.ddeig_batch_create.argtypes = [PP, ctypes.c_int, ctypes.c_int, PP]
    lib.ddeig_batch_query.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int), dp]
    lib.ddeig_batch_tuning.argtypes = [P, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_double)]
    lib.ddeig_batch_pcg_solve.argtypes = [P, PP, PP, ctypes.c_double, ctypes.c_int,
                                          ctypes.POINTER(PcgInfo)]
    lib.ddeig_batch_inverse_iteration.argtypes = [P, PP, ctypes.c_double, ctypes.c_int,
                                                  ctypes.c_double, ctypes.c_int,
                                                  ctypes.POINTER(EigInfo)]
    lib.ddeig_batch_destroy.argtypes = [P]
    lib.ddeig_batch_destroy.restype = None
    lib.ddeig_query.argtypes = [P, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long),
                                ctypes.POINTER(ctypes.c_int)]
    lib.ddeig_destroy.argtypes = [P]
    lib.ddeig_destroy.restype = None
    lib.ddeig_status_string.argtypes = [ctypes.c_int]
    lib.ddeig_status_string.restype = ctypes.c_char_p
    lib.ddeig_last_error.argtypes = []
    lib.ddeig_last_error.restype = ctypes.c_char_p
    for f in EXPORTS:
        if f not in ("ddeig_destroy", "ddeig_batch_destroy", "ddeig_status_string",
                     "ddeig_last_error"):
            getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status, func):
    if status != DDEIG_OK:
        msg = load_library().ddeig_last_error().decode()
        raise DdeigError(status, func, msg)


def _ptr(t, n=None, name="vector"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """Owns a ddeig_problem handle (destroyed with the object)."""

    def __init__(self, handle, n_dof, n_cell, n_sub, stream):
        self.handle = handle
        self.n_dof, self.n_cell, self.n_sub = n_dof, n_cell, n_sub
        self.stream = stream
        self.sigma = None
        self.nterms = 0

    def __del__(self):
        h = getattr(self, "handle", None)
        self.handle = None
        if h and _lib is not None:
            try:
                _lib.ddeig_destroy(h)
            except Exception:  # interpreter shutdown
                pass


def _potential(spec):
    kind = spec["kind"]
    keep = []

    def darr(x):
        a = (ctypes.c_double * max(len(x), 1))(*[float(v) for v in x])
        keep.append(a)
        return ctypes.cast(a, ctypes.POINTER(ctypes.c_double))

    def iarr(x):
        a = (ctypes.c_int * max(len(x), 1))(*[int(v) for v in x])
        keep.append(a)
        return ctypes.cast(a, ctypes.POINTER(ctypes.c_int))

    V = Potential()
    V.kind = V_KINDS[kind]
    V.nterms = 0
    V.cy = 0.0
    V.c0 = 0.0
    if kind == "const":
        V.c0 = float(spec["c"])
    elif kind == "sep_fourier":
        V.nterms = len(spec["a"])
        V.a, V.phi, V.k = darr(spec["a"]), darr(spec["phi"]), iarr(spec["k"])
        V.cy = float(spec["cy"])
    elif kind == "fourier2":
        V.nterms = len(spec["a"])
        V.a, V.phi = darr(spec["a"]), darr(spec["phi"])
        V.k, V.m = iarr(spec["k"]), iarr(spec["m"])
    elif kind == "sin4":
        V.c0 = float(spec["amp"])
    elif kind == "sep_sum":
        terms = spec["terms"]
        V.nterms = len(terms)
        V.a = darr([t[0] for t in terms])
        V.m = iarr([t[1] for t in terms])
        V.k = iarr([t[2] for t in terms])
        V.c0 = float(spec["c0"])
        V.g = darr(spec.get("g", []))
    elif kind == "quad_table":
        tab = np.ascontiguousarray(spec["table"], dtype=np.float64)
        keep.append(tab)
        V.table = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        V.table_len = tab.size
    else:
        raise ValueError(kind)
    return V, keep


def assemble(p, q, L, ne, V, delta, ell=1, pu="equal", coarse=True, local_prec="fp64",
             batch_iters=8, graphs=False, stream=None, sweep="auto"):
    """ddeig_assemble: geometry (0,L)^p x (0,ell)^q, h = 1/ne, potential dict V;
    sweep: the A_sigma sweep ("auto", "tiles" or "march")."""
    import torch
    lib = load_library()
    geom = Geometry(p, q, L, float(ell))
    Vs, keep = _potential(V)
    opts = Options({"equal": 0, "distance": 1}[pu], 1 if coarse else 0,
                   {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16": 3}[local_prec], batch_iters,
                   1 if graphs else 0, {"auto": 0, "tiles": 1, "march": 2}[sweep])
    if stream is None:
        stream = torch.cuda.current_stream()
    handle = ctypes.c_void_p()
    st = lib.ddeig_assemble(ctypes.byref(geom), 1.0 / ne, ctypes.byref(Vs), delta,
                            ctypes.byref(opts), ctypes.c_void_p(stream.cuda_stream),
                            ctypes.byref(handle))
    del keep
    _check(st, "ddeig_assemble")
    n_dof, n_cell, n_sub = query_handle(handle)
    prob = Problem(handle, n_dof, n_cell, n_sub, stream)
    # Fourier terms of the potential (the parameters of the derivative calls)
    prob.nterms = len(V["a"]) if V["kind"] in ("sep_fourier", "fourier2") else 0
    return prob


def query_handle(handle):
    lib = load_library()
    nd, nc, ns = ctypes.c_long(), ctypes.c_long(), ctypes.c_int()
    _check(lib.ddeig_query(handle, ctypes.byref(nd), ctypes.byref(nc), ctypes.byref(ns)),
           "ddeig_query")
    return nd.value, nc.value, ns.value


def query(prob):
    return query_handle(prob.handle)


def cell_shift(prob):
    """ddeig_cell_shift: returns (sigma, psi as a numpy array of n_cell values)."""
    lib = load_library()
    sig = ctypes.c_double()
    psi = np.zeros(prob.n_cell)
    _check(lib.ddeig_cell_shift(prob.handle, ctypes.byref(sig),
                                psi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "ddeig_cell_shift")
    prob.sigma = sig.value
    return sig.value, psi


def set_shift(prob, sigma, psi=None):
    lib = load_library()
    ptr = None
    if psi is not None:
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        if psi.size != prob.n_cell:
            raise ValueError("psi must have n_cell entries")
        ptr = psi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib.ddeig_set_shift(prob.handle, float(sigma), ptr), "ddeig_set_shift")
    prob.sigma = float(sigma)


def debug_force_breakdown(prob, count=1):
    """ddeig_debug_force_breakdown: the next `count` reduced-precision PCG solves report r.z <= 0."""
    _check(load_library().ddeig_debug_force_breakdown(prob.handle, int(count)),
           "ddeig_debug_force_breakdown")


def apply_op(prob, which, x, y):
    """ddeig_apply_op: y = Op x, which in {"A_sigma", "A", "M", "K"} or 0..3."""
    w = OPS[which] if isinstance(which, str) else int(which)
    _check(load_library().ddeig_apply_op(prob.handle, w, _ptr(x, prob.n_dof, "x"),
                                         _ptr(y, prob.n_dof, "y")), "ddeig_apply_op")


def apply_precond(prob, r, z):
    _check(load_library().ddeig_apply_precond(prob.handle, _ptr(r, prob.n_dof, "r"),
                                              _ptr(z, prob.n_dof, "z")), "ddeig_apply_precond")


def _krylov(fn, name, prob, lead, b, x, tail, hist_cap, raise_on_error):
    info = PcgInfo()
    hist = np.zeros(max(hist_cap, 1))
    info.hist = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if hist_cap > 0 else None
    info.hist_cap = hist_cap
    st = fn(prob.handle, *lead, _ptr(b, prob.n_dof, "b"), _ptr(x, prob.n_dof, "x"), *tail,
            ctypes.byref(info))
    out = dict(status=STATUS.get(st, st), iters=info.iters, relres=info.relres,
               true_relres=info.true_relres, breakdown=info.breakdown, fallback=info.fallback,
               hist=hist[:min(hist_cap, info.iters + 1)] if hist_cap > 0 else None)
    if raise_on_error and st != DDEIG_OK:
        _check(st, name)
    return out


def pcg_solve(prob, b, x, rtol=1e-10, maxit=1000, hist_cap=0, raise_on_error=True):
    """ddeig_pcg_solve; returns dict(status, iters, relres, breakdown, hist)."""
    lib = load_library()
    return _krylov(lib.ddeig_pcg_solve, "ddeig_pcg_solve", prob, (), b, x,
                   (float(rtol), int(maxit)), hist_cap, raise_on_error)


PREC_KINDS = {"as1": 0, "as2": 1, "ras1": 2, "ras2": 3, "coarse": 4}


def _prec_kind(kind):
    return PREC_KINDS[kind] if isinstance(kind, str) else int(kind)


def apply_schwarz(prob, kind, r, z):
    """ddeig_apply_schwarz: z = M^{-1} r for kind 'as1', 'as2', 'ras1', 'ras2' or 'coarse'."""
    _check(load_library().ddeig_apply_schwarz(prob.handle, _prec_kind(kind),
                                              _ptr(r, prob.n_dof, "r"), _ptr(z, prob.n_dof, "z")),
           "ddeig_apply_schwarz")


def stationary_ras(prob, b, x, levels=2, rtol=1e-10, maxit=10000, hist_cap=0,
                   raise_on_error=True):
    """ddeig_stationary_ras; returns dict(status, iters, relres, breakdown, hist)."""
    lib = load_library()
    return _krylov(lib.ddeig_stationary_ras, "ddeig_stationary_ras", prob, (int(levels),), b, x,
                   (float(rtol), int(maxit)), hist_cap, raise_on_error)


def gmres_solve(prob, b, x, kind="ras2", rtol=1e-10, maxit=1000, restart=0, hist_cap=0,
                raise_on_error=True):
    """ddeig_gmres_solve (right-preconditioned); returns dict(status, iters, relres, breakdown, hist)."""
    lib = load_library()
    return _krylov(lib.ddeig_gmres_solve, "ddeig_gmres_solve", prob, (_prec_kind(kind),), b, x,
                   (float(rtol), int(maxit), int(restart)), hist_cap, raise_on_error)


def inverse_iteration(prob, x, tol_x=1e-9, maxit_outer=100, rtol_inner=1e-10, maxit_inner=1000,
                      raise_on_error=True):
    """ddeig_inverse_iteration; x (in: start or zeros, out: eigenvector)."""
    lib = load_library()
    info = EigInfo()
    st = lib.ddeig_inverse_iteration(prob.handle, _ptr(x, prob.n_dof, "x"), float(tol_x),
                                     int(maxit_outer), float(rtol_inner), int(maxit_inner),
                                     ctypes.byref(info))
    out = dict(status=STATUS.get(st, st), lam=info.lambda_, dx_M=info.dx_M,
               outer_its=info.outer_its, inner_sum=info.inner_sum, inner_max=info.inner_max,
               t_solve_ms=info.t_solve_ms, spec_res=info.spec_res, t_setup_ms=info.t_setup_ms,
               inner_unconverged=info.inner_unconverged, fallback=info.fallback)
    if raise_on_error and st != DDEIG_OK:
        _check(st, "ddeig_inverse_iteration")
    return out


def status_string(code):
    return load_library().ddeig_status_string(int(code)).decode()


def profile_kernel(prob, which, reps=20, x=None, y=None):
    """ddeig_profile_kernel: mean launch time (us) of one hot kernel and its algorithmic work."""
    lib = load_library()
    avg = ctypes.c_double()
    work = ctypes.c_double()
    xp = _ptr(x, prob.n_dof, "x") if x is not None else None
    yp = _ptr(y, prob.n_dof, "y") if y is not None else None
    names = {"stencil": 0, "local": 1, "precond": 2, "restrict": 3, "extend": 4, "correct": 5}
    w = names[which] if isinstance(which, str) else int(which)
    _check(lib.ddeig_profile_kernel(prob.handle, w, int(reps), xp, yp, ctypes.byref(avg),
                                    ctypes.byref(work)), "ddeig_profile_kernel")
    return avg.value, work.value


ITERATION_PARTS = ("stencil_dir", "restrict_xr", "local_solves", "correction", "extend_check")


def profile_iteration(prob, b, reps=30):
    """ddeig_profile_iteration: mean time (us) of each part of one PCG iteration."""
    lib = load_library()
    us = (ctypes.c_double * len(ITERATION_PARTS))()
    _check(lib.ddeig_profile_iteration(prob.handle, _ptr(b, prob.n_dof, "b"), int(reps), us),
           "ddeig_profile_iteration")
    return dict(zip(ITERATION_PARTS, list(us)))


def potential_form(prob, W, x, y, space="global"):
    """ddeig_potential_form: x^T M_W y for a potential dict W.

    space "global": x, y are n_dof CUDA float64 vectors; "cell": n_cell vectors
    of the periodic cell (the layout of cell_shift's psi).
    """
    lib = load_library()
    sp = {"global": 0, "cell": 1}[space] if isinstance(space, str) else int(space)
    n = prob.n_cell if sp == 1 else prob.n_dof
    Ws, keep = _potential(W)
    out = ctypes.c_double()
    st = lib.ddeig_potential_form(prob.handle, sp, ctypes.byref(Ws), _ptr(x, n, "x"),
                                  _ptr(y, n, "y"), ctypes.byref(out))
    del keep
    _check(st, "ddeig_potential_form")
    return out.value


def potential_form_noalloc(prob, W, x, y, space="global"):
    """ddeig_potential_form_noalloc: x^T M_W y like potential_form, without device allocation."""
    lib = load_library()
    sp = {"global": 0, "cell": 1}[space] if isinstance(space, str) else int(space)
    n = prob.n_cell if sp == 1 else prob.n_dof
    Ws, keep = _potential(W)
    out = ctypes.c_double()
    st = lib.ddeig_potential_form_noalloc(prob.handle, sp, ctypes.byref(Ws), _ptr(x, n, "x"),
                                          _ptr(y, n, "y"), ctypes.byref(out))
    del keep
    _check(st, "ddeig_potential_form_noalloc")
    return out.value


def _nparams(prob):
    return 2 * int(prob.nterms)


def eig_grad(prob, x):
    """ddeig_eig_grad: dlambda/dtheta (numpy, 2T values) for the eigenvector x."""
    n = _nparams(prob)
    g = (ctypes.c_double * n)()
    _check(load_library().ddeig_eig_grad(prob.handle, _ptr(x, prob.n_dof, "x"), g, n),
           "ddeig_eig_grad")
    return np.array(g[:], dtype=np.float64)


def shift_grad(prob):
    """ddeig_shift_grad: dsigma/dtheta (numpy, 2T values)."""
    n = _nparams(prob)
    g = (ctypes.c_double * n)()
    _check(load_library().ddeig_shift_grad(prob.handle, g, n), "ddeig_shift_grad")
    return np.array(g[:], dtype=np.float64)


def solve_grad(prob, u, w):
    """ddeig_solve_grad: dl/dtheta for u = A_sigma^{-1} b and the adjoint solution w."""
    n = _nparams(prob)
    g = (ctypes.c_double * n)()
    _check(load_library().ddeig_solve_grad(prob.handle, _ptr(u, prob.n_dof, "u"),
                                           _ptr(w, prob.n_dof, "w"), g, n), "ddeig_solve_grad")
    return np.array(g[:], dtype=np.float64)


class Batch:
    """Owns a ddeig_batch handle; keeps its problems alive while it exists."""

    def __init__(self, handle, probs):
        self.handle = handle
        self.probs = list(probs)

    def __len__(self):
        return len(self.probs)

    def __del__(self):
        h = getattr(self, "handle", None)
        self.handle = None
        if h and _lib is not None:
            try:
                _lib.ddeig_batch_destroy(h)
            except Exception:  # interpreter shutdown
                pass


def _ptr_array(ts, ns, name):
    arr = (ctypes.c_void_p * len(ts))()
    for j, (t, n) in enumerate(zip(ts, ns)):
        arr[j] = _ptr(t, n, f"{name}[{j}]").value
    return arr


def batch_create(probs, graphs=True, reproducible=False, tile64=False):
    """ddeig_batch_create over a list of Problems (runs the GEMM autotuner, or
    reuses its choice for the same shapes); graphs: replay the grouped
    iterations from captured HIP graphs; reproducible: no timing, the
    single-problem K split (DDEIG_BATCH_REPRODUCIBLE); tile64 (with
    reproducible): 64-row GEMM tiles (DDEIG_BATCH_TILE64)."""
    lib = load_library()
    arr = (ctypes.c_void_p * len(probs))(*[p.handle.value if isinstance(p.handle, ctypes.c_void_p)
                                           else p.handle for p in probs])
    h = ctypes.c_void_p()
    flags = (1 if graphs else 0) | (2 if reproducible else 0) | (4 if tile64 else 0)
    _check(lib.ddeig_batch_create(arr, len(probs), flags, ctypes.byref(h)),
           "ddeig_batch_create")
    return Batch(h, probs)


def batch_query(batch):
    """ddeig_batch_query + ddeig_batch_tuning: the autotuner's K split, order,
    tile rows, tile count, the six 128-row timings and all twelve."""
    lib = load_library()
    ks, order, nt, tr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    tune = (ctypes.c_double * 6)()
    tune12 = (ctypes.c_double * 12)()
    _check(lib.ddeig_batch_query(batch.handle, ctypes.byref(ks), ctypes.byref(order),
                                 ctypes.byref(nt), tune), "ddeig_batch_query")
    _check(lib.ddeig_batch_tuning(batch.handle, ctypes.byref(tr), tune12), "ddeig_batch_tuning")
    return dict(ksplit=ks.value, order=order.value, tile_rows=tr.value, ntiles=nt.value,
                tune_us=list(tune), tune_us_all=list(tune12))


def batch_pcg_solve(batch, bs, xs, rtol=1e-10, maxit=1000, raise_on_error=True):
    """ddeig_batch_pcg_solve; returns (status, [dict(iters, relres, breakdown)])."""
    lib = load_library()
    ns = [p.n_dof for p in batch.probs]
    info = (PcgInfo * len(ns))()
    st = lib.ddeig_batch_pcg_solve(batch.handle, _ptr_array(bs, ns, "b"), _ptr_array(xs, ns, "x"),
                                   float(rtol), int(maxit), info)
    if raise_on_error and st != DDEIG_OK:
        _check(st, "ddeig_batch_pcg_solve")
    return STATUS.get(st, st), [dict(iters=i.iters, relres=i.relres, breakdown=i.breakdown,
                                     true_relres=i.true_relres) for i in info]


def batch_inverse_iteration(batch, xs, tol_x=1e-9, maxit_outer=100, rtol_inner=1e-10,
                            maxit_inner=1000, raise_on_error=True):
    """ddeig_batch_inverse_iteration; returns (status, [dict per instance])."""
    lib = load_library()
    ns = [p.n_dof for p in batch.probs]
    info = (EigInfo * len(ns))()
    st = lib.ddeig_batch_inverse_iteration(batch.handle, _ptr_array(xs, ns, "x"), float(tol_x),
                                           int(maxit_outer), float(rtol_inner), int(maxit_inner),
                                           info)
    if raise_on_error and st != DDEIG_OK:
        _check(st, "ddeig_batch_inverse_iteration")
    return STATUS.get(st, st), [dict(lam=i.lambda_, dx_M=i.dx_M, outer_its=i.outer_its,
                                     inner_sum=i.inner_sum, inner_max=i.inner_max,
                                     t_solve_ms=i.t_solve_ms, spec_res=i.spec_res,
                                     t_setup_ms=i.t_setup_ms,
                                     inner_unconverged=i.inner_unconverged) for i in info]


def batch_eig_grad(batch, xs):
    """ddeig_batch_eig_grad: (n, 2T) numpy array of dlambda_j/dtheta_j."""
    ns = [p.n_dof for p in batch.probs]
    npar = _nparams(batch.probs[0])
    g = (ctypes.c_double * (npar * len(ns)))()
    _check(load_library().ddeig_batch_eig_grad(batch.handle, _ptr_array(xs, ns, "x"), g, npar),
           "ddeig_batch_eig_grad")
    return np.array(g[:], dtype=np.float64).reshape(len(ns), npar)


def batch_solve_grad(batch, us, ws):
    """ddeig_batch_solve_grad: (n, 2T) numpy array of dl/dtheta_j."""
    ns = [p.n_dof for p in batch.probs]
    npar = _nparams(batch.probs[0])
    g = (ctypes.c_double * (npar * len(ns)))()
    _check(load_library().ddeig_batch_solve_grad(batch.handle, _ptr_array(us, ns, "u"),
                                                 _ptr_array(ws, ns, "w"), g, npar),
           "ddeig_batch_solve_grad")
    return np.array(g[:], dtype=np.float64).reshape(len(ns), npar)


LOPCG_MODES = {"fixed": 0, "adaptive": 1, "fused": 2}


LOPCG_INNER = {"cg": 0, "cg+asm2": 0, "gmres": 1, "gmres+ras2": 1, "ras2": 2, "ras1": 3}


def lopcg(prob, x, x_prev=None, tol_o=1e-8, maxit_outer=500, mode="fixed", rtol_inner=1e-8,
          maxit_inner=10000, inner="cg", raise_on_error=True):
    """ddeig_lopcg: inexact SI-preconditioned LOPCG; x in: start (zeros: constant), out:
    eigenvector; x_prev: x_0 (None: first unit vector).  mode: fixed / adaptive / fused;
    inner: cg (CG+ASM2), gmres (GMRES+RAS2), ras2, ras1 (stationary); with fused, cg
    applies M_AS,2 and gmres M_RAS,2."""
    lib = load_library()
    info = LopcgInfo()
    m = LOPCG_MODES[mode] if isinstance(mode, str) else int(mode)
    inn = LOPCG_INNER[inner] if isinstance(inner, str) else int(inner)
    xp = _ptr(x_prev, prob.n_dof, "x_prev") if x_prev is not None else None
    st = lib.ddeig_lopcg(prob.handle, _ptr(x, prob.n_dof, "x"), xp, float(tol_o), int(maxit_outer),
                         m, inn, float(rtol_inner), int(maxit_inner), ctypes.byref(info))
    out = dict(status=STATUS.get(st, st), lam=info.lambda_, res_norm=info.res_norm,
               outer_its=info.outer_its, inner_sum=info.inner_sum, inner_max=info.inner_max,
               t_solve_ms=info.t_solve_ms)
    if raise_on_error and st != DDEIG_OK:
        _check(st, "ddeig_lopcg")
    return out
