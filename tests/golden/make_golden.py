"""Writes the stored oracle results for the full-size configurations.

Calls only the oracle (plain FP64 CPU): for each configuration the shift
sigma (cell problem), the smallest eigenpair by sigma-shifted inverse
iteration with exact solves to ||x_{k+1} - x_k||_M <= 1e-13, the second
eigenvalue (for the contraction rate), and the eigenvector at seeded sample
nodes.  "batch" writes the same for every instance of the batched 2-D
workload (oracle_batch.json, 32 sample nodes per instance) together with
the Hellmann-Feynman derivative dlambda/dtheta of every instance for its
eight Fourier parameters.  "pcg<c>" adds to oracle_config<c>.json the
iteration count of the oracle's PCG with the two-level additive Schwarz
preconditioner (exact local solves, equal weights) on A_sigma u = M 1 from
u = 0 to rtol 1e-10 (the first inner solve of the inverse iteration) and
the true relative residual ||b - A_sigma u|| / ||b|| of the returned u (the
recursively updated residual drifts from it by the rounding of the updates).
Usage:  python tests/golden/make_golden.py 1 2 [3 4] [batch] [pcg2 pcg4]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle.fem import Grid, assemble_kron  # noqa: E402
from oracle.potential import kron_terms  # noqa: E402
from oracle.cell import cell_problem  # noqa: E402
from oracle.ipm import inverse_iteration_direct, spectral_residual  # noqa: E402
from oracle.grad import eigenvalue_grad  # noqa: E402
from oracle.pcg import pcg  # noqa: E402
from oracle.problem import Problem  # noqa: E402


def golden(c, nsample=256, cfg=None, with_grad=False):
    cfg = W.config(c) if cfg is None else cfg
    t0 = time.time()
    p, q, L, ne = cfg["p"], cfg["q"], cfg["L"], cfg["ne"]
    cell = cell_problem(p, q, ne, cfg["V"], route="kron")
    g = Grid(p, q, L, ne)
    K, M, MV = assemble_kron(g, kron_terms(cfg["V"], p, q))
    A = (K + MV).tocsr()
    res = inverse_iteration_direct(A, M, cell["sigma"], g if g.d == 2 else None, tol=1e-13,
                                   maxit=200)
    x = res["x"]
    idx = np.sort(np.random.default_rng(77 + c).choice(g.n, size=min(nsample, g.n), replace=False))
    out = dict(config=c, name=cfg["name"], n=int(g.n), sigma=cell["sigma"], sigma2=cell["sigma2"],
               lam=res["lam"], outer_its=int(res["its"]), dx_last=float(res["dx_hist"][-1]),
               spectral_residual=spectral_residual(A, M, res["lam"], x),
               sample_idx=idx.tolist(), sample_x=x[idx].tolist(),
               xMx=float(x @ (M @ x)), sumMx=float(np.sum(M @ x)),
               seconds=time.time() - t0)
    if with_grad:
        out["grad"] = eigenvalue_grad(g, M, x, cfg["V"]).tolist()
    return out


def golden_batch(nsample=32):
    out = []
    for j, cfg in enumerate(W.batch_config()):
        d = golden(100 + j, nsample=nsample, cfg=cfg, with_grad=True)
        d["instance"], d["L"] = j, cfg["L"]
        out.append(d)
        print("batch", j, cfg["L"], d["lam"], d["outer_its"], f"{d['seconds']:.1f}s", flush=True)
    return out


def pcg_count(c):
    """Iterations of the oracle's PCG + AS2 on A_sigma u = M 1, u0 = 0, rtol 1e-10."""
    P = Problem(W.config(c), route="kron")
    b = P.M @ np.ones(P.grid.n)
    res = pcg(lambda v: P.A_sigma @ v, b, P.preconditioner(True).apply, rtol=1e-10, maxit=2000)
    assert res.status == "ok", res.status
    true_rel = float(np.linalg.norm(b - P.A_sigma @ res.x) / np.linalg.norm(b))
    return int(res.iters), true_rel


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        if arg.startswith("pcg"):
            c = int(arg[3:])
            path = os.path.join(HERE, f"oracle_config{c}.json")
            d = json.load(open(path))
            d["pcg_iters_M1"], d["pcg_true_relres_M1"] = pcg_count(c)
            json.dump(d, open(path, "w"), indent=1)
            print("pcg", c, d["pcg_iters_M1"], d["pcg_true_relres_M1"], flush=True)
            continue
        if arg == "batch":
            json.dump(golden_batch(), open(os.path.join(HERE, "oracle_batch.json"), "w"), indent=1)
            continue
        c = int(arg)
        d = golden(c)
        path = os.path.join(HERE, f"oracle_config{c}.json")
        json.dump(d, open(path, "w"), indent=1)
        print(c, d["n"], d["sigma"], d["lam"], d["outer_its"], f"{d['seconds']:.1f}s", flush=True)
