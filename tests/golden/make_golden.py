"""Writes the stored oracle results for the full-size configurations.

Calls only the oracle (plain FP64 CPU): for each configuration the shift
sigma (cell problem), the smallest eigenpair by sigma-shifted inverse
iteration with exact solves to ||x_{k+1} - x_k||_M <= 1e-13, the second
eigenvalue (for the contraction rate), and the eigenvector at seeded sample
nodes.  "batch" writes the same for every instance of the batched 2-D
workload (oracle_batch.json, 32 sample nodes per instance).
Usage:  python tests/golden/make_golden.py 1 2 [3 4] [batch]
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


def golden(c, nsample=256, cfg=None):
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
    return out


def golden_batch(nsample=32):
    out = []
    for j, cfg in enumerate(W.batch_config()):
        d = golden(100 + j, nsample=nsample, cfg=cfg)
        d["instance"], d["L"] = j, cfg["L"]
        out.append(d)
        print("batch", j, cfg["L"], d["lam"], d["outer_its"], f"{d['seconds']:.1f}s", flush=True)
    return out


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        if arg == "batch":
            json.dump(golden_batch(), open(os.path.join(HERE, "oracle_batch.json"), "w"), indent=1)
            continue
        c = int(arg)
        d = golden(c)
        path = os.path.join(HERE, f"oracle_config{c}.json")
        json.dump(d, open(path, "w"), indent=1)
        print(c, d["n"], d["sigma"], d["lam"], d["outer_its"], f"{d['seconds']:.1f}s", flush=True)
