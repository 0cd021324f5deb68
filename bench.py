"""Benchmark of the hot path: time-to-eigenpair and PCG DOF*iter/s on one GPU.

A step is one full eigen-solve: sigma-shifted inverse iteration from the
start vector 1/||1||_M to ||x_{k+1} - x_k||_M <= 1e-9 with PCG + two-level
additive Schwarz (PerFact coarse space) inner solves to rtol 1e-10, on the
2-D workload Omega = (0,256) x (0,1), Q1 with h = 1/64 (1,032,129 unknowns),
256 unit-cell subdomains with 4 overlap layers and the seeded 4-term periodic
potential.  Set-up (tables, cell problem, local factorisations, coarse
matrix) happens once before the timed region.  value = n_dof * (sum of PCG
iterations) / time.  The eigenvalue of every timed solve is checked against
the stored oracle result.

The default local solves are the dense bf16 inverses on MFMA (FP32
accumulation; CG, residuals, Rayleigh quotient and coarse solve in FP64); the
same solve with FP64 block-chain local solves is timed as the comparison.
Also reports the roofline of the dominant kernel (live HIP-event timing on the
library's stream) and the oracle's CPU throughput on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0

# HBM bytes per launch of the dense local-solve GEMM on the 2-D L=256, h=1/64
# workload, from rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs, each scaled by
# what the counter read for a plain device copy of known size (FETCH x 2.0,
# WRITE x 1.0).  Valid only for the kernel source they were taken from (the
# text from the tile constants to the end of k_dense_gemm): when it changes the
# figure is reported as null until the counters are taken again.
COUNTED_TRAFFIC = {
    "source": "paper_2311_08757_amd/csrc/k_dense.hip",
    "begin": "constexpr int kTM = 128", "end": "// Batches of at most kGemvMax rows",
    # the coarse right-hand-side workgroups the GEMM launch carries
    "extra_sources": ["paper_2311_08757_amd/csrc/k_coarse.h"],
    "sha256": "97d476567b86f46f118c15c9f7e05948a6434cd5400de9e84224921632e8fe4f",
    "workload": "2d-L256-ne64", "local_prec": "bf16",
    "fetch_kib": 34436.4, "fetch_factor": 2.0, "write_kib": 13448.1, "write_factor": 1.0,
}


def counted_traffic(workload, local_prec):
    c = COUNTED_TRAFFIC
    if workload != c["workload"] or local_prec != c["local_prec"]:
        return None
    with open(os.path.join(ROOT, c["source"])) as f:
        src = f.read()
    a, b = src.find(c["begin"]), src.find(c["end"])
    if a < 0 or b < a:
        return None
    text = src[a:b]
    for extra in c["extra_sources"]:
        with open(os.path.join(ROOT, extra)) as f:
            text += f.read()
    if hashlib.sha256(text.encode()).hexdigest() != c["sha256"]:
        return None
    return 1024.0 * (c["fetch_kib"] * c["fetch_factor"] + c["write_kib"] * c["write_factor"])


# The local-solve kernel of each precision, the peak it is measured against and
# what its executed work counts.
LOCAL_PATHS = {
    "bf16": {"kernel": "k_dense_gemm (single-bf16 dense inverse on MFMA, all subdomains)",
             "bound": "mfma", "peak": BF16_PEAK_TFLOPS,
             "executed": "dense inverse applied once: 2 m^2 flop per subdomain"},
    "bf16x3": {"kernel": "k_dense_gemm (bf16 hi/lo dense inverse on MFMA, all subdomains)",
               "bound": "mfma", "peak": BF16_PEAK_TFLOPS,
               "executed": "dense inverse applied once: 2 m^2 flop per subdomain"},
    "fp32": {"kernel": "batched block-chain solves, FP32 (k_chain_*)",
             "bound": "mfma", "peak": FP32_PEAK_TFLOPS,
             "executed": "block-chain sweeps: 4 nch b^2 flop per subdomain"},
    "fp64": {"kernel": "block-chain solves, FP64 (k_local_solves_2d / k_chain_*)",
             "bound": "alu", "peak": FP64_PEAK_TFLOPS,
             "executed": "block-chain sweeps: 4 nch b^2 flop per subdomain"},
}


def subdomain_boxes(cfg):
    """Extents of every subdomain box: cells of the expanding axes extended by
    delta layers and clipped to the domain, all unknowns of the fixed axes."""
    import itertools
    p, q, L, ne, delta = cfg["p"], cfg["q"], cfg["L"], cfg["ne"], cfg["delta"]
    nfix = int(round(cfg.get("ell", 1) * ne)) - 1
    ext = []
    for c in range(1, L + 1):
        lo = max((c - 1) * ne - delta + 1, 1)
        hi = min(c * ne + delta - 1, L * ne - 1)
        ext.append(hi - lo + 1)
    return [list(e) + [nfix] * q for e in itertools.product(ext, repeat=p)]


def local_solve_work(cfg):
    """Algorithmic flops of one application of all local solves: an exact banded
    Cholesky solve per subdomain (forward and backward substitution, 4 m hb
    flops for m unknowns and half-bandwidth hb; the box ordered with its
    longest direction slowest: hb = f + 1 in 2-D, f (g + 1) + 1 in 3-D for the
    extents f <= g of the two shorter directions)."""
    flop = 0.0
    entries = 0
    for dims in subdomain_boxes(cfg):
        d = sorted(dims)
        m = 1
        for v in d:
            m *= v
        hb = d[0] + 1 if len(d) == 2 else d[0] * (d[1] + 1) + 1
        flop += 4.0 * m * hb
        entries += m
    n = 1
    for a in range(cfg["p"] + cfg["q"]):
        n *= cfg["L"] * cfg["ne"] - 1 if a < cfg["p"] else int(round(cfg.get("ell", 1) * cfg["ne"])) - 1
    return {"flop": flop, "flop_per_dof": flop / n, "batch_entries": entries, "n": n}


def iteration_table(parts, cfg, prob, alg, local_prec, path):
    """Per-part work, time and fraction of one PCG iteration.  Vector bytes are
    algorithmic FP64 traffic (each vector read or written once); restricted
    residuals and local solutions count once per subdomain entry at the width
    the path stores them."""
    n = prob.n_dof
    ent = alg["batch_entries"]
    rbytes = {"bf16": 2, "bf16x3": 4, "fp32": 8, "fp64": 8}[local_prec]
    ybytes = {"bf16": 4, "bf16x3": 4, "fp32": 8, "fp64": 8}[local_prec]
    rows = [
        {"part": "stencil_dir", "does": "p = z + beta p, q = A_sigma p, p.q", "bound": "hbm",
         "work": 32.0 * n, "work_unit": "B"},
        {"part": "restrict_xr", "does": "x += alpha p, r -= alpha q, ||r||^2, R_i r",
         "bound": "hbm", "work": 48.0 * n + rbytes * ent, "work_unit": "B"},
        {"part": "local_solves", "does": path["kernel"], "bound": path["bound"],
         "work": alg["flop"], "work_unit": "flop"},
        {"part": "correction", "does": "clipped-class Schur correction and A_0^{-1} c (dense paths)",
         "bound": "latency", "work": None, "work_unit": None},
        {"part": "extend_check", "does": "z = sum R_i^T y_i + coarse field, stopping test, r.z",
         "bound": "hbm", "work": 16.0 * n + ybytes * ent, "work_unit": "B"},
    ]
    total = 0.0
    for r in rows:
        us = parts[r["part"]]
        r["us"] = us
        total += us
        if r["work"] and us > 0:
            if r["work_unit"] == "B":
                r["achieved"], r["unit"] = r["work"] / us / 1e3, "GB/s"
                r["frac"] = r["achieved"] / HBM_PEAK_GBS
            else:
                r["achieved"], r["unit"] = r["work"] / us / 1e6, "TFLOP/s"
                r["frac"] = r["achieved"] / path["peak"]
    vec = sum(r["work"] for r in rows if r["work_unit"] == "B")
    return {"parts": rows, "us_per_iteration": total,
            "vector_bytes": vec, "vector_floor_us": vec / HBM_PEAK_GBS / 1e3,
            "method": "HIP events between the launches of 30 PCG iterations on the library stream "
                      "(ddeig_profile_iteration); vectors of the config sizes sit in the 256 MB "
                      "Infinity Cache, so B rates are effective rates"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--local-prec", default=None, choices=["fp64", "fp32", "bf16x3", "bf16"],
                    help="local solve precision (default bf16; fp32 for the 3-D workload with one "
                         "expanding axis, whose clipped subdomains miss more unknowns than the "
                         "dense path's corrections take)")
    ap.add_argument("--graphs", type=int, default=1, choices=[0, 1],
                    help="replay PCG iteration blocks from captured HIP graphs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--kernels-only", action="store_true",
                    help="set-up, then only the per-kernel timings (for counter runs)")
    ap.add_argument("--hbm-only", action="store_true",
                    help="only the HBM-scale stencil sweeps (2-D and 3-D), one JSON line each")
    ap.add_argument("--no-hbm", action="store_true",
                    help="skip the stencil measurement at the HBM-sized 2-D workload")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    ap.add_argument("--cpu-sample", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-pcg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-tol", type=float, default=1e-9, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-pin", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--solver", default=None,
                    choices=["cg_asm2", "gmres_ras2", "stationary_ras2", "stationary_ras1"],
                    help="time only shifted solves A_sigma u = b (b seeded, rtol 1e-10) with this "
                         "inner solver, one per step (for kernel profiles of that solver)")
    args = ap.parse_args()
    if args.local_prec is None:
        args.local_prec = "fp32" if args.config == 3 else "bf16"
    return args


def host_info():
    """CPU model, usable cores and RAM of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cores_usable": len(os.sched_getaffinity(0)), "ram_gib": ram}


def cpu_direct(cfgno, tol_x):
    """The oracle's direct route to the eigenpair on the same workload, timed by
    phase: assembly (Kronecker route), cell problem (dense eigh), banded
    Cholesky of A_sigma, shifted inverse iteration with exact solves to
    ||x_{k+1} - x_k||_M <= tol_x (the GPU's stopping rule)."""
    import workloads as W
    from oracle.fem import Grid, assemble_kron
    from oracle.potential import kron_terms
    from oracle.cell import cell_problem
    from oracle.ipm import DirectSolver, inverse_iteration
    cfg = W.config(cfgno)
    p, q, L, ne = cfg["p"], cfg["q"], cfg["L"], cfg["ne"]
    t = {}
    t0 = time.perf_counter()
    g = Grid(p, q, L, ne)
    K, M, MV = assemble_kron(g, kron_terms(cfg["V"], p, q))
    A = (K + MV).tocsr()
    t1 = time.perf_counter()
    cell = cell_problem(p, q, ne, cfg["V"], route="kron")
    t2 = time.perf_counter()
    ds = DirectSolver(A - cell["sigma"] * M, g)
    t3 = time.perf_counter()
    res = inverse_iteration(A, M, cell["sigma"], lambda b: (ds.solve(b), 0), tol=tol_x, maxit=200)
    t4 = time.perf_counter()
    t = {"assembly_s": t1 - t0, "cell_problem_s": t2 - t1, "factorisation_s": t3 - t2,
         "inverse_iteration_s": t4 - t3, "total_s": t4 - t0}
    return dict(phases=t, outer_its=int(res["its"]), lam=res["lam"], n=int(g.n),
                threads=os.environ.get("OPENBLAS_NUM_THREADS"),
                affinity=sorted(os.sched_getaffinity(0)))


def cpu_pcg(cfgno, iters=10):
    """The oracle's PCG with its two-level additive Schwarz preconditioner
    (exact local solves) on the same workload: `iters` iterations of one
    inner solve (b = M 1) after the oracle's own set-up, as DOF*iter/s."""
    import numpy as np
    import workloads as W
    from oracle.problem import Problem
    from oracle.pcg import pcg
    cfg = W.config(cfgno)
    t0 = time.perf_counter()
    P = Problem(cfg, route="kron")
    M2 = P.preconditioner(True)
    t_setup = time.perf_counter() - t0
    b = P.M @ np.ones(P.grid.n)
    t1 = time.perf_counter()
    res = pcg(lambda v: P.A_sigma @ v, b, M2.apply, rtol=0.0, maxit=iters)
    dt = time.perf_counter() - t1
    return dict(value=P.grid.n * res.iters / dt, iters=res.iters, seconds=dt, setup_s=t_setup,
                n=int(P.grid.n), affinity=sorted(os.sched_getaffinity(0)))


def run_cpu_baseline(cfgno, tol_x):
    """The oracle in child processes: its PCG rate on one pinned core (the
    metric's unit), and its direct route to the eigenpair (cpu_direct) on one
    pinned core and on all usable cores."""
    out = {}
    ncores = len(os.sched_getaffinity(0))
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    env["CUDA_VISIBLE_DEVICES"] = ""
    env["HIP_VISIBLE_DEVICES"] = ""
    res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample", "--cpu-pcg",
                          "--cpu-pin", "--config", str(cfgno)], capture_output=True, text=True,
                         env=env, timeout=900)
    if res.returncode != 0:
        raise RuntimeError("cpu baseline failed: " + res.stderr[-2000:])
    out["pcg"] = json.loads(res.stdout.strip().splitlines()[-1])
    print(f"# oracle PCG (one core): {out['pcg']['iters']} iterations in "
          f"{out['pcg']['seconds']:.2f} s", file=sys.stderr, flush=True)
    for leg, threads in (("one_core", 1), ("all_cores", ncores)):
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = str(threads)
        env["CUDA_VISIBLE_DEVICES"] = ""
        env["HIP_VISIBLE_DEVICES"] = ""
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-sample", "--config", str(cfgno),
               "--cpu-tol", repr(tol_x)]
        if threads == 1:
            cmd += ["--cpu-pin"]
        res = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=900)
        if res.returncode != 0:
            raise RuntimeError("cpu baseline failed: " + res.stderr[-2000:])
        out[leg] = json.loads(res.stdout.strip().splitlines()[-1])
        out[leg]["cores"] = threads
        print(f"# oracle direct route ({leg}, {threads} thread(s)): "
              f"{out[leg]['phases']['total_s']:.2f} s", file=sys.stderr, flush=True)
    return out


HBM_WORKLOADS = {
    # name: (p, q, L, n_e, delta, potential config) -- vectors far beyond the
    # 256 MB Infinity Cache, so the sweep streams from HBM
    "2d": ("2d-L16384-ne64", 1, 1, 16384, 64, 4, 2),
    "3d": ("3d-p1q2-L2048-ne32", 1, 2, 2048, 32, 2, 3),
}


def hbm_stencil(dd, W, torch, which="2d"):
    """The A_sigma stencil at HBM scale, timed live with HIP events next to a
    plain device copy of the same bytes: 2-D L = 16384, h = 1/64 (66,060,225
    unknowns, 1.06 GB per apply) or 3-D p = 1, q = 2, L = 2048, h = 1/32
    (62,980,096 unknowns, 1.01 GB per apply)."""
    name, p, q, L, ne, delta, cfgno = HBM_WORKLOADS[which]
    prob = dd.assemble(p, q, L, ne, W.config(cfgno)["V"], delta, coarse=False, local_prec="fp64")
    dd.cell_shift(prob)
    n = prob.n_dof
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    t_us, nbytes = dd.profile_kernel(prob, "stencil", reps=20, x=x, y=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    y.copy_(x)
    e0.record()
    for _ in range(20):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    t_copy = e0.elapsed_time(e1) * 1e3 / 20
    del prob, x, y
    torch.cuda.empty_cache()
    return {"workload": f"{name} ({n:,} unknowns)", "launch_us": t_us,
            "bytes_per_launch": nbytes, "achieved": nbytes / t_us / 1e3, "unit": "GB/s",
            "peak": HBM_PEAK_GBS, "frac": nbytes / t_us / 1e3 / HBM_PEAK_GBS,
            "device_copy_same_bytes_GBs": nbytes / t_copy / 1e3}


def bench_batch(args):
    """The batched workload: 64 independent 2-D instances (L_j uniform in
    16..256, h = 1/32, 2 overlap layers, each with its own seeded potential) in
    one batch: every PCG iteration is one grouped launch per kernel over all
    instances.  A step is the inverse iteration of all 64 instances to their
    eigenpairs; value = sum_j n_j * (PCG iterations of j) / time.  The same
    eigenpairs solved one instance after another with the single-problem path
    are timed as the comparison."""
    import numpy as np
    import torch
    import paper_2311_08757_amd as dd
    import workloads as W

    inst = W.batch_config()
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_batch.json")))
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    probs = []
    for c in inst:
        prob = dd.assemble(c["p"], c["q"], c["L"], c["ne"], c["V"], c["delta"],
                           local_prec=args.local_prec)
        dd.cell_shift(prob)
        probs.append(prob)
    batch = dd.batch_create(probs, graphs=bool(args.graphs))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    tune = dd.batch_query(batch)
    ns = [p.n_dof for p in probs]
    xs = [torch.zeros(n, dtype=torch.float64, device="cuda") for n in ns]
    print(f"# batch setup {t_setup:.2f}s, {len(probs)} instances, {sum(ns)} unknowns, "
          f"GEMM tuning {tune}", file=sys.stderr, flush=True)

    def solve_all():
        for x in xs:
            x.zero_()
        st, info = dd.batch_inverse_iteration(batch, xs, tol_x=1e-9, rtol_inner=1e-10,
                                              maxit_inner=3000)
        return info

    for i in range(args.warmup):
        solve_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dof_iters = 0
    for i in range(args.steps):
        info = solve_all()
        dof_iters += sum(n * f["inner_sum"] for n, f in zip(ns, info))
    torch.cuda.synchronize()
    T = max(time.perf_counter() - t0, 1e-9)
    lam_err = max(abs(f["lam"] - g["lam"]) / abs(g["lam"]) for f, g in zip(info, gold))
    print(f"# timed {args.steps} batched solves in {T:.3f}s, max lambda rel err {lam_err:.2e}",
          file=sys.stderr, flush=True)
    # the same eigenpairs one instance at a time
    t_seq, seq_iters = None, None
    if not args.no_compare:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        seq_iters = 0
        for p, x in zip(probs, xs):
            x.zero_()
            o = dd.inverse_iteration(p, x, tol_x=1e-9, rtol_inner=1e-10, maxit_inner=3000)
            seq_iters += o["inner_sum"]
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t1
    c0 = inst[0]
    m = (c0["ne"] + 2 * c0["delta"] - 1) * (c0["ne"] - 1)  # unknowns of the unclipped box
    flop = 2.0 * m * m * sum(p.n_sub for p in probs)
    t_gemm = tune["tune_us"][(tune["ksplit"] - 1) * 2 + tune["order"]]
    res = {
        "metric": "PCG DOF*iter/s inside time-to-eigenpair, batched (64 independent instances, "
                  "sigma-shifted inverse iteration, PCG + two-level additive Schwarz)",
        "value": dof_iters / T,
        "unit": "DOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / max(args.steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "f64 (bf16x3 MFMA local solves, f32 accumulate)",
                  "bf16": "f64 (bf16 MFMA local solves, f32 accumulate)"}[args.local_prec],
        "data": "synthetic (seeded periodic potentials)",
        "config": {"workload": "2d-batch64-L16..256-ne32", "instances": len(probs),
                   "n_dof_total": sum(ns), "local_prec": args.local_prec,
                   "time_to_all_eigenpairs_ms": T / max(args.steps, 1) * 1e3, "setup_s": t_setup,
                   "gemm_autotune": tune, "lambda_max_rel_err_vs_oracle": lam_err,
                   "pcg_iters_per_step": dof_iters and sum(f["inner_sum"] for f in info),
                   "sequential_time_ms": t_seq * 1e3 if t_seq else None,
                   "sequential_pcg_iters": seq_iters,
                   "speedup_vs_sequential": t_seq / (T / max(args.steps, 1)) if t_seq else None},
        "roofline": {"bound": "mfma", "kernel": "k_dense_gemm, grouped over all instances",
                     "achieved": flop / t_gemm / 1e6, "peak": BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": flop / t_gemm / 1e6 / BF16_PEAK_TFLOPS,
                     "traffic": None, "launch_us": t_gemm, "work_per_launch_flop": flop},
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def bench_solver(args, dd, W, prob, cfg, t_setup):
    """--solver: one shifted solve per step with the named inner solver."""
    import torch
    n = prob.n_dof
    b = torch.as_tensor(W.random_vector(n, 15), dtype=torch.float64, device="cuda")
    u = torch.zeros_like(b)
    run = {"cg_asm2": lambda: dd.pcg_solve(prob, b, u, rtol=1e-10, maxit=5000),
           "gmres_ras2": lambda: dd.gmres_solve(prob, b, u, kind="ras2", rtol=1e-10, maxit=5000),
           "stationary_ras2": lambda: dd.stationary_ras(prob, b, u, levels=2, rtol=1e-10,
                                                        maxit=10000),
           "stationary_ras1": lambda: dd.stationary_ras(prob, b, u, levels=1, rtol=1e-10,
                                                        maxit=100000)}[args.solver]
    for i in range(args.warmup):
        u.zero_()
        run()
    torch.cuda.synchronize()
    its = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        u.zero_()
        its += run()["iters"]
    torch.cuda.synchronize()
    T = max(time.perf_counter() - t0, 1e-9)
    print(f"# {args.solver}: {args.steps} solves in {T * 1e3:.1f} ms, {its} iterations",
          file=sys.stderr, flush=True)
    print(json.dumps({
        "metric": f"shifted-solve DOF*iter/s ({args.solver}, rtol 1e-10)", "value": n * its / T,
        "unit": "DOF*iter/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": T / max(args.steps, 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": f"f64 ({args.local_prec} local solves)",
        "data": "synthetic (seeded periodic potential, seeded right-hand side)",
        "config": {"workload": cfg["name"], "n_dof": n, "solver": args.solver,
                   "iters_per_solve": its / max(args.steps, 1), "setup_s": t_setup}}),
        flush=True)


def main():
    args = parse()
    if args.cpu_sample:
        if args.cpu_pin:
            os.sched_setaffinity(0, {min(os.sched_getaffinity(0))})
        if args.cpu_pcg:
            print(json.dumps(cpu_pcg(args.config)))
        else:
            print(json.dumps(cpu_direct(args.config, args.cpu_tol)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding "
              "of this path is a design note, not a built component.", file=sys.stderr)
        sys.exit(2)
    if args.hbm_only:
        import torch
        import paper_2311_08757_amd as dd
        import workloads as W
        torch.cuda.set_device(0)
        for which in ("2d", "3d"):
            print(json.dumps(hbm_stencil(dd, W, torch, which)), flush=True)
        return
    if args.config == 5:
        bench_batch(args)
        return
    import numpy as np
    import torch
    import paper_2311_08757_amd as dd
    import workloads as W

    cfg = W.config(args.config)
    gold_path = os.path.join(ROOT, "tests", "golden", f"oracle_config{args.config}.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else None
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    prob = dd.assemble(cfg["p"], cfg["q"], cfg["L"], cfg["ne"], cfg["V"], cfg["delta"],
                       local_prec=args.local_prec, graphs=bool(args.graphs))
    sigma, _ = dd.cell_shift(prob)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    n = prob.n_dof
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    print(f"# setup {t_setup:.2f}s n={n} sigma={sigma:.12f}", file=sys.stderr, flush=True)
    if args.solver:
        bench_solver(args, dd, W, prob, cfg, t_setup)
        return
    if args.kernels_only:
        args.warmup = 0
        args.steps = 0
        args.no_compare = True
        args.no_cpu = True
        args.no_hbm = True
    for i in range(args.warmup):
        x.zero_()
        out = dd.inverse_iteration(prob, x, tol_x=1e-9, rtol_inner=1e-10, maxit_inner=2000)
        print(f"# warmup {i}: lambda={out['lam']:.14f} outer={out['outer_its']} "
              f"inner={out['inner_sum']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inner = 0
    lams = []
    outers = []
    per_solve = []
    spec_res = None
    for i in range(args.steps):
        ts = time.perf_counter()
        x.zero_()
        out = dd.inverse_iteration(prob, x, tol_x=1e-9, rtol_inner=1e-10, maxit_inner=2000)
        per_solve.append((time.perf_counter() - ts) * 1e3)  # the call synchronises
        inner += out["inner_sum"]
        lams.append(out["lam"])
        outers.append(out["outer_its"])
        spec_res = out["spec_res"]
    torch.cuda.synchronize()
    T = max(time.perf_counter() - t0, 1e-9)
    print(f"# timed {args.steps} solves in {T:.3f}s, inner={inner}", file=sys.stderr, flush=True)
    lam_err = None
    if gold is not None and lams:
        lam_err = max(abs(l - gold["lam"]) / abs(gold["lam"]) for l in lams)
        xs = x.cpu().numpy()[gold["sample_idx"]]
        vec_err = float(np.max(np.abs(xs - np.array(gold["sample_x"]))))
        print(f"# lambda rel err vs oracle {lam_err:.3e}, max sampled |x - x_ref| {vec_err:.3e}",
              file=sys.stderr, flush=True)

    # roofline of the dominant kernel (the local solves) and of the stencil,
    # timed live with HIP events on the library's stream
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    dd.apply_precond(prob, x, z)
    t_loc, work_exec = dd.profile_kernel(prob, "local", reps=20)
    t_op, bytes_op = dd.profile_kernel(prob, "stencil", reps=200, x=x, y=y)
    t_pre, _ = dd.profile_kernel(prob, "precond", reps=20, x=x, y=z)
    torch.cuda.synchronize()
    alg = local_solve_work(cfg)
    path = LOCAL_PATHS[args.local_prec]
    print(f"# local solves {t_loc:.2f} us ({alg['flop'] / t_loc / 1e6:.2f} TFLOP/s algorithmic, "
          f"{work_exec / t_loc / 1e6:.1f} TFLOP/s executed), stencil {t_op:.2f} us "
          f"({bytes_op / t_op / 1e3:.1f} GB/s), apply_precond {t_pre:.1f} us",
          file=sys.stderr, flush=True)
    roof = {"bound": path["bound"], "kernel": path["kernel"],
            "achieved": alg["flop"] / t_loc / 1e6, "peak": path["peak"], "unit": "TFLOP/s",
            "frac": alg["flop"] / t_loc / 1e6 / path["peak"],
            "traffic": counted_traffic(cfg["name"], args.local_prec), "traffic_unit": "B",
            "launch_us": t_loc,
            "work_per_launch_flop": alg["flop"],
            "work_basis": "algorithmic: exact banded solves of every subdomain, 4 m_i hb_i flop "
                          f"per subdomain ({alg['flop_per_dof']:.0f} flop per unknown)",
            "executed_flop_per_launch": work_exec,
            "achieved_executed": work_exec / t_loc / 1e6,
            "frac_executed": work_exec / t_loc / 1e6 / path["peak"],
            "executed_basis": path["executed"]}
    if roof["traffic"] is not None:
        # the counted HBM-side bytes of the same launch against the HBM peak:
        # at about 120 executed flop per counted byte the dense GEMM sits below
        # the bf16 ridge (2.5 PFLOP/s / 8 TB/s = 312 flop/B)
        roof["achieved_traffic_GBs"] = roof["traffic"] / t_loc / 1e3
        roof["frac_traffic_hbm"] = roof["traffic"] / t_loc / 1e3 / HBM_PEAK_GBS
    # one PCG iteration part by part (events between the launches of the loop)
    bvec0 = torch.as_tensor(W.random_vector(n, 15), dtype=torch.float64, device="cuda")
    parts = dd.profile_iteration(prob, bvec0, reps=30)
    per_iter = iteration_table(parts, cfg, prob, alg, args.local_prec, path)
    for row in per_iter["parts"]:
        print(f"# iteration part {row['part']}: {row['us']:.2f} us "
              f"({row.get('achieved', '-')} {row.get('unit', '')})", file=sys.stderr, flush=True)
    stencil_roof = {"bound": "hbm", "kernel": "k_stencil2d (A_sigma apply)" if cfg["p"] + cfg["q"] == 2
                    else "k_stencil3d (A_sigma apply)",
                    "workload": cfg["name"] + " (vectors resident in the 256 MB Infinity Cache: "
                                              "effective rate)",
                    "achieved": bytes_op / t_op / 1e3, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": bytes_op / t_op / 1e3 / HBM_PEAK_GBS, "launch_us": t_op,
                    "bytes_per_launch": bytes_op}
    if not args.no_hbm:
        stencil_roof["hbm_scale"] = hbm_stencil(dd, W, torch, "2d")
        stencil_roof["hbm_scale_3d"] = hbm_stencil(dd, W, torch, "3d")
    if args.calib_copy_mib > 0:
        # plain copy of known size for counter calibration; a larger buffer is
        # written in between so that the source is not in the Infinity Cache
        nb = args.calib_copy_mib * (1 << 20) // 8
        a = torch.empty(nb, dtype=torch.float64, device="cuda").fill_(1.0)
        flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(2.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b, flush

    # the same eigen-solve with FP64 block-chain local solves
    cmp = None
    if not args.no_compare and args.local_prec != "fp64":
        # the plain FP64 baseline: FP64 block-chain local solves, no graph capture;
        # its set-up (assemble, cell problem, factorisation, coarse matrix) timed too
        torch.cuda.synchronize()
        ts0 = time.perf_counter()
        p64 = dd.assemble(cfg["p"], cfg["q"], cfg["L"], cfg["ne"], cfg["V"], cfg["delta"],
                          local_prec="fp64", graphs=False)
        dd.cell_shift(p64)
        torch.cuda.synchronize()
        t64_setup = time.perf_counter() - ts0
        x.zero_()
        dd.inverse_iteration(p64, x, tol_x=1e-9, rtol_inner=1e-10, maxit_inner=2000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x.zero_()
        o64 = dd.inverse_iteration(p64, x, tol_x=1e-9, rtol_inner=1e-10, maxit_inner=2000)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        t_mixed = T / max(args.steps, 1)
        cmp = {"fp64_time_to_eigenpair_ms": t64 * 1e3, "fp64_setup_s": t64_setup,
               "fp64_time_to_eigenpair_with_setup_ms": (t64 + t64_setup) * 1e3,
               "fp64_pcg_iters": o64["inner_sum"], "fp64_lambda": o64["lam"],
               "speedup_vs_fp64": t64 / t_mixed,
               "speedup_vs_fp64_with_setup": (t64 + t64_setup) / (t_mixed + t_setup)}
        print(f"# fp64 comparison: {t64 * 1e3:.1f} ms (+ {t64_setup:.2f} s set-up), "
              f"inner={o64['inner_sum']}", file=sys.stderr, flush=True)
        del p64

    # the same dense-inverse local solves at the other MFMA precision: one
    # algorithm, bf16 hi/lo pairs (three products) against single bf16, set-up
    # (the dense inverse) timed too
    prec_cmp = None
    if not args.no_compare and args.local_prec in ("bf16", "bf16x3"):
        other = "bf16x3" if args.local_prec == "bf16" else "bf16"
        torch.cuda.synchronize()
        ts0 = time.perf_counter()
        po = dd.assemble(cfg["p"], cfg["q"], cfg["L"], cfg["ne"], cfg["V"], cfg["delta"],
                         local_prec=other, graphs=bool(args.graphs))
        dd.cell_shift(po)
        torch.cuda.synchronize()
        to_setup = time.perf_counter() - ts0
        x.zero_()
        dd.inverse_iteration(po, x, tol_x=1e-9, rtol_inner=1e-10, maxit_inner=2000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x.zero_()
        oo = dd.inverse_iteration(po, x, tol_x=1e-9, rtol_inner=1e-10, maxit_inner=2000)
        torch.cuda.synchronize()
        to = time.perf_counter() - t1
        prec_cmp = {"local_prec": other, "time_to_eigenpair_ms": to * 1e3, "setup_s": to_setup,
                    "pcg_iters": oo["inner_sum"], "lambda": oo["lam"],
                    "time_ratio_vs_this_run": to / (T / max(args.steps, 1))}
        print(f"# {other} comparison (same dense algorithm): {to * 1e3:.1f} ms "
              f"(+ {to_setup:.2f} s set-up), inner={oo['inner_sum']}", file=sys.stderr, flush=True)
        del po

    # the paper's outer variant (alg:si-lopcg) on the same problem and
    # accuracy: time to the eigenpair with fixed / adaptive inner tolerances
    # and with the preconditioner applied directly (fused)
    # (keys: mode, or inner solver and mode: CG+ASM2 is the default inner
    # solver, gmres_ras2 / stationary_ras2 those of §4.2, ras2_fused applies
    # M_RAS,2 once per step as in §4.3)
    outer = None
    if not args.no_compare:
        outer = {}
        variants = [("fixed", "fixed", "cg"), ("adaptive", "adaptive", "cg"),
                    ("fused", "fused", "cg"), ("gmres_ras2_fixed", "fixed", "gmres"),
                    ("gmres_ras2_adaptive", "adaptive", "gmres"), ("ras2_fused", "fused", "gmres"),
                    ("stationary_ras2_fixed", "fixed", "ras2")]
        for key, mode, inner_solver in variants:
            for rep in range(2):   # the first run allocates the work space
                x.zero_()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                o = dd.lopcg(prob, x, tol_o=1e-9, maxit_outer=5000, mode=mode, rtol_inner=1e-8,
                             inner=inner_solver)
                torch.cuda.synchronize()
                tl = time.perf_counter() - t1
            err = abs(o["lam"] - gold["lam"]) / abs(gold["lam"]) if gold is not None else None
            outer[key] = {"time_to_eigenpair_ms": tl * 1e3, "outer_its": o["outer_its"],
                          "inner_sum": o["inner_sum"], "inner_max": o["inner_max"],
                          "res_norm": o["res_norm"], "lambda_rel_err_vs_oracle": err}
            print(f"# SI-LOPCG {key}: {tl * 1e3:.1f} ms, outer {o['outer_its']}, inner "
                  f"{o['inner_sum']}, lambda err {err}", file=sys.stderr, flush=True)

    # one shifted solve A_sigma u = b (b seeded, rtol 1e-10) by each inner solver
    solvers = None
    if not args.no_compare:
        solvers = {}
        bvec = torch.as_tensor(W.random_vector(n, 15), dtype=torch.float64, device="cuda")
        u = torch.zeros_like(bvec)
        runs = {"cg_asm2": lambda: dd.pcg_solve(prob, bvec, u, rtol=1e-10, maxit=2000),
                "gmres_ras2": lambda: dd.gmres_solve(prob, bvec, u, kind="ras2", rtol=1e-10,
                                                     maxit=2000),
                "stationary_ras2": lambda: dd.stationary_ras(prob, bvec, u, levels=2, rtol=1e-10,
                                                             maxit=5000)}
        for key, f in runs.items():
            for rep in range(2):
                u.zero_()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                o = f()
                torch.cuda.synchronize()
                tl = time.perf_counter() - t1
            solvers[key] = {"time_ms": tl * 1e3, "iters": o["iters"],
                            "us_per_iter": tl * 1e6 / max(o["iters"], 1), "relres": o["relres"]}
            print(f"# solve {key}: {tl * 1e3:.1f} ms, {o['iters']} its", file=sys.stderr,
                  flush=True)

    cpu = None
    if not args.no_cpu and cfg["p"] + cfg["q"] == 2:
        c = run_cpu_baseline(args.config, 1e-9)
        one, pc = c["one_core"], c["pcg"]
        cpu = {"value": pc["value"], "unit": "DOF*iter/s", "cores": 1, "kind": "oracle",
               "sample": f"oracle PCG with its two-level additive Schwarz preconditioner (exact "
                         f"local solves) on the same {pc['n']}-unknown workload: {pc['iters']} "
                         f"iterations of one inner solve (b = M 1) in {pc['seconds']:.2f} s after "
                         f"its {pc['setup_s']:.1f} s set-up; one thread pinned to one core",
               "time_to_eigenpair": {
                   "unit": "ms (incl. set-up)",
                   "route": f"oracle direct route: Kronecker assembly, dense-eigh cell problem, "
                            f"banded Cholesky of A_sigma, inverse iteration with exact solves to "
                            f"||dx||_M <= 1e-9 ({one['outer_its']} steps)",
                   "one_core": {"cores": 1, "value": one["phases"]["total_s"] * 1e3,
                                "phases_s": one["phases"]},
                   "all_cores": {"cores": c["all_cores"]["cores"],
                                 "value": c["all_cores"]["phases"]["total_s"] * 1e3,
                                 "phases_s": c["all_cores"]["phases"]},
                   "gpu_ms_with_setup": T / max(args.steps, 1) * 1e3 + t_setup * 1e3,
                   "lambda_rel_err_vs_gpu": abs(one["lam"] - lams[-1]) / abs(lams[-1])
                   if lams else None},
               "host": host_info()}
    res = {
        "metric": "PCG DOF*iter/s inside time-to-eigenpair (sigma-shifted inverse iteration, "
                  "PCG + two-level additive Schwarz, lambda to 1e-10)",
        "value": n * inner / T,
        "unit": "DOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / max(args.steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f64 (f32 local solves)",
                  "bf16x3": "f64 (bf16x3 MFMA local solves, f32 accumulate)",
                  "bf16": "f64 (bf16 MFMA local solves, f32 accumulate)"}[args.local_prec],
        "data": "synthetic (seeded periodic potential)",
        "config": {"workload": cfg["name"], "p": cfg["p"], "q": cfg["q"], "L": cfg["L"],
                   "h": f"1/{cfg['ne']}", "overlap": cfg["delta"], "n_dof": n,
                   "subdomains": prob.n_sub, "local_prec": args.local_prec,
                   "hip_graphs": bool(args.graphs),
                   "time_to_eigenpair_ms": T / max(args.steps, 1) * 1e3, "setup_s": t_setup,
                   "time_to_eigenpair_with_setup_ms": T / max(args.steps, 1) * 1e3 + t_setup * 1e3,
                   "outer_its": outers[-1] if outers else None,
                   "pcg_iters_per_solve": inner / max(args.steps, 1),
                   "solve_ms_median": float(np.median(per_solve)) if per_solve else None,
                   "solve_ms_min": min(per_solve) if per_solve else None,
                   "lambda": lams[-1] if lams else None, "lambda_rel_err_vs_oracle": lam_err,
                   "spectral_residual": spec_res},
        "env": {"torch": torch.__version__, "hip": torch.version.hip,
                "device": torch.cuda.get_device_name(0)},
        "roofline": roof,
        "pcg_iteration": per_iter,
        "stencil_roofline": stencil_roof,
        "fp64_comparison": cmp,
        "dense_precision_comparison": prec_cmp,
        "si_lopcg": outer,
        "inner_solvers": solvers,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
