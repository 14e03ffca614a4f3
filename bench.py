#!/usr/bin/env python3
"""Benchmark of the sparse CG hot path on one MI355X.

Default workload: 3D 7-point Poisson on a 256^3 grid (n = 16,777,216,
nnz = 117,047,296, int32 CSR, float64), x* ~ U[-1,1] (seeded), b = A x*,
unpreconditioned float64 CG for a fixed 500 iterations, all rows on the GPU.
One step = one cg_solve (setup residual, 500 iterations, true residual).

Prints one JSON line: CG iterations/s (whole job), the SpMV roofline of the
dominant kernel (algorithmic bytes per launch / mean launch time measured with
HIP events on the solver's stream), and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def spmv_algorithmic_bytes(n: int, nnz: int) -> int:
    """int32 col + float64 val per nonzero, row pointers, q written once, p read once."""
    return 12 * nnz + 4 * (n + 1) + 8 * n + 8 * n


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for fn in sorted(os.listdir(os.path.join(ROOT, "paper_2608_09647_amd", "csrc"))):
        if fn.endswith((".hip", ".h")):
            with open(os.path.join(ROOT, "paper_2608_09647_amd", "csrc", fn), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str):
    """Per-launch HBM bytes from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            table = json.load(f)
        ent = table.get(key)
        if ent and ent.get("source_hash") == kernel_source_hash():
            return ent.get("bytes_per_launch")
    except (OSError, ValueError):
        return None
    return None


def cpu_baseline_cg(problem, iters_hint: int, target_s: float = 12.0) -> dict:
    """The oracle's CG, untouched, on a bounded sample: a fixed number of CG
    iterations of the same system, all host threads for its row loops."""
    import oracle
    t0 = time.perf_counter()
    oracle.cg(problem.A, problem.b, tol=0.0, maxit=2)
    t_cal = time.perf_counter() - t0
    k = max(3, min(iters_hint, int(target_s / max(t_cal / 2.0, 1e-6))))
    t0 = time.perf_counter()
    out = oracle.cg(problem.A, problem.b, tol=0.0, maxit=k)
    dt = time.perf_counter() - t0
    return {"value": out["iterations"] / dt, "unit": "iter/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{out['iterations']} fixed-work CG iterations of the same system "
                      f"({dt:.1f} s, including its setup residual and final true residual)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="poisson3d_256")
    ap.add_argument("--iters", type=int, default=500, help="fixed CG iterations per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X "
              "(multi-GPU row sharding is described in DESIGN.md, not run).", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2608_09647_amd import inputs as I
    from paper_2608_09647_amd import cgmi

    if args.config != "poisson3d_256":
        raise SystemExit(f"unknown config {args.config}")
    t0 = time.perf_counter()
    prob = I.poisson3d_problem(256, seed=2)
    A = prob.A
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated {prob.name} n={A.n} nnz={A.nnz} in {gen_s:.1f}s", file=sys.stderr,
          flush=True)

    dev = torch.device("cuda:0")
    b = torch.from_numpy(prob.b).to(dev)
    x = torch.zeros_like(b)
    solver = cgmi.Solver(A)
    solver.set_opts(profile=1)
    for _ in range(args.warmup):
        x.zero_()
        solver.solve(b, x, tol=0.0, maxit=args.iters)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    t_spmv = 0.0
    n_spmv = 0
    iters = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x.zero_()
        _, res = solver.solve(b, x, tol=0.0, maxit=args.iters)
        t_spmv += res["t_spmv"]
        n_spmv += res["n_spmv"]
        iters += res["iterations"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f}s, rel_res_true={res['rel_res_true']:.3e}",
          file=sys.stderr, flush=True)

    spmv_bytes = spmv_algorithmic_bytes(A.n, A.nnz)
    t_launch = t_spmv / max(n_spmv, 1)
    achieved = spmv_bytes / t_launch / 1e9
    line = {
        "metric": "CG iters/s + SpMV GB/s (%HBM peak); time to 1e-10 residual, plain vs learned-PC",
        "value": iters / elapsed,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson3d_7pt_256^3_fp64_cg_fixed_work", "n": A.n, "nnz": A.nnz,
                   "iterations_per_step": args.iters, "row_share_gpu": 1.0, "index": "int32",
                   "seed": 2},
        "spmv_gbs": achieved,
        "spmv_us": 1e6 * t_launch,
        "rel_res_true": res["rel_res_true"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("spmv_poisson3d_256")},
    }
    solver.close()
    del b, x
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_cg(prob, args.iters)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
