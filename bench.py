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


SPMV_SOURCES = ("kernels_cg.hip", "cgmi_internal.h")


def kernel_source_hash() -> str:
    """Hash of the sources that define the CG kernels (the counters in
    profiles/traffic.json are valid only for these exact sources)."""
    h = hashlib.sha256()
    for fn in SPMV_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_09647_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str, spmv_kind: int):
    """Per-launch HBM bytes from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources with the same SpMV tiling; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            table = json.load(f)
        ent = table.get(key)
        if ent and ent.get("source_hash") == kernel_source_hash() and ent.get("spmv_kind") == spmv_kind:
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


def _timed_solve(solver, b, x0, tol, maxit, reps):
    import torch
    times, res = [], None
    for _ in range(reps):
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, res = solver.solve(b, x, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return x, res, times


def bench_time_to_tol(args, prob, variants, metric, workload, extra=None):
    """Time-to-1e-10 comparisons on one system: each variant is a dict of
    solver options; reports the mean of `steps` solves after `warmup`."""
    import numpy as np
    import torch
    from paper_2608_09647_amd import cgmi
    dev = torch.device("cuda:0")
    b = torch.from_numpy(prob.b).to(dev)
    x0 = torch.zeros_like(b)
    out = {}
    xs = {}
    for name, opts in variants.items():
        solver = cgmi.Solver(prob.A)
        solver.set_opts(**opts)
        _timed_solve(solver, b, x0, 1e-10, 200000, args.warmup)
        x, res, times = _timed_solve(solver, b, x0, 1e-10, 200000, args.steps)
        xs[name] = x.cpu().numpy()
        out[name] = {"seconds": float(np.mean(times)), "min_seconds": float(np.min(times)),
                     "iterations": res["iterations"], "fp64_residuals": res["fp64_residuals"],
                     "rel_res_true": res["rel_res_true"], "status": res["code"],
                     "fell_back": res["fell_back"]}
        solver.close()
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)
    return out, xs


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="poisson3d_256",
                    choices=["poisson3d_256", "poisson3d_256_split", "poisson2d_64", "random_spd_2m"])
    ap.add_argument("--share", type=float, default=0.5, help="GPU row share for the split config")
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

    if args.config == "random_spd_2m":
        return bench_mixed(args)
    if args.config == "poisson2d_64":
        return bench_small(args)
    if args.config == "poisson3d_256_split":
        return bench_split(args)
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
        "spmv_kind": {1: "vector_bins", 2: "stream", 3: "sliced"}.get(res["spmv_kind"]),
        "rel_res_true": res["rel_res_true"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("spmv_poisson3d_256", res["spmv_kind"])},
    }
    solver.close()
    del b, x
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_cg(prob, args.iters)
    print(json.dumps(line), flush=True)
    return 0


def _line(metric, value, unit, args, ms, config, higher=True, **extra):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
         "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak",
         "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": config}
    d.update(extra)
    return d


def bench_mixed(args) -> int:
    """Random SPD n = 2M: float32-inner/float64-refined CG vs plain float64 CG to 1e-10."""
    import numpy as np
    from paper_2608_09647_amd import inputs as I
    prob = I.random_spd_problem(2_000_000, seed=3)
    print(f"[bench] generated {prob.name} nnz={prob.A.nnz}", file=sys.stderr, flush=True)
    out, xs = bench_time_to_tol(args, prob, {"fp64": {}, "mixed": {"precision": 1}},
                                None, None)
    err = float(np.linalg.norm(xs["mixed"] - xs["fp64"]) / np.linalg.norm(xs["fp64"]))
    sp = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    line = _line("time to 1e-10 true relative residual: float32-inner/float64-refined CG "
                 "vs plain float64 CG", out["mixed"]["seconds"], "s", args,
                 1e3 * out["mixed"]["seconds"],
                 {"workload": "random_spd_lognormal_n2M_mixed_vs_fp64", "n": prob.A.n,
                  "nnz": prob.A.nnz, "tol": 1e-10, "seed": 3}, higher=False,
                 plain_fp64=out["fp64"], mixed=out["mixed"], speedup_vs_fp64=sp,
                 mixed_rel_error_vs_fp64_solution=err)
    line["dtype"] = "f32+f64"
    print(json.dumps(line), flush=True)
    return 0


def bench_small(args) -> int:
    """2D Poisson 64x64 to 1e-10, all rows on the GPU (single-workgroup path)."""
    from paper_2608_09647_amd import inputs as I
    prob = I.poisson2d_problem(64, seed=1)
    out, _ = bench_time_to_tol(args, prob, {"small_path": {"small_path": 1},
                                            "multi_kernel": {"small_path": 0}}, None, None)
    best = out["small_path"]
    line = _line("CG iterations/s to 1e-10 (2D Poisson 64x64)",
                 best["iterations"] / best["seconds"], "iter/s", args, 1e3 * best["seconds"],
                 {"workload": "poisson2d_5pt_64x64_fp64_cg_to_1e-10", "n": prob.A.n,
                  "nnz": prob.A.nnz, "seed": 1}, paths=out)
    print(json.dumps(line), flush=True)
    return 0


def bench_split(args) -> int:
    """256^3 Poisson with the GPU owning the first share of rows and host
    threads the rest, p exchanged every iteration (whole segments and halo)."""
    import numpy as np
    import torch
    from paper_2608_09647_amd import inputs as I, cgmi
    prob = I.poisson3d_problem(256, seed=2)
    n = prob.A.n
    n_gpu = int(np.floor(args.share * n + 0.5))
    iters = min(args.iters, 50)
    b = torch.from_numpy(prob.b).cuda()
    res_all = {}
    for name, ex in (("whole", 0), ("halo", 1)):
        s = cgmi.Solver(prob.A, 0, n_gpu)
        s.set_opts(exchange=ex)
        _timed_solve(s, b, torch.zeros_like(b), 0.0, iters, max(1, args.warmup))
        _, res, times = _timed_solve(s, b, torch.zeros_like(b), 0.0, iters, args.steps)
        res_all[name] = {"seconds": float(np.mean(times)), "iter_per_s": iters / float(np.mean(times)),
                         **{k: res[k] for k in ("t_gpu", "t_cpu", "t_barrier", "t_d2h", "t_h2d",
                                                 "rows_gpu", "rows_cpu", "nnz_gpu", "nnz_cpu")}}
        s.close()
        print(f"[bench] split {name}: {res_all[name]}", file=sys.stderr, flush=True)
    best = max(res_all.values(), key=lambda r: r["iter_per_s"])
    line = _line("CG iters/s, split rows (GPU share + host complement, explicit p exchange)",
                 best["iter_per_s"], "iter/s", args, 1e3 * best["seconds"],
                 {"workload": f"poisson3d_7pt_256^3_fp64_cg_split_g{args.share}",
                  "n": n, "nnz": prob.A.nnz, "iterations_per_step": iters,
                  "row_share_gpu": args.share}, exchange=res_all)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
