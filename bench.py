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
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X, all 256 compute units
N_CUS = 256


SPMV_EVENT_STRIDE = 10


def spmv_algorithmic_bytes(n: int, nnz: int) -> int:
    """int32 col + float64 val per nonzero, row pointers, q written once, p read once."""
    return 12 * nnz + 4 * (n + 1) + 8 * n + 8 * n


SPMV_SOURCES = ("kernels_cg.hip", "cgmi_internal.h")
BATCH_SOURCES = ("kernels_batch.hip", "batch_internal.h")


def kernel_source_hash(sources=SPMV_SOURCES) -> str:
    """Hash of the sources that define a kernel (the counters in
    profiles/traffic.json are valid only for these exact sources)."""
    h = hashlib.sha256()
    for fn in sources:
        with open(os.path.join(ROOT, "paper_2608_09647_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str, spmv_kind, sources=SPMV_SOURCES):
    """Per-launch HBM bytes from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources with the same SpMV tiling (None:
    no tiling to match); else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            table = json.load(f)
        ent = table.get(key)
        if ent and ent.get("source_hash") == kernel_source_hash(sources) and ent.get("spmv_kind") == spmv_kind:
            return ent.get("bytes_per_launch")
    except (OSError, ValueError):
        return None
    return None


def roofline_hbm(alg_bytes: float, t_launch: float, traffic, **extra) -> dict:
    """The dominant kernel's HBM roofline.  `achieved` is algorithmic bytes per
    launch (CSR with int32 indices: what the method must move) over the mean
    launch time; a storage format that skips index streams moves fewer bytes,
    so when the counters give the bytes actually moved (`traffic`) their rate
    is reported beside it as `achieved_measured_bytes` / `frac_measured_bytes`."""
    a = alg_bytes / t_launch / 1e9
    d = {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS,
         "traffic": traffic, "algorithmic_bytes_per_launch": int(alg_bytes), "launch_us": 1e6 * t_launch}
    if traffic:
        m = traffic / t_launch / 1e9
        d["achieved_measured_bytes"] = m
        d["frac_measured_bytes"] = m / HBM_PEAK_GBS
    d.update(extra)
    return d


def _sample_iterations(run, cap: int, target_s: float) -> int:
    """Iterations of a fixed-work oracle run that take about target_s seconds
    (per-iteration cost from a 2- and a 6-iteration run)."""
    t0 = time.perf_counter()
    run(2)
    t1 = time.perf_counter()
    run(6)
    t2 = time.perf_counter()
    per_it = max((t2 - t1) - (t1 - t0), 1e-6) / 4.0
    return max(3, min(cap, int(target_s / per_it)))


def measured_copy_gbs(reps: int = 5) -> dict:
    """Bandwidth of a plain device copy of 1 GiB (read + write bytes / time),
    the achievable-peak reference next to the 8 TB/s specification: the
    library's own streaming copy kernel (cg_hbm_copy) and torch's copy."""
    import torch
    from paper_2608_09647_amd import cgmi
    a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, copy in (("library", lambda: cgmi.hbm_copy(a, b)), ("torch", lambda: b.copy_(a))):
        copy()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            copy()
        e1.record()
        torch.cuda.synchronize()
        out[name] = 2 * a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    assert torch.equal(a, b)
    del a, b
    torch.cuda.empty_cache()
    return out


def host_info() -> dict:
    """CPU model of the host and a single-thread numpy triad rate, the context
    next to the oracle's timing."""
    import numpy as np
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = 1 << 25
    bv, cv = np.ones(n), np.ones(n)
    av = np.empty(n)
    best = float("inf")
    for _ in range(3):
        t0 = time.perf_counter()
        np.multiply(cv, 3.0, out=av)
        np.add(av, bv, out=av)
        best = min(best, time.perf_counter() - t0)
    # a = b + 3 c as two numpy passes: 5 vectors of traffic
    return {"cpu_model": model, "logical_cpus": os.cpu_count(),
            "numpy_triad_gbs_one_thread": 5 * 8 * n / best / 1e9}


def cpu_baseline_cg(problem, iters_hint: int, target_s: float = 12.0) -> dict:
    """The oracle's CG, untouched, on a bounded sample: a fixed number of CG
    iterations of the same system, all host threads for its row loops."""
    import oracle
    k = _sample_iterations(lambda m: oracle.cg(problem.A, problem.b, tol=0.0, maxit=m), iters_hint,
                           target_s)
    t0 = time.perf_counter()
    out = oracle.cg(problem.A, problem.b, tol=0.0, maxit=k)
    dt = time.perf_counter() - t0
    return {"value": out["iterations"] / dt, "unit": "iter/s", "cores": oracle.max_threads(),
            "kind": "oracle", "host": host_info(),
            "sample": f"{out['iterations']} fixed-work CG iterations of the same system "
                      f"({dt:.1f} s, including its setup residual and final true residual)"}


def _timed_solve(solver, b, x0, tol, maxit, reps, ktimes=None):
    """ktimes: when a list, the event-timed seconds of each solve's one
    launch (single-workgroup path with cg_opts.profile) are appended."""
    import torch
    times, res = [], None
    x = x0.clone()            # returned as is when reps = 0 (no warmup)
    for _ in range(reps):
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, res = solver.solve(b, x, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if ktimes is not None and res["n_spmv"] == 1:
            ktimes.append(res["t_spmv"])
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
    from paper_2608_09647_amd import autotune
    for name, opts in variants.items():
        solver = cgmi.Solver(prob.A)
        autotune.spmv_schedule(solver, prob.A, b, tune_if_missing=False)   # tabled SpMV tiling, if any
        solver.set_opts(**opts)
        _timed_solve(solver, b, x0, 1e-10, 200000, args.warmup)
        ktimes = []
        x, res, times = _timed_solve(solver, b, x0, 1e-10, 200000, args.steps, ktimes)
        xs[name] = x.cpu().numpy()
        out[name] = {"seconds": float(np.mean(times)), "min_seconds": float(np.min(times)),
                     "iterations": res["iterations"], "fp64_residuals": res["fp64_residuals"],
                     "rel_res_true": res["rel_res_true"], "status": res["code"],
                     "fell_back": res["fell_back"]}
        if ktimes:
            out[name]["kernel_seconds"] = float(np.mean(ktimes))
        solver.close()
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)
    return out, xs


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the paper's protocol: 3 warm-up passes, then 10 measured passes (Section 4.1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="poisson3d_256",
                    choices=["poisson3d_256", "poisson3d_256_split", "poisson2d_64", "random_spd_2m",
                             "diffusion_1024", "batch_256", "split_sweep", "matrix_market"])
    ap.add_argument("--mtx", default=None, help="Matrix Market file of the matrix_market config")
    ap.add_argument("--share", type=float, default=0.5, help="GPU row share for the split config")
    ap.add_argument("--sweep-matrix", default="poisson3d_256", choices=["poisson3d_256", "random_spd_2m"],
                    help="system of the split_sweep config")
    ap.add_argument("--by-nnz", action="store_true",
                    help="split_sweep: place the split at a share of the nonzeros instead of the rows")
    ap.add_argument("--iters", type=int, default=500, help="fixed CG iterations per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--train-steps", type=int, default=2000, help="learned-FSAI training steps")
    ap.add_argument("--train-fields", type=int, default=2000, help="128x128 training fields")
    ap.add_argument("--batch-iters", type=int, default=30, help="fixed iterations per batched step")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the timed path of the workload (no comparison solves), for profilers")
    ap.add_argument("--spmv-kind", type=int, default=None,
                    help="default workload: force this SpMV tiling (cg_opts.spmv_kind) instead of the "
                         "tabled one, e.g. 3 for the generic sliced CSR tiling")
    ap.add_argument("--fuse-dir", type=int, default=0, choices=[0, 1, 2],
                    help="cg_opts.fuse_dir: automatic (0), the direction update inside the next SpMV (1) or in "
                         "separate kernels (2)")
    ap.add_argument("--batch-launch", default="cooperative", choices=["cooperative", "ordinary"],
                    help="launch form of the batched kernel (ordinary: for profilers that cannot "
                         "follow cooperative launches)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X "
              "(sharding rows across GPUs is a design, not a measured path).", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2608_09647_amd import inputs as I
    from paper_2608_09647_amd import cgmi

    if args.config == "random_spd_2m":
        return bench_mixed(args)
    if args.config == "diffusion_1024":
        return bench_learned(args)
    if args.config == "batch_256":
        return bench_batch(args)
    if args.config == "poisson2d_64":
        return bench_small(args)
    if args.config == "poisson3d_256_split":
        return bench_split(args)
    if args.config == "split_sweep":
        return bench_split_sweep(args)
    if args.config == "matrix_market":
        return bench_matrix_market(args)
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
    from paper_2608_09647_amd import autotune
    if args.spmv_kind is None:
        autotune.spmv_schedule(solver, A, b, tune_if_missing=False)   # tabled SpMV tiling, if any
    else:
        solver.set_opts(spmv_kind=args.spmv_kind)
    # HIP events around the SpMV of every SPMV_EVENT_STRIDE-th iteration of
    # the timed steps (an event pair adds a few microseconds of stream time)
    solver.set_opts(profile=SPMV_EVENT_STRIDE, fuse_dir=args.fuse_dir)
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
    step_s = []
    for _ in range(args.steps):
        x.zero_()
        ts = time.perf_counter()
        _, res = solver.solve(b, x, tol=0.0, maxit=args.iters)   # blocking
        step_s.append(time.perf_counter() - ts)
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
    copies = measured_copy_gbs()
    copy_gbs = copies["library"]
    line = {
        "metric": "CG iters/s + SpMV GB/s (%HBM peak); time to 1e-10 residual, plain vs learned-PC",
        "value": iters / elapsed,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "ms_per_step_min": 1e3 * min(step_s),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson3d_7pt_256^3_fp64_cg_fixed_work", "n": A.n, "nnz": A.nnz,
                   "spmv_kind_forced": args.spmv_kind,
                   "iterations_per_step": args.iters, "row_share_gpu": 1.0, "index": "int32",
                   "seed": 2},
        "spmv_gbs": achieved,
        "spmv_us": 1e6 * t_launch,
        "spmv_timed_launches": {"count": n_spmv, "every_nth_iteration": SPMV_EVENT_STRIDE},
        "hbm_copy_gbs_measured": copy_gbs,
        "hbm_copy_gbs": copies,
        "spmv_frac_of_measured_copy": achieved / copy_gbs,
        "spmv_kind": {1: "vector_bins", 2: "stream", 3: "sliced", 4: "sliced_dict",
                      5: "column_blocks", 6: "stencil_slices", 7: "gap_slices"}.get(res["spmv_kind"]),
        "rel_res_true": res["rel_res_true"],
        "roofline": roofline_hbm(spmv_bytes, t_launch,
                                 measured_traffic("spmv_poisson3d_256" + (
                                     "" if res["spmv_kind"] == 6 else f"_kind{res['spmv_kind']}"),
                                     res["spmv_kind"]),
                                 kernel="k_spmv (dot mode)"),
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


def profiled_spmv_us(prob, opts: dict) -> float:
    """Mean SpMV time of one solve to 1e-10 with HIP events around every SpMV
    (a separate solve, so the events stay out of the timed ones)."""
    import torch
    from paper_2608_09647_amd import autotune, cgmi
    b = torch.from_numpy(prob.b).to(torch.device("cuda:0"))
    with cgmi.Solver(prob.A) as s:
        autotune.spmv_schedule(s, prob.A, b, tune_if_missing=False)
        s.set_opts(profile=1, **opts)
        _, res = s.solve(b, torch.zeros_like(b), tol=1e-10, maxit=200000)
        torch.cuda.synchronize()
    return 1e6 * res["t_spmv"] / max(res["n_spmv"], 1)


def spmv_algorithmic_bytes_f32(n: int, nnz: int) -> int:
    """Float32 CSR SpMV: 4-byte columns and values, row pointers, q written
    and p read once (4 bytes each)."""
    return 8 * nnz + 4 * (n + 1) + 8 * n


def cpu_baseline_mixed(prob, iterations: int, target_s: float = 12.0) -> dict:
    """The oracle's float32-inner CG with float64 refinement, fixed work on a
    bounded number of inner iterations, scaled to the GPU solve's count."""
    import oracle
    k = _sample_iterations(lambda m: oracle.cg_mixed(prob.A, prob.b, tol=0.0, maxit=m), iterations,
                           target_s)
    t0 = time.perf_counter()
    out = oracle.cg_mixed(prob.A, prob.b, tol=0.0, maxit=k)
    dt = time.perf_counter() - t0
    per_it = dt / max(out["iterations"], 1)
    return {"value": per_it * iterations, "unit": "s", "cores": oracle.max_threads(), "kind": "oracle",
            "host": host_info(),
            "sample": f"{out['iterations']} fixed-work float32-inner iterations of the oracle's mixed "
                      f"CG ({dt:.1f} s), scaled to the {iterations} iterations of the GPU solve"}


def gather_ceiling(count: int, reps: int = 5) -> dict:
    """The library's plain random gather (cg_gather) of `count` float64 values
    with uniformly random int32 indices, from a vector of one column block
    (262,144 values, 2 MB: held in each XCD's L2) and from the whole 2M
    vector (16 MB: held in the last-level cache): gathers per second
    (median of `reps` launches, HIP events on torch's stream)."""
    import torch
    from paper_2608_09647_amd import cgmi
    out = {}
    g = torch.Generator(device="cuda").manual_seed(17)
    dst = torch.empty(count, dtype=torch.float64, device="cuda")
    for name, size in (("l2_2MB", 262_144), ("llc_16MB", 2_000_000)):
        src = torch.rand(size, dtype=torch.float64, device="cuda")
        idx = torch.randint(0, size, (count,), dtype=torch.int32, device="cuda", generator=g)
        cgmi.gather(src, idx, dst)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            cgmi.gather(src, idx, dst)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        t = sorted(ts)[len(ts) // 2]
        out[name] = {"vector_bytes": 8 * size, "gathers": count, "seconds": t, "gathers_per_s": count / t,
                     "bytes_per_s_idx_dst_gathered": 20 * count / t}
        del src, idx
    return out


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
    # the mixed solve's dominant kernel is its float32 SpMV (column blocks)
    us32 = profiled_spmv_us(prob, {"precision": 1})
    us64 = profiled_spmv_us(prob, {})
    n, nnz = prob.A.n, prob.A.nnz
    a32 = spmv_algorithmic_bytes_f32(n, nnz) / (us32 * 1e-6) / 1e9
    a64 = spmv_algorithmic_bytes(n, nnz) / (us64 * 1e-6) / 1e9
    # the ceiling for SpMVs bound by random gathers: one column block's
    # gathers from an L2-resident segment, scaled to the SpMV's nnz gathers
    gc = gather_ceiling(nnz // 8)
    t_g = nnz / gc["l2_2MB"]["gathers_per_s"]
    print(f"[bench] gather ceiling {gc}", file=sys.stderr, flush=True)
    line = _line("time to 1e-10 true relative residual: float32-inner/float64-refined CG "
                 "vs plain float64 CG", out["mixed"]["seconds"], "s", args,
                 1e3 * out["mixed"]["seconds"],
                 {"workload": "random_spd_lognormal_n2M_mixed_vs_fp64", "n": n,
                  "nnz": nnz, "tol": 1e-10, "seed": 3}, higher=False,
                 plain_fp64=out["fp64"], mixed=out["mixed"], speedup_vs_fp64=sp,
                 mixed_rel_error_vs_fp64_solution=err,
                 spmv_us={"float32": us32, "float64": us64},
                 spmv_gbs={"float32": a32, "float64": a64},
                 gather_ceiling=gc,
                 spmv_frac_of_gather_ceiling={"float64": 1e6 * t_g / us64, "float32": 1e6 * t_g / us32,
                                              "meaning": "time of the library's plain gather of nnz "
                                                         "values from a 2 MB vector / SpMV time"},
                 roofline=roofline_hbm(spmv_algorithmic_bytes_f32(n, nnz), us32 * 1e-6,
                                       measured_traffic("spmv_random_spd_2m_f32", 5),
                                       kernel="float32 column-blocked SpMV (start, 8 passes, finish)",
                                       note="CSR-algorithmic bytes (8 nnz + 4 (n+1) + 8 n) per SpMV; its "
                                            "uniformly random columns make it bound by L2 gathers: see "
                                            "spmv_frac_of_gather_ceiling"),
                 traffic_fp64_spmv=measured_traffic("spmv_random_spd_2m_f64", 5))
    line["dtype"] = "f32+f64"
    line["rel_error_vs_xstar"] = {k: float(np.linalg.norm(xs[k] - prob.xstar) / np.linalg.norm(prob.xstar))
                                  for k in ("fp64", "mixed")}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_mixed(prob, out["mixed"]["iterations"])
        # each GPU solution against the float64 oracle's solution of the same system
        import oracle
        t0 = time.perf_counter()
        ref = oracle.cg(prob.A, prob.b, tol=1e-10, maxit=200000)
        dt = time.perf_counter() - t0
        nref = float(np.linalg.norm(ref["x"]))
        line["oracle_fp64"] = {"seconds": dt, "iterations": ref["iterations"],
                               "rel_error": {k: float(np.linalg.norm(xs[k] - ref["x"]) / nref)
                                             for k in ("fp64", "mixed")}}
    print(json.dumps(line), flush=True)
    return 0


def bench_small(args) -> int:
    """2D Poisson 64x64 to 1e-10, all rows on the GPU (single-workgroup path)."""
    from paper_2608_09647_amd import inputs as I
    prob = I.poisson2d_problem(64, seed=1)
    # the third variant repeats the first with an event pair around its
    # launch (kept out of the headline solves, where it would add stream time)
    out, _ = bench_time_to_tol(args, prob, {"small_path": {"small_path": 1},
                                            "multi_kernel": {"small_path": 0},
                                            "small_path_events": {"small_path": 1, "profile": 1}},
                               None, None)
    best = out["small_path"]
    # Roofline of the one launch: the solve is a single workgroup on one
    # compute unit, with A in registers and p in LDS, so no HBM or chip-wide
    # figure bounds it; it is priced against that unit's float64 vector rate
    # (78.6 TFLOP/s over 256 CUs).  Algorithmic flops per iteration: the
    # SpMV's 2 nnz, two dot products and three vector updates of 2 n each.
    flops_it = 2 * prob.A.nnz + 10 * prob.A.n
    cu_peak = FP64_VECTOR_PEAK_TFLOPS / N_CUS
    ev = out["small_path_events"]
    ks = ev.get("kernel_seconds")
    ach = flops_it * ev["iterations"] / ks / 1e12 if ks else None
    line = _line("CG iterations/s to 1e-10 (2D Poisson 64x64)",
                 best["iterations"] / best["seconds"], "iter/s", args, 1e3 * best["seconds"],
                 {"workload": "poisson2d_5pt_64x64_fp64_cg_to_1e-10", "n": prob.A.n,
                  "nnz": prob.A.nnz, "seed": 1},
                 roofline={"bound": "alu", "achieved": ach, "peak": cu_peak, "unit": "TFLOP/s",
                           "frac": ach / cu_peak if ach else None, "traffic": None,
                           "kernel": "k_cg_small (one launch per solve)", "launch_us": 1e6 * ks if ks else None,
                           "flops_per_iteration": flops_it,
                           "scope": "one compute unit: the whole solve is one workgroup",
                           "note": "latency-bound: three workgroup barriers, two 16-term serial sums "
                                   "and two float64 divisions per iteration"},
                 paths=out)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_repeat(prob)
    print(json.dumps(line), flush=True)
    return 0


def cpu_baseline_repeat(prob, target_s: float = 10.0) -> dict:
    """The oracle's CG to 1e-10 on the same small system, repeated for about
    target_s seconds (one solve takes milliseconds)."""
    import oracle
    its, solves = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < target_s:
        its += oracle.cg(prob.A, prob.b, tol=1e-10, maxit=20000)["iterations"]
        solves += 1
    dt = time.perf_counter() - t0
    return {"value": its / dt, "unit": "iter/s", "cores": oracle.max_threads(), "kind": "oracle",
            "host": host_info(),
            "sample": f"{solves} oracle solves to 1e-10 of the same system ({its} iterations, {dt:.1f} s)"}


SPLIT_MODES = (("whole", 0), ("halo", 1), ("mapped", 2), ("managed", 3))


def _split_run(cgmi, s, b, iters, warmup, steps, exchange):
    """Fixed-work split solves in one memory mode; None when the mode is not
    available on this device (the library's error message instead)."""
    import numpy as np
    import torch
    try:
        s.set_opts(exchange=exchange)
    except cgmi.CgError as e:
        return {"unavailable": str(e)}
    _timed_solve(s, b, torch.zeros_like(b), 0.0, iters, max(1, warmup))
    _, res, times = _timed_solve(s, b, torch.zeros_like(b), 0.0, iters, steps)
    sec = float(np.mean(times))
    return {"seconds": sec, "seconds_per_iter": sec / iters, "iter_per_s": iters / sec,
            **{k: res[k] for k in ("iterations", "t_gpu", "t_cpu", "t_barrier", "t_d2h", "t_h2d",
                                    "rows_gpu", "rows_cpu", "nnz_gpu", "nnz_cpu")}}


def bench_split(args) -> int:
    """256^3 Poisson with the GPU owning the first share of rows and host
    threads the rest; p made visible by each memory mode of Section 3.4
    (explicit copy of whole segments or of the halo, mapped host memory,
    managed memory where the device supports it)."""
    import numpy as np
    import torch
    from paper_2608_09647_amd import inputs as I, cgmi, split
    prob = I.poisson3d_problem(256, seed=2)
    n = prob.A.n
    n_gpu = split.rows_for_share(n, args.share)
    iters = min(args.iters, 50)
    b = torch.from_numpy(prob.b).cuda()
    res_all = {}
    with cgmi.Solver(prob.A, 0, n_gpu) as s:
        for name, ex in SPLIT_MODES:
            res_all[name] = _split_run(cgmi, s, b, iters, args.warmup, args.steps, ex)
            print(f"[bench] split {name}: {res_all[name]}", file=sys.stderr, flush=True)
    ran = {k: v for k, v in res_all.items() if "seconds" in v}
    best = max(ran.values(), key=lambda r: r["iter_per_s"])
    line = _line("CG iters/s, split rows (GPU share + host complement, p made visible each iteration)",
                 best["iter_per_s"], "iter/s", args, 1e3 * best["seconds"],
                 {"workload": f"poisson3d_7pt_256^3_fp64_cg_split_g{args.share}",
                  "n": n, "nnz": prob.A.nnz, "iterations_per_step": iters,
                  "row_share_gpu": args.share}, exchange=res_all,
                 best_mode=max(ran, key=lambda k: ran[k]["iter_per_s"]))
    print(json.dumps(line), flush=True)
    return 0


def bench_split_sweep(args) -> int:
    """The paper's protocol on one synthetic system: every GPU row share of
    the sweep under every memory mode (Section 4.1), fixed work, the 1.25x
    competitive classification, and the planner's automatic choice fitted
    from the g = 0.5 runs alone, checked against the sweep."""
    import numpy as np
    import torch
    from paper_2608_09647_amd import inputs as I, cgmi, split
    if args.sweep_matrix == "random_spd_2m":
        prob = I.random_spd_problem(2_000_000, seed=3)
    else:
        prob = I.poisson3d_problem(256, seed=2)
    A, n = prob.A, prob.A.n
    iters = min(args.iters, 30)
    steps = max(1, min(args.steps, 2))
    b = torch.from_numpy(prob.b).cuda()
    rows_fn = (lambda g: split.rows_for_nnz_share(A.row_ptr, g)) if args.by_nnz else \
        (lambda g: split.rows_for_share(n, g))
    managed_ok = None
    sweep = {}
    for g in split.SHARES:
        rows = rows_fn(g)
        if rows == 0:
            modes = (("host", 0),)
        elif rows == n:
            modes = (("device", 0), ("mapped", 2), ("managed", 3))
        else:
            modes = SPLIT_MODES
        with cgmi.Solver(A, 0, rows) as s:
            s.set_opts(host_threads=0)
            for name, ex in modes:
                if name == "managed" and managed_ok is False:
                    continue
                r = _split_run(cgmi, s, b, iters, 1, steps, ex)
                if name == "managed" and managed_ok is None:
                    managed_ok = "seconds" in r
                if "seconds" in r:
                    sweep[f"g{g:.2f}/{name}"] = {"share": g, "mode": name, **r}
                    print(f"[bench] sweep g={g:.2f} {name}: {1e3 * r['seconds_per_iter']:.2f} ms/iter",
                          file=sys.stderr, flush=True)
    times = {k: v["seconds_per_iter"] for k, v in sweep.items()}
    flags = split.competitive(times)
    for k in sweep:
        sweep[k]["competitive"] = flags[k]
    best_key = min(times, key=times.get)
    # planner: models fitted from the g = 0.5 runs only
    models = {}
    for name, _ in SPLIT_MODES:
        r = sweep.get(f"g0.50/{name}")
        if r is not None:
            models[name] = split.IterationModel.fit(r, r["seconds"], A.nnz)
    choice = split.choose_config(models, A.row_ptr, by_nnz=args.by_nnz)
    g_c = choice["share"]
    mode_c = choice["mode"]
    if g_c == 0.0:
        key_c = "g0.00/host"
    elif g_c == 1.0:
        key_c = f"g1.00/{'mapped' if mode_c in ('mapped', 'managed') else 'device'}"
    else:
        key_c = f"g{g_c:.2f}/{mode_c}"
    measured_c = times.get(key_c)
    auto = {"mode": mode_c, "share": g_c, "rows_gpu": choice["rows_gpu"],
            "predicted_seconds_per_iter": choice["predicted"], "measured_key": key_c,
            "measured_seconds_per_iter": measured_c,
            "ratio_to_best": None if measured_c is None else measured_c / times[best_key],
            "competitive": None if measured_c is None else flags[key_c],
            "models": {m: vars(md) for m, md in models.items()}}
    print(f"[bench] best {best_key}; planner chose {key_c} ({auto['ratio_to_best']})", file=sys.stderr,
          flush=True)
    # interconnect bound (Section 4.4) over the explicit-copy configurations
    explicit = {k: v for k, v in sweep.items() if v["mode"] in ("host", "device", "whole", "halo")}
    tb = split.transfer_bound_table(explicit)
    line = _line("CG iters/s, best configuration of the GPU-share x memory-mode sweep",
                 1.0 / times[best_key], "iter/s", args, 1e3 * iters * times[best_key],
                 {"workload": f"{prob.name}_split_sweep", "n": n, "nnz": A.nnz,
                  "iterations_per_solve": iters, "shares": list(split.SHARES),
                  "split_by": "nnz" if args.by_nnz else "rows"},
                 best=best_key, managed_supported=bool(managed_ok), sweep=sweep, planner=auto,
                 transfer_bound=tb)
    print(json.dumps(line), flush=True)
    return 0


def bench_matrix_market(args) -> int:
    """A user's matrix from a Matrix Market file (read by the library's
    reader, symmetric storage expanded): x* ~ U[-1,1] (seed 0), b = A x*,
    float64 CG on the GPU, a fixed-work run (--iters) timed over --steps and
    one solve to 1e-10."""
    import numpy as np
    import torch
    from paper_2608_09647_amd import cgmi, inputs as I
    if not args.mtx:
        print("--config matrix_market needs --mtx PATH", file=sys.stderr)
        return 2
    t0 = time.perf_counter()
    A, info = cgmi.read_matrix_market(args.mtx)
    t_read = time.perf_counter() - t0
    print(f"[bench] read {args.mtx}: n={A.n} nnz={A.nnz} in {t_read:.2f}s", file=sys.stderr, flush=True)
    xs = I.uniform_vector(A.n, [0, 1])
    b = torch.from_numpy(I.rhs_of(A, xs)).cuda()
    with cgmi.Solver(A) as s:
        s.set_opts(profile=1)
        _timed_solve(s, b, torch.zeros_like(b), 0.0, args.iters, max(1, args.warmup))
        _, res, times = _timed_solve(s, b, torch.zeros_like(b), 0.0, args.iters, args.steps)
        spmv_us = 1e6 * res["t_spmv"] / max(res["n_spmv"], 1)
        s.set_opts(profile=0)
        x, res_tol, t_tol = _timed_solve(s, b, torch.zeros_like(b), 1e-10, 200000, 1)
    sec = float(np.mean(times))
    gbs = spmv_algorithmic_bytes(A.n, A.nnz) / (spmv_us * 1e-6) / 1e9
    err = float(np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs))
    kinds = {1: "vector_bins", 2: "stream", 3: "sliced", 4: "sliced_dict", 5: "column_blocks",
             6: "stencil_slices", 7: "gap_slices"}
    line = _line("CG iters/s on a Matrix Market matrix (fixed work); time to 1e-10", res["iterations"] / sec,
                 "iter/s", args, 1e3 * sec,
                 {"workload": f"matrix_market:{os.path.basename(args.mtx)}", "n": A.n, "nnz": A.nnz,
                  "symmetric_file": info["symmetric"], "iterations_per_step": args.iters},
                 read_seconds=t_read, spmv_us=spmv_us, spmv_gbs=gbs, spmv_kind=kinds.get(res["spmv_kind"]),
                 roofline={"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": gbs / HBM_PEAK_GBS, "traffic": None},
                 to_tolerance={"seconds": t_tol[0], "iterations": res_tol["iterations"],
                               "status": res_tol["code"], "rel_res_true": res_tol["rel_res_true"],
                               "rel_err_vs_xstar": err})
    print(json.dumps(line), flush=True)
    return 0


def _training_fields(count: int, nx: int = 128):
    """Seeded training operators, generated in worker processes (host only)."""
    from concurrent.futures import ProcessPoolExecutor
    from paper_2608_09647_amd import inputs as I
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(I.training_field, range(count), [nx] * count, chunksize=16))


def bench_learned(args) -> int:
    """1024^2 log-normal diffusion: plain float64 CG vs PCG with the learned
    FSAI factor, both to 1e-10; the network is first trained on the GPU on
    128^2 fields (seeds 0..train_fields-1).  The learned time includes the
    factor's setup on the device (features, inference, assembly of G and G^T;
    the first setup also builds the factor's structure on the host)."""
    import numpy as np
    import scipy.sparse as sp
    import torch
    from paper_2608_09647_amd import cgmi, fsai, inputs as I

    t0 = time.perf_counter()
    systems = _training_fields(args.train_fields)
    t_gen = time.perf_counter() - t0
    print(f"[bench] {len(systems)} training fields in {t_gen:.1f}s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    tr = cgmi.FsaiTrainer(systems, fsai.init_params(0))
    t_upload = time.perf_counter() - t0
    hist = fsai.train(tr, steps=args.train_steps, nsel=8, rows_per=1024, lr=1e-3, lr_final=1e-4,
                      seed=0, log=lambda s: print(f"[bench] train {s}", file=sys.stderr, flush=True))
    theta = tr.params()
    tr.close()
    del systems
    train = {"fields": args.train_fields, "field_side": 128, "steps": hist["steps"],
             "fields_per_step": hist["nsel"], "rows_per_field": hist["rows_per"],
             "seconds": hist["seconds"], "upload_seconds": t_upload, "generate_seconds": t_gen,
             "loss_first10": float(np.mean(hist["losses"][:10])),
             "loss_last10": float(np.mean(hist["losses"][-10:]))}

    prob = I.diffusion_problem(1024, seed=10_000)
    A = prob.A
    print(f"[bench] {prob.name} n={A.n} nnz={A.nnz} contrast={prob.meta['k_max'] / prob.meta['k_min']:.3g}",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    b = torch.from_numpy(prob.b).to(dev)
    x0 = torch.zeros_like(b)
    out = {}

    from paper_2608_09647_amd import autotune

    def run(name, prepare, reps, warm, precond=cgmi.PC_NONE, profiled=False):
        s = cgmi.Solver(A)
        autotune.spmv_schedule(s, A, b, tune_if_missing=False)   # tabled SpMV tiling, if any
        # timed solves without per-SpMV events; the SpMV time comes from one
        # more (profiled) solve where it is needed
        s.set_opts(profile=0, precond=precond, fuse_dir=args.fuse_dir)
        times, setups = [], []
        res = None
        spmv_us = None
        for k in range(warm + reps):
            x = x0.clone()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            prepare(s, k)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            _, res = s.solve(b, x, tol=1e-10, maxit=500_000)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            if k >= warm:
                setups.append(t2 - t1)
                times.append(t3 - t2)
        err = float(np.linalg.norm(x.cpu().numpy() - prob.xstar) / np.linalg.norm(prob.xstar))
        if profiled:
            s.set_opts(profile=1, precond=precond)
            _, pres = s.solve(b, x0.clone(), tol=1e-10, maxit=500_000)
            torch.cuda.synchronize()
            spmv_us = 1e6 * pres["t_spmv"] / max(pres["n_spmv"], 1)
        s.close()
        out[name] = {"seconds": float(np.mean(times)) + float(np.mean(setups)),
                     "solve_seconds": float(np.mean(times)), "setup_seconds": float(np.mean(setups)),
                     "iterations": res["iterations"], "status": res["code"], "fell_back": res["fell_back"],
                     "rel_res_true": res["rel_res_true"], "rel_err_vs_xstar": err,
                     "fused_dir": res["fused_dir"]}
        if spmv_us is not None:
            out[name]["spmv_us"] = spmv_us
            out[name]["spmv_launches_timed"] = pres["n_spmv"]
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)

    def plain(s, k):
        pass

    def learned(s, k):
        s.fsai_setup(theta)

    def untrained(s, k):
        s.fsai_setup(fsai.init_params(0))

    d = A.scipy().diagonal()
    J = sp.diags(1.0 / np.sqrt(d)).tocsr()

    def jacobi(s, k):
        s.set_fsai(J)

    def classic(s, k):
        s.fsai_classic()

    # learned: a fresh handle per repetition would re-upload A; instead the
    # first (cold) setup of a fresh handle is timed separately (median of
    # three handles) and each timed repetition re-runs the device setup with
    # the same parameters
    colds = []
    for _ in range(3):
        s = cgmi.Solver(A)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.fsai_setup(theta)
        torch.cuda.synchronize()
        colds.append(time.perf_counter() - t1)
        s.close()
    cold_setup = float(np.median(colds))
    if args.profile_run:
        run("learned", learned, args.steps, args.warmup, cgmi.PC_FSAI, profiled=True)
        print(json.dumps({"profile_run": "diffusion_1024", "learned": out["learned"]}), flush=True)
        return 0
    run("plain", plain, min(args.steps, 3), min(args.warmup, 1))   # ~6 s per plain solve
    run("learned", learned, args.steps, args.warmup, cgmi.PC_FSAI, profiled=True)
    out["learned"]["cold_setup_seconds"] = cold_setup
    out["learned"]["seconds_with_cold_setup"] = out["learned"]["solve_seconds"] + cold_setup
    run("jacobi", jacobi, 1, 0, cgmi.PC_FSAI)
    run("untrained", untrained, 1, 0, cgmi.PC_FSAI)
    run("classic_fsai", classic, 1, 0, cgmi.PC_FSAI)
    spmv_bytes = spmv_algorithmic_bytes(A.n, A.nnz)
    kernel = "k_spmv (dot mode), A p"
    if out["learned"]["fused_dir"]:
        # iteration 0's SpMV alone; every later launch also reads z, writes
        # p_{k+1} and reads and writes x (the direction update it carries)
        nl = max(out["learned"]["spmv_launches_timed"], 1)
        spmv_bytes += 32 * A.n * (nl - 1) / nl
        kernel = "k_spmv_dir (A p with the direction update, z and x)"
    t_spmv = out["learned"]["spmv_us"] * 1e-6
    achieved = spmv_bytes / t_spmv / 1e9
    traffic = measured_traffic("pcg_learned_diffusion_1024", 6) if out["learned"]["fused_dir"] else None
    line = _line("CG iters/s + SpMV GB/s (%HBM peak); time to 1e-10 residual, plain vs learned-PC",
                 out["learned"]["seconds_with_cold_setup"], "s", args,
                 1e3 * out["learned"]["seconds_with_cold_setup"],
                 {"workload": "diffusion2d_5pt_1024^2_lognormal_learned_fsai_vs_plain_cg_to_1e-10",
                  "n": A.n, "nnz": A.nnz, "tol": 1e-10, "seed": 10_000,
                  "contrast": prob.meta["k_max"] / prob.meta["k_min"]},
                 higher=False, plain=out["plain"], learned=out["learned"], jacobi=out["jacobi"],
                 untrained=out["untrained"], classic_fsai=out["classic_fsai"], training=train,
                 speedup_vs_plain=out["plain"]["seconds"] / out["learned"]["seconds_with_cold_setup"],
                 roofline={"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
                           "algorithmic_bytes_per_launch": int(spmv_bytes),
                           **({"achieved_measured_bytes": traffic / t_spmv / 1e9,
                               "frac_measured_bytes": traffic / t_spmv / 1e9 / HBM_PEAK_GBS} if traffic else {}),
                           "note": "A, G, G^T and the vectors (~200 MB) fit the 256 MB last-level "
                                   "cache, so the HBM roofline does not bound this SpMV; traffic counts "
                                   "the bytes fetched and written past the L2, from that cache or HBM"})
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_pcg(prob, theta, out["learned"]["iterations"])
    print(json.dumps(line), flush=True)
    return 0


def batch_algorithmic_bytes(n_total: int, nnz_total: int, nrhs: int) -> int:
    """Per batched iteration: the matrix once (int32 col + float64 val per
    nonzero, row pointers) and six float64 vector passes per right-hand side
    and row (p gathered, q written, x and r read and written)."""
    return 12 * nnz_total + 4 * (n_total + 1) + 8 * 6 * nrhs * n_total


def bench_batch(args) -> int:
    """256 uneven 2-D diffusion systems (sides 32..512) x 16 right-hand sides:
    fixed-work throughput of the one-launch batched solve (schedule from the
    autotuner table, or tuned here), against one cg_solve per (system,
    right-hand side); plus a to-1e-10 comparison on the sub-batch of systems
    with side <= 64, where every pair's separate solve is timed."""
    import numpy as np
    import torch
    from paper_2608_09647_amd import autotune, cgmi, inputs as I

    t0 = time.perf_counter()
    probs = I.batch_problem(256, 16, seed=5)
    systems = [p.A for p in probs]
    n_total = sum(A.n for A in systems)
    nnz_total = sum(A.nnz for A in systems)
    print(f"[bench] batch of {len(systems)} systems, n_total={n_total}, nnz={nnz_total} "
          f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)
    B = torch.from_numpy(np.ascontiguousarray(np.concatenate([p.b for p in probs], axis=0))).cuda()
    X = torch.zeros_like(B)
    batch = cgmi.Batch(systems, 16)
    sched = autotune.batch_schedule(batch, systems, B, store=False,
                                    log=lambda s: print(f"[bench] tune {s}", file=sys.stderr, flush=True))
    if args.batch_launch == "ordinary":
        batch.set_sched(launch=cgmi.BATCH_LAUNCH_ORDINARY)
        sched = {"sched": batch.sched.as_dict(), "source": sched["source"]}
    print(f"[bench] schedule {sched}", file=sys.stderr, flush=True)
    K = args.batch_iters
    for _ in range(args.warmup):
        X.zero_()
        batch.solve(B, X, tol=0.0, maxit=K)
    torch.cuda.synchronize()
    t_kernel = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        X.zero_()
        _, res, st, _ = batch.solve(B, X, tol=0.0, maxit=K)
        t_kernel.append(st["t_kernel"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert np.all(res["iterations"] == K)
    pairs = len(systems) * 16
    value = pairs * K * args.steps / elapsed
    bytes_it = batch_algorithmic_bytes(n_total, nnz_total, 16)
    t_k = float(np.mean(t_kernel))
    print(f"[bench] batched: {args.steps} x {K} iterations in {elapsed:.3f}s, stats {st}",
          file=sys.stderr, flush=True)
    batch.close()
    del X
    if args.profile_run:
        print(json.dumps({"profile_run": "batch_256", "pair_iterations_per_s": value,
                          "kernel_seconds": t_k, "stats": st, "launch": args.batch_launch}), flush=True)
        return 0

    # one cg_solve per (system, right-hand side), every pair timed at the
    # same fixed work (K iterations), device-resident vectors
    t_all, per_sys = 0.0, []
    for k, A in enumerate(systems):
        s = cgmi.Solver(A)
        bk = torch.from_numpy(np.ascontiguousarray(probs[k].b.T)).cuda()   # 16 x n
        xk = torch.zeros_like(bk[0])
        s.solve(bk[0], xk, tol=0.0, maxit=K)                                 # warm: first-use setup
        t_k_sys = 0.0
        for j in range(16):
            xk.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, r1 = s.solve(bk[j], xk, tol=0.0, maxit=K)
            torch.cuda.synchronize()
            t_k_sys += time.perf_counter() - t1
            assert r1["iterations"] == K
        s.close()
        per_sys.append(t_k_sys)
        t_all += t_k_sys
    single = {"measured_seconds_all_pairs": t_all, "pairs": pairs, "iterations_per_pair": K,
              "pair_iterations_per_s": pairs * K / t_all,
              "seconds_largest_system_16_pairs": float(max(per_sys)),
              "seconds_smallest_system_16_pairs": float(min(per_sys))}
    print(f"[bench] one cg_solve per pair, all {pairs} pairs timed: {t_all:.3f}s", file=sys.stderr, flush=True)

    # to tolerance on the small-system sub-batch, every pair's solve timed,
    # repeated `steps` times (batched and separate alternating)
    small = [k for k in range(len(systems)) if probs[k].meta["side"] <= 64]
    tol_cmp = None
    if small:
        sub = [systems[k] for k in small]
        Bs = torch.from_numpy(np.ascontiguousarray(np.concatenate([probs[k].b for k in small], axis=0))).cuda()
        bt = cgmi.Batch(sub, 16)
        autotune.batch_schedule(bt, sub, Bs, store=False)
        bt.solve(Bs, torch.zeros_like(Bs), tol=1e-10, maxit=200000)
        solvers = [cgmi.Solver(systems[k]) for k in small]
        bsmall = [torch.from_numpy(np.ascontiguousarray(probs[k].b.T)).cuda() for k in small]
        speedups, t_bs, t_seps = [], [], []
        for _ in range(max(1, args.steps)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, rs, _, code = bt.solve(Bs, torch.zeros_like(Bs), tol=1e-10, maxit=200000)
            torch.cuda.synchronize()
            t_b = time.perf_counter() - t1
            t_sep, its = 0.0, 0
            for s, bk in zip(solvers, bsmall):
                for j in range(16):
                    xj = torch.zeros_like(bk[j])
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    _, r1 = s.solve(bk[j], xj, tol=1e-10, maxit=200000)
                    torch.cuda.synchronize()
                    t_sep += time.perf_counter() - t1
                    its += r1["iterations"]
            speedups.append(t_sep / t_b)
            t_bs.append(t_b)
            t_seps.append(t_sep)
        for s in solvers:
            s.close()
        bt.close()
        tol_cmp = {"systems": len(small), "pairs": 16 * len(small), "runs": len(speedups),
                   "batched_seconds_median": float(np.median(t_bs)),
                   "separate_seconds_median": float(np.median(t_seps)),
                   "speedup_min": float(min(speedups)), "speedup_median": float(np.median(speedups)),
                   "speedup_max": float(max(speedups)),
                   "batched_max_iterations": int(rs["iterations"].max()),
                   "separate_total_iterations": its, "all_converged": bool(np.all(rs["status"] == 0)),
                   "max_rel_res_true": float(rs["rel_res_true"].max())}
        print(f"[bench] to 1e-10, sides <= 64: {tol_cmp}", file=sys.stderr, flush=True)

    traffic = measured_traffic("batch_256", None, BATCH_SOURCES)
    line = _line("CG iters/s + SpMV GB/s (%HBM peak); time to 1e-10 residual, plain vs learned-PC",
                 value, "iter/s", args, 1e3 * elapsed / args.steps,
                 {"workload": "batch_256_diffusion2d_sides_32-512_16rhs_fp64_fixed_work",
                  "systems": len(systems), "nrhs": 16, "n_total": n_total, "nnz_total": nnz_total,
                  "iterations_per_step": K, "seed": 5},
                 value_meaning="(system, right-hand side) CG iterations per second, one persistent launch per step",
                 schedule=sched, kernel_seconds=t_k,
                 one_solve_per_launch=single,
                 speedup_vs_one_solve_per_launch=t_all / (elapsed / args.steps),
                 to_tolerance_small_systems=tol_cmp,
                 roofline=roofline_hbm(bytes_it * K, t_k, traffic, kernel="k_batch_cg (whole launch)",
                                       note="algorithmic bytes of all K iterations of one launch"))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(systems, probs, K, pairs)
    print(json.dumps(line), flush=True)
    return 0


def cpu_baseline_batch(systems, probs, K: int, pairs: int, target_s: float = 12.0) -> dict:
    """The oracle's CG on one right-hand side of sampled systems for K
    iterations; the batch's pair-iterations per second estimated from the
    per-row cost."""
    import numpy as np
    import oracle
    order = np.argsort([A.n for A in systems])
    picks = order[np.linspace(0, len(order) - 1, 5).astype(int)]
    secs, row_its, done = 0.0, 0, []
    rounds = 0
    while secs < target_s and rounds < 200:   # whole passes over the sampled systems
        for k in picks:
            t0 = time.perf_counter()
            oracle.cg(systems[k], probs[k].b[:, rounds % 16], tol=0.0, maxit=K)
            secs += time.perf_counter() - t0
            row_its += systems[k].n * K
        rounds += 1
    n_total = sum(A.n for A in systems)
    est = secs / row_its * n_total * 16 * K     # seconds for every pair, K iterations
    return {"value": pairs * K / est, "unit": "iter/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{rounds} passes of {K} fixed-work CG iterations over one right-hand side of "
                      f"systems {list(map(int, picks))} ({secs:.1f} s), scaled by rows to all 256 x 16 pairs"}


def cpu_baseline_pcg(prob, theta, iterations: int, target_s: float = 12.0) -> dict:
    """The oracle's PCG with the same learned factor (computed by the oracle's
    own network forward), timed on a bounded number of iterations and scaled
    to the iteration count the GPU solve needed."""
    import numpy as np
    import scipy.sparse as sp
    import oracle
    import oracle.fsai as OF
    from paper_2608_09647_amd import inputs as I
    A = prob.A
    o, _ = OF.mlp_forward(np.asarray(theta, np.float64), OF.features(A), round_bf16=True)
    Ahat, d = OF.scaled_operator(A)
    G = OF.g_unscaled(OF.g_tilde(A, o), d).tocsr()
    G.sort_indices()
    Gt = G.T.tocsr()
    Gt.sort_indices()
    Gc = I.CSR(A.n, G.indptr.astype(np.int32), G.indices.astype(np.int32), G.data)
    Gtc = I.CSR(A.n, Gt.indptr.astype(np.int32), Gt.indices.astype(np.int32), Gt.data)
    k = _sample_iterations(lambda m: oracle.pcg(A, Gc, Gtc, prob.b, tol=0.0, maxit=m), iterations,
                           target_s)
    t0 = time.perf_counter()
    out = oracle.pcg(A, Gc, Gtc, prob.b, tol=0.0, maxit=k)
    dt = time.perf_counter() - t0
    per_it = dt / max(out["iterations"], 1)
    return {"value": per_it * iterations, "unit": "s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{out['iterations']} fixed-work PCG iterations with the same factor "
                      f"({dt:.1f} s), scaled to the {iterations} iterations of the GPU solve"}


if __name__ == "__main__":
    sys.exit(main())
