"""Schedule autotuner for the batched persistent solve and for the SpMV
tiling of single-system solves.

Both tuners time short fixed-work solves (tol = 0, a fixed iteration count,
so every candidate does identical arithmetic) for each candidate schedule on
the caller's own inputs and keep the fastest.  Results are stored in a JSON
table keyed by a workload signature (sizes and row-length statistics), so a
later run on a workload of the same shape looks the schedule up instead of
searching again.  Every candidate is a documented option of the C ABI
(cg_batch_sched, cg_opts.spmv_kind / spmv_grid); nothing outside those
bounds is launched.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

import numpy as np

from . import cgmi

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_schedules.json")


# ----------------------------------------------------------------------------- signatures

def _size_hist(sizes) -> list:
    """Counts of sizes per power-of-two bucket (log2 of the row count)."""
    b = np.floor(np.log2(np.maximum(np.asarray(sizes, np.float64), 1))).astype(int)
    lo, hi = int(b.min()), int(b.max())
    return [lo, [int((b == v).sum()) for v in range(lo, hi + 1)]]


def batch_signature(systems, nrhs: int) -> str:
    n = [int(A.n) for A in systems]
    nnz = sum(int(A.row_ptr[-1]) for A in systems)
    return json.dumps({"kind": "batch", "nsys": len(n), "nrhs": int(nrhs), "rows_log2": _size_hist(n),
                       "nnz_per_row": round(nnz / max(sum(n), 1), 1)}, sort_keys=True)


def matrix_signature(A) -> str:
    lens = np.diff(np.asarray(A.row_ptr, np.int64))
    return json.dumps({"kind": "spmv", "n_log2": int(math.log2(max(A.n, 1))),
                       "mean_len": round(float(lens.mean()), 1) if lens.size else 0.0,
                       "max_len_log2": int(math.log2(max(int(lens.max()) if lens.size else 1, 1))),
                       "cv_len": round(float(lens.std() / max(lens.mean(), 1e-12)), 1) if lens.size else 0.0},
                      sort_keys=True)


# ----------------------------------------------------------------------------- table

def load_table(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_table(table: dict, path: str = TABLE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(signature: str, path: str = TABLE):
    ent = load_table(path).get(signature)
    return None if ent is None else ent["best"]


# ----------------------------------------------------------------------------- batch

# max_team bounds a system's team: every team barrier costs a round trip
# through memory shared by the team's workgroups, so systems that converge
# in many short iterations may run faster on fewer workgroups
BATCH_SPACE = {"blocks_per_cu": [4, 8], "rows_per_thread": [1, 2], "team_exponent": [1.0, 1.25],
               "rhs_per_lane": [1, 2], "max_team": [0, 8, 32]}


def batch_candidates(space: dict | None = None) -> list:
    space = BATCH_SPACE if space is None else space
    keys = sorted(space)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(space[k] for k in keys))]


def tune_batch(batch: "cgmi.Batch", B, iters: int = 10, reps: int = 2, space: dict | None = None,
               log=None) -> dict:
    """Time every candidate schedule on `batch` with right-hand sides B
    (fixed work: tol = 0, `iters` iterations per pair); returns
    {"best": schedule dict, "seconds": best time, "trials": [...]}."""
    import torch
    trials = []
    X = torch.zeros_like(B)
    for cand in batch_candidates(space):
        batch.set_sched(**cand)
        times = []
        for _ in range(reps):
            X.zero_()
            _, _, st, _ = batch.solve(B, X, tol=0.0, maxit=iters)
            times.append(st["t_kernel"])
        t = float(min(times))
        trials.append({"sched": dict(cand), "seconds": t, "grid": st["grid"], "max_team": st["max_team"]})
        if log:
            log(f"batch {cand}: {1e3 * t:.2f} ms for {iters} iterations (grid {st['grid']})")
    best = min(trials, key=lambda r: r["seconds"])
    batch.set_sched(**best["sched"])
    return {"best": best["sched"], "seconds": best["seconds"], "iters": iters, "trials": trials}


def batch_schedule(batch: "cgmi.Batch", systems, B, tune_if_missing: bool = True, store: bool = True,
                   path: str = TABLE, log=None) -> dict:
    """The tabled schedule for this batch's signature (tuning and storing it
    when absent); the schedule is applied to `batch`."""
    sig = batch_signature(systems, batch.nrhs)
    best = lookup(sig, path)
    source = "table"
    if best is None:
        if not tune_if_missing:
            return {"sched": batch.sched.as_dict(), "source": "default"}
        res = tune_batch(batch, B, log=log)
        best = res["best"]
        source = "tuned"
        if store:
            table = load_table(path)
            table[sig] = {"best": best, "seconds": res["seconds"], "iters": res["iters"],
                          "trials": res["trials"], "when": time.strftime("%Y-%m-%d")}
            save_table(table, path)
    batch.set_sched(**best)
    return {"sched": dict(best), "source": source}


# ----------------------------------------------------------------------------- single-system SpMV tiling

SPMV_KINDS = {1: "vector_bins", 2: "stream", 3: "sliced", 4: "sliced_dict", 5: "column_blocks",
              6: "stencil_slices", 7: "gap_slices"}


def tune_spmv(solver: "cgmi.Solver", b, iters: int = 20, grids=(0, 1024, 2048, 4096), reps: int = 3,
              log=None) -> dict:
    """Fixed-work CG timings of each SpMV tiling and grid on `solver`: the
    SpMV's own time (HIP events) and the whole iteration's (wall clock, best
    of `reps`, no events); the best iteration wins, since the SpMV grid also
    sets how many partials the next kernel sums."""
    import time
    import torch
    trials = []
    for kind, grid in itertools.product(SPMV_KINDS, grids):
        try:
            solver.set_opts(spmv_kind=kind, spmv_grid=grid, profile=1)
        except cgmi.CgError:
            continue   # tiling not applicable to this matrix
        x = torch.zeros_like(b)
        solver.solve(b, x, tol=0.0, maxit=2)
        x.zero_()
        _, res = solver.solve(b, x, tol=0.0, maxit=iters)
        t = res["t_spmv"] / max(res["n_spmv"], 1)
        solver.set_opts(spmv_kind=kind, spmv_grid=grid, profile=0)
        it_best = float("inf")
        for _ in range(reps):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solver.solve(b, x, tol=0.0, maxit=iters)
            torch.cuda.synchronize()
            it_best = min(it_best, (time.perf_counter() - t0) / iters)
        trials.append({"spmv_kind": kind, "spmv_grid": grid, "spmv_us": 1e6 * t, "iter_us": 1e6 * it_best,
                       "chosen_kind": res["spmv_kind"]})
        if log:
            log(f"spmv kind {SPMV_KINDS[kind]} grid {grid}: SpMV {1e6 * t:.1f} us, iteration {1e6 * it_best:.1f} us")
    best = min(trials, key=lambda r: r["iter_us"])
    solver.set_opts(spmv_kind=best["spmv_kind"], spmv_grid=best["spmv_grid"])
    return {"best": {"spmv_kind": best["spmv_kind"], "spmv_grid": best["spmv_grid"]},
            "spmv_us": best["spmv_us"], "iter_us": best["iter_us"], "trials": trials}


def spmv_schedule(solver: "cgmi.Solver", A, b, tune_if_missing: bool = True, store: bool = True,
                  path: str = TABLE, log=None) -> dict:
    sig = matrix_signature(A)
    best = lookup(sig, path)
    source = "table"
    if best is None:
        if not tune_if_missing:
            return {"sched": {}, "source": "default"}
        res = tune_spmv(solver, b, log=log)
        best = res["best"]
        source = "tuned"
        if store:
            table = load_table(path)
            table[sig] = {"best": best, "spmv_us": res["spmv_us"], "trials": res["trials"],
                          "when": time.strftime("%Y-%m-%d")}
            save_table(table, path)
    solver.set_opts(**best)
    return {"sched": dict(best), "source": source}


# ----------------------------------------------------------------------------- offline sweep

def main(argv=None) -> int:
    """Tune the standard workloads on this GPU and write the table:
    python -m paper_2608_09647_amd.autotune --out <path>"""
    import argparse
    import sys

    import torch

    from . import inputs as I
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--workloads", default="batch_256,poisson3d_256,random_spd_2m,diffusion_1024")
    args = ap.parse_args(argv)
    log = lambda s: print(f"[tune] {s}", flush=True)  # noqa: E731
    table = load_table(args.out)
    for name in args.workloads.split(","):
        t0 = time.perf_counter()
        if name == "batch_256":
            probs = I.batch_problem(256, 16, seed=5)
            systems = [p.A for p in probs]
            B = torch.from_numpy(np.ascontiguousarray(np.concatenate([p.b for p in probs], axis=0))).cuda()
            with cgmi.Batch(systems, 16) as b:
                res = tune_batch(b, B, log=log)
            table[batch_signature(systems, 16)] = {"best": res["best"], "seconds": res["seconds"],
                                                   "iters": res["iters"], "trials": res["trials"],
                                                   "workload": name, "when": time.strftime("%Y-%m-%d")}
            del B
        else:
            prob = {"poisson3d_256": lambda: I.poisson3d_problem(256, seed=2),
                    "random_spd_2m": lambda: I.random_spd_problem(2_000_000, seed=3),
                    "diffusion_1024": lambda: I.diffusion_problem(1024, seed=10_000)}[name]()
            b = torch.from_numpy(prob.b).cuda()
            with cgmi.Solver(prob.A) as s:
                res = tune_spmv(s, b, log=log)
            table[matrix_signature(prob.A)] = {"best": res["best"], "spmv_us": res["spmv_us"],
                                               "iter_us": res["iter_us"],
                                               "trials": res["trials"], "workload": name,
                                               "when": time.strftime("%Y-%m-%d")}
            del b
        torch.cuda.empty_cache()
        save_table(table, args.out)
        log(f"{name}: best {table and res['best']} ({time.perf_counter() - t0:.1f}s)")
    print(json.dumps({k: v["best"] for k, v in table.items()}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
