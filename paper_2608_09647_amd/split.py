"""Planning of the CPU-GPU row split.

The GPU owns rows [0, n_gpu) and host threads the rest (Section 3.2); p is
made visible to both sides by one of the Section 3.4 memory modes (explicit
copy of whole segments or of the halo, or one copy in mapped host memory).
The paper sweeps fixed GPU fractions g under each memory mode and calls a
configuration competitive when its run time is within 1.25x of the best one
for the matrix (Section 4.1); it notes that equal row shares need not be
equal work, and leaves the automatic choice of partition and memory strategy
to future work (Section 5).  This module holds that bookkeeping and a simple
automatic choice:

* split points: ``rows_for_share`` (g of the rows, rounded half away from
  zero, the paper's split) and ``rows_for_nnz_share`` (g of the nonzeros);
* ``competitive``: the 1.25x classification of measured configurations;
* ``IterationModel``: per-iteration time of a split solve, fitted from the
  timers of one probe solve (cg_result.t_gpu, t_cpu, t_d2h, t_h2d and the
  wall time) at one split and mode:
      T(g) = max(nnz_gpu(g) / R_gpu, nnz_cpu(g) / R_cpu) + E(g) + O
  with R_gpu, R_cpu the nonzeros per second each side sustained, E the
  exchange time per iteration (0 at g = 0 and g = 1, where nothing is
  exchanged) and O the rest (reductions, synchronisation);
* ``choose_split``: the candidate share with the smallest predicted time
  for one mode's model; ``choose_config`` the best (mode, share) over
  several modes' models;
* ``transfer_bound``: the interconnect-bound estimate of Section 4.4, where
  only the vector-transfer part of an explicit-copy run time is divided by
  a bandwidth ratio R (the paper's R = 900 / 128, a coherent 900 GB/s link
  over PCIe Gen5 x16's 128 GB/s, which is also this GPU's host link).

Everything here is host arithmetic on timings; the solves it plans run in
the library's kernels and host loops.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SHARES = (0.0, 0.25, 0.5, 0.75, 0.8, 0.85, 0.9, 0.95, 1.0)
COMPETITIVE_FACTOR = 1.25
LINK_RATIO = 900.0 / 128.0


def rows_for_share(n: int, g: float) -> int:
    """round(g n) with halves rounded away from zero (GPU rows [0, n_gpu))."""
    if not 0.0 <= g <= 1.0:
        raise ValueError("share must lie in [0, 1]")
    return min(n, int(math.floor(g * n + 0.5)))


def rows_for_nnz_share(row_ptr, g: float) -> int:
    """Smallest n_gpu whose rows [0, n_gpu) hold at least g of the nonzeros."""
    if not 0.0 <= g <= 1.0:
        raise ValueError("share must lie in [0, 1]")
    rp = np.asarray(row_ptr, dtype=np.int64)
    target = g * float(rp[-1])
    return int(np.searchsorted(rp, target, side="left"))


def competitive(times: dict, factor: float = COMPETITIVE_FACTOR) -> dict:
    """{key: True when times[key] <= factor * min(times)}; non-finite times
    are never competitive."""
    finite = [t for t in times.values() if t is not None and math.isfinite(t)]
    if not finite:
        return {k: False for k in times}
    best = min(finite)
    return {k: (t is not None and math.isfinite(t) and t <= factor * best) for k, t in times.items()}


@dataclass
class IterationModel:
    gpu_rate: float    # nonzeros per second on the GPU side
    cpu_rate: float    # nonzeros per second on the host side
    exchange: float    # seconds per iteration making p visible (split only)
    other: float       # seconds per iteration outside compute and exchange
    nnz: int           # nonzeros of the whole matrix

    @classmethod
    def fit(cls, probe: dict, seconds: float, nnz: int) -> "IterationModel":
        """probe: cg_result fields of a split solve (0 < rows_gpu < n) that ran
        probe['iterations'] iterations in `seconds` of wall time."""
        it = max(int(probe["iterations"]), 1)
        ng, nc = int(probe["nnz_gpu"]), int(probe["nnz_cpu"])
        if ng <= 0 or nc <= 0:
            raise ValueError("the probe must split the rows between GPU and host")
        tg, tc = probe["t_gpu"] / it, probe["t_cpu"] / it
        if tg <= 0 or tc <= 0:
            raise ValueError("the probe's GPU and host times must be positive")
        ex = (probe["t_d2h"] + probe["t_h2d"]) / it
        wall = seconds / it
        return cls(gpu_rate=ng / tg, cpu_rate=nc / tc, exchange=ex,
                   other=max(0.0, wall - max(tg, tc) - ex), nnz=int(nnz))

    def predict(self, nnz_gpu: int) -> float:
        """Seconds per iteration with nnz_gpu nonzeros on the GPU."""
        nnz_gpu = min(max(int(nnz_gpu), 0), self.nnz)
        nnz_cpu = self.nnz - nnz_gpu
        t = max(nnz_gpu / self.gpu_rate, nnz_cpu / self.cpu_rate)
        if 0 < nnz_gpu < self.nnz:
            t += self.exchange
        return t + self.other


def choose_split(model: IterationModel, row_ptr, shares=SHARES, by_nnz: bool = False) -> dict:
    """Candidate share with the smallest predicted time per iteration.
    Returns {"share", "rows_gpu", "nnz_gpu", "predicted", "table"}."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    n = rp.size - 1
    table = []
    for g in shares:
        rows = rows_for_nnz_share(rp, g) if by_nnz else rows_for_share(n, g)
        nz = int(rp[rows])
        table.append({"share": float(g), "rows_gpu": rows, "nnz_gpu": nz, "predicted": model.predict(nz)})
    best = min(table, key=lambda r: (r["predicted"], -r["share"]))
    return {**best, "table": table}


def choose_config(models: dict, row_ptr, shares=SHARES, by_nnz: bool = False) -> dict:
    """models: {mode name: IterationModel}.  The (mode, share) with the
    smallest predicted time: {"mode", "share", "rows_gpu", "nnz_gpu",
    "predicted", "per_mode": {mode: choose_split result}}."""
    per = {m: choose_split(md, row_ptr, shares, by_nnz) for m, md in models.items()}
    mode = min(per, key=lambda m: per[m]["predicted"])
    best = {k: v for k, v in per[mode].items() if k != "table"}
    return {"mode": mode, **best, "per_mode": per}


def transfer_bound(seconds: float, transfer_seconds: float, ratio: float = LINK_RATIO) -> float:
    """Run time with the transfer component (initial, final and per-iteration
    vector copies) scaled by 1 / ratio and everything else unchanged."""
    if ratio <= 0:
        raise ValueError("ratio must be positive")
    if not 0.0 <= transfer_seconds <= seconds:
        raise ValueError("the transfer time must lie within the run time")
    return seconds - transfer_seconds + transfer_seconds / ratio


def transfer_bound_table(runs: dict, ratio: float = LINK_RATIO) -> dict:
    """runs: {key: {"seconds", "t_d2h", "t_h2d"}} of explicit-copy (or
    transfer-free) configurations.  Returns the bound per key and the
    preferred key before and after scaling."""
    bound = {k: transfer_bound(r["seconds"], min(r["t_d2h"] + r["t_h2d"], r["seconds"]), ratio)
             for k, r in runs.items()}
    before = min(runs, key=lambda k: runs[k]["seconds"])
    after = min(bound, key=bound.get)
    return {"ratio": ratio, "bound_seconds": bound, "preferred_measured": before,
            "preferred_bound": after, "preferred_changes": before != after}
