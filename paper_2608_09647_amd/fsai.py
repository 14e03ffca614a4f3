"""Learned FSAI preconditioner: parameter initialisation and the training loop.

The network, loss, gradients and Adam steps all run in libcgmi (include/
cgmi_fsai.h); this module draws the random numbers (initial weights, sampled
systems and rows) and drives the steps.  Training systems are the seeded
2-D log-normal diffusion operators of ``inputs.training_field``.
"""
from __future__ import annotations

import time

import numpy as np

from . import cgmi, inputs

N_FEAT, HIDDEN, N_OUT = 12, 64, 5
SHAPES = [(HIDDEN, N_FEAT), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (N_OUT, HIDDEN), (N_OUT,)]


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights (limit sqrt(6 / (fan_in + fan_out))), zero biases,
    flat float32 in the order W1, b1, W2, b2, W3, b3."""
    rng = np.random.default_rng([seed, 7])
    parts = []
    for shape in SHAPES:
        if len(shape) == 2:
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(rng.uniform(-lim, lim, size=shape).reshape(-1))
        else:
            parts.append(np.zeros(shape))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == cgmi.FSAI_NPARAMS
    return theta


def training_systems(count: int = 2000, nx: int = 128, first: int = 0) -> list:
    """The training operators with seeds first .. first + count - 1."""
    return [inputs.training_field(first + i, nx) for i in range(count)]


def sample(rng, sizes, nsel: int, rows_per: int):
    """nsel distinct systems and rows_per distinct rows of each."""
    sys = rng.choice(len(sizes), size=min(nsel, len(sizes)), replace=False).astype(np.int32)
    rows = np.stack([rng.choice(sizes[s], size=min(rows_per, sizes[s]), replace=False)
                     for s in sys]).astype(np.int32)
    return sys, rows


def _sampler(seed: int, start: int, sizes, nsel: int, rows_per: int):
    """The sample generator of a run with this seed, advanced past its first
    `start` steps (so a resumed run draws the samples the uninterrupted run
    would have drawn)."""
    rng = np.random.default_rng([seed, 11])
    for _ in range(start):
        sample(rng, sizes, nsel, rows_per)
    return rng


def train(trainer: "cgmi.FsaiTrainer", steps: int, nsel: int = 8, rows_per: int = 1024,
          lr: float = 1e-3, seed: int = 0, lr_final: float | None = None, log=None,
          start: int = 0, total: int | None = None) -> dict:
    """Adam steps on random (system, rows) samples.  With lr_final the
    learning rate decays geometrically from lr to lr_final over `total`
    steps (default: steps).  start > 0 resumes a run of `total` steps after
    its first `start` steps (a trainer restored by load_checkpoint): the
    samples and learning rates are those of the uninterrupted run.  Returns
    the loss history and timing."""
    total = steps + start if total is None else total
    rows_per = min(rows_per, min(trainer.sizes))
    rng = _sampler(seed, start, trainer.sizes, nsel, rows_per)
    losses = []
    t0 = time.perf_counter()
    decay = 1.0 if lr_final is None or total <= 1 else (lr_final / lr) ** (1.0 / (total - 1))
    for k in range(start, start + steps):
        sys, rows = sample(rng, trainer.sizes, nsel, rows_per)
        losses.append(trainer.step(sys, rows, lr * decay ** k))
        if log and (k % max(1, total // 10) == 0 or k == start + steps - 1):
            log(f"step {k}: loss {losses[-1]:.4e}")
    return {"losses": losses, "seconds": time.perf_counter() - t0, "steps": steps, "start": start,
            "total": total, "nsel": nsel, "rows_per": rows_per, "lr": lr, "lr_final": lr_final}


def save_checkpoint(path: str, trainer: "cgmi.FsaiTrainer", seed: int, **meta) -> None:
    """theta, Adam's m and v, the step count and the sampling seed in one
    .npz (plain arrays, no pickled objects); meta adds scalar settings."""
    st = trainer.state()
    extra = {k: np.asarray(v) for k, v in meta.items()}
    np.savez(path, theta=st["theta"], m=st["m"], v=st["v"], step=np.int64(st["step"]),
             seed=np.int64(seed), **extra)


def load_checkpoint(path: str, trainer: "cgmi.FsaiTrainer" | None = None) -> dict:
    """Read a checkpoint (allow_pickle off); with a trainer, restore its state."""
    with np.load(path, allow_pickle=False) as z:
        ck = {k: z[k] for k in z.files}
    ck["step"], ck["seed"] = int(ck["step"]), int(ck["seed"])
    if trainer is not None:
        trainer.set_state(ck["theta"], ck["m"], ck["v"], ck["step"])
    return ck
