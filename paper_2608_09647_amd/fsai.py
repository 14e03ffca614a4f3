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


def train(trainer: "cgmi.FsaiTrainer", steps: int, nsel: int = 8, rows_per: int = 1024,
          lr: float = 1e-3, seed: int = 0, lr_final: float | None = None, log=None) -> dict:
    """Adam steps on random (system, rows) samples.  With lr_final the
    learning rate decays geometrically from lr to lr_final.  Returns the loss
    history and timing."""
    rng = np.random.default_rng([seed, 11])
    rows_per = min(rows_per, min(trainer.sizes))
    losses = []
    t0 = time.perf_counter()
    decay = 1.0 if lr_final is None or steps <= 1 else (lr_final / lr) ** (1.0 / (steps - 1))
    for k in range(steps):
        sys, rows = sample(rng, trainer.sizes, nsel, rows_per)
        losses.append(trainer.step(sys, rows, lr * decay ** k))
        if log and (k % max(1, steps // 10) == 0 or k == steps - 1):
            log(f"step {k}: loss {losses[-1]:.4e}")
    return {"losses": losses, "seconds": time.perf_counter() - t0, "steps": steps,
            "nsel": nsel, "rows_per": rows_per, "lr": lr, "lr_final": lr_final}
