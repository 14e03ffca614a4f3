"""Seeded synthetic inputs for the sparse CG path.

This module only *generates* problems: CSR matrices, manufactured solutions
x* and right-hand sides b = A x*.  It holds none of the solver's arithmetic
(no CG step, no preconditioner, no reduction of the method); both the CPU
oracle and the GPU library consume what it produces.  b is formed with
scipy.sparse, a third-party routine that neither side shares code with.

The paper (Section 4.1) measures on SuiteSparse matrices that are not
available here; the families below stand in for them and span the same
range of row lengths (about 5 to about 60 nonzeros per row):

* ``poisson2d`` / ``poisson3d``: Dirichlet 5-/7-point Laplacian, x-fastest
  ordering, values 4/-1 and 6/-1.
* ``random_spd_lognormal``: random symmetric diagonally dominant matrix with
  lognormal row degrees, uniform random columns and U[-1,0) off-diagonals,
  mirrored, diagonal = off-diagonal absolute row sum + shift.
* ``diffusion2d``: cell-centred finite-volume 5-point diffusion operator with
  harmonic-mean face transmissibilities on a log-normal coefficient field.

All CSR arrays use int32 row pointers / column indices and float64 values,
with columns sorted and unique inside each row (Section 3.2 stores the full
matrix in CSR).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    """A square CSR matrix (int32 indices, float64 values)."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _csr_from_slots(cols: np.ndarray, vals: np.ndarray, mask: np.ndarray) -> CSR:
    """Pack an (n, S) slot table (slots already in ascending column order)."""
    n = cols.shape[0]
    counts = mask.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    return CSR(n, row_ptr.astype(np.int32), cols[mask].astype(np.int32, copy=False),
               vals[mask].astype(np.float64, copy=False))


def poisson2d(nx: int, ny: int | None = None) -> CSR:
    """Dirichlet 5-point Laplacian on an nx*ny grid (diag 4, neighbours -1)."""
    ny = nx if ny is None else ny
    n = nx * ny
    i = np.arange(n, dtype=np.int64)
    ix, iy = i % nx, i // nx
    offs = [-nx, -1, 0, 1, nx]
    ok = [iy > 0, ix > 0, np.ones(n, bool), ix < nx - 1, iy < ny - 1]
    cols = np.stack([(i + o).astype(np.int32) for o in offs], axis=1)
    mask = np.stack(ok, axis=1)
    vals = np.full((n, 5), -1.0)
    vals[:, 2] = 4.0
    return _csr_from_slots(cols, vals, mask)


def poisson3d(nx: int, ny: int | None = None, nz: int | None = None) -> CSR:
    """Dirichlet 7-point Laplacian on an nx*ny*nz grid (diag 6, neighbours -1)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    pl = nx * ny
    i = np.arange(n, dtype=np.int64)
    ix, iy, iz = i % nx, (i // nx) % ny, i // pl
    del i
    cols = np.empty((n, 7), dtype=np.int32)
    mask = np.empty((n, 7), dtype=bool)
    base = np.arange(n, dtype=np.int32)
    for s, (o, ok) in enumerate([(-pl, iz > 0), (-nx, iy > 0), (-1, ix > 0), (0, None),
                                 (1, ix < nx - 1), (nx, iy < ny - 1), (pl, iz < nz - 1)]):
        cols[:, s] = base + np.int32(o)
        mask[:, s] = True if ok is None else ok
    del ix, iy, iz, base
    vals = np.full((n, 7), -1.0)
    vals[:, 3] = 6.0
    return _csr_from_slots(cols, vals, mask)


def random_spd_lognormal(n: int, seed: int, mean_degree: float = 30.0, sigma: float = 1.0,
                         max_degree: int = 2000, shift: float = 0.01) -> CSR:
    """Random symmetric, strictly diagonally dominant matrix.

    Row i draws d_i = clip(rint(LogNormal(mu, sigma)), 1, max_degree) columns
    uniformly among j != i, with mu chosen so that E[LogNormal] = mean_degree.
    Each draw (i, j, v), v ~ U[-1, 0), is mirrored to (j, i, v); coincident
    entries are summed.  The diagonal is the off-diagonal absolute row sum
    plus ``shift``, so A*1 = shift*1 and the smallest eigenvalue is ``shift``.
    """
    rng = np.random.default_rng([seed, 0])
    mu = math.log(mean_degree) - 0.5 * sigma * sigma
    deg = np.clip(np.rint(rng.lognormal(mu, sigma, size=n)), 1, max_degree).astype(np.int64)
    deg = np.minimum(deg, n - 1)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    cols = rng.integers(0, n - 1, size=rows.size, dtype=np.int64)
    cols += cols >= rows
    v = rng.uniform(-1.0, 0.0, size=rows.size)
    key = np.concatenate([rows * n + cols, cols * n + rows])
    del rows, cols
    vv = np.concatenate([v, v])
    del v
    order = np.argsort(key, kind="stable")
    key = key[order]
    vv = vv[order]
    del order
    first = np.empty(key.size, dtype=bool)
    first[0] = True
    np.not_equal(key[1:], key[:-1], out=first[1:])
    starts = np.flatnonzero(first)
    del first
    off_val = np.add.reduceat(vv, starts)
    del vv
    key = key[starts]
    del starts
    r = (key // n).astype(np.int64)
    c = (key % n).astype(np.int64)
    del key
    absrow = np.bincount(r, weights=np.abs(off_val), minlength=n)
    diag = absrow + shift
    cnt = np.bincount(r, minlength=n).astype(np.int64)
    lower = np.bincount(r, weights=(c < r), minlength=n).astype(np.int64)
    total = off_val.size + n
    if total >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt + 1, out=row_ptr[1:])
    col = np.empty(total, dtype=np.int32)
    val = np.empty(total, dtype=np.float64)
    pos = np.arange(off_val.size, dtype=np.int64) + r + (c > r)
    col[pos] = c
    val[pos] = off_val
    dpos = row_ptr[:-1] + lower
    col[dpos] = np.arange(n, dtype=np.int32)
    val[dpos] = diag
    return CSR(n, row_ptr.astype(np.int32), col, val)


def gaussian_weights(sigma: float, radius: int) -> np.ndarray:
    """Truncated Gaussian taps normalised to unit sum of squares."""
    t = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-0.5 * (t / sigma) ** 2)
    return w / math.sqrt(float(np.sum(w * w)))


def log_normal_field(nx: int, ny: int, seed, log_std: float = 2.0, smooth_sigma: float = 4.0,
                     radius: int = 16) -> np.ndarray:
    """Smoothed log-normal coefficient field k[iy, ix].

    iid N(0,1) cell values are filtered periodically by a separable Gaussian
    (std ``smooth_sigma`` cells, truncated at ``radius``) whose taps have unit
    sum of squares, so the smoothed field is again N(0,1) at every cell; then
    k = exp(log_std * z), i.e. marginals exp(N(0, log_std^2)).
    """
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((ny, nx))
    w = gaussian_weights(smooth_sigma, radius)
    for axis in (0, 1):
        acc = np.zeros_like(z)
        for t, wt in zip(range(-radius, radius + 1), w):
            acc += wt * np.roll(z, t, axis=axis)
        z = acc
    return np.exp(log_std * z)


def diffusion2d(k: np.ndarray) -> CSR:
    """Cell-centred 5-point finite-volume operator for -div(k grad u) = f.

    Unit cells; the face transmissibility between cells a and b is the
    harmonic mean 2 k_a k_b / (k_a + k_b); a boundary face (Dirichlet 0 at the
    half-cell distance) contributes 2 k to the diagonal.  Symmetric bit for
    bit, SPD, same pattern as ``poisson2d``.
    """
    ny, nx = k.shape
    n = nx * ny
    tx = 2.0 * k[:, :-1] * k[:, 1:] / (k[:, :-1] + k[:, 1:])   # face (ix, ix+1)
    ty = 2.0 * k[:-1, :] * k[1:, :] / (k[:-1, :] + k[1:, :])   # face (iy, iy+1)
    tw = np.empty((ny, nx)); tw[:, 0] = 2.0 * k[:, 0]; tw[:, 1:] = tx
    te = np.empty((ny, nx)); te[:, -1] = 2.0 * k[:, -1]; te[:, :-1] = tx
    ts = np.empty((ny, nx)); ts[0, :] = 2.0 * k[0, :]; ts[1:, :] = ty
    tn = np.empty((ny, nx)); tn[-1, :] = 2.0 * k[-1, :]; tn[:-1, :] = ty
    diag = ((tw + te) + (ts + tn)).reshape(n)
    i = np.arange(n, dtype=np.int64)
    ix, iy = i % nx, i // nx
    cols = np.stack([(i + o).astype(np.int32) for o in (-nx, -1, 0, 1, nx)], axis=1)
    mask = np.stack([iy > 0, ix > 0, np.ones(n, bool), ix < nx - 1, iy < ny - 1], axis=1)
    vals = np.stack([-ts.reshape(n), -tw.reshape(n), diag, -te.reshape(n), -tn.reshape(n)], axis=1)
    return _csr_from_slots(cols, vals, mask)


def uniform_vector(n: int, seed, nrhs: int | None = None) -> np.ndarray:
    """x* ~ U[-1, 1]; shape (n,) or (n, nrhs) (right-hand sides fastest)."""
    rng = np.random.default_rng(seed)
    shape = (n,) if nrhs is None else (n, nrhs)
    return rng.uniform(-1.0, 1.0, size=shape)


def rhs_of(A: CSR, xstar: np.ndarray) -> np.ndarray:
    """b = A x* via scipy.sparse (input preparation only)."""
    return np.ascontiguousarray(A.scipy() @ xstar)


# ----------------------------------------------------------------------------
# Named workloads.  ``scale`` shrinks a workload for quick parity cases while
# keeping its family, value law and seeds.
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    name: str
    A: CSR
    xstar: np.ndarray
    b: np.ndarray
    meta: dict


def poisson2d_problem(nx: int = 64, seed: int = 1) -> Problem:
    A = poisson2d(nx)
    xs = uniform_vector(A.n, [seed, 1])
    return Problem(f"poisson2d_{nx}x{nx}", A, xs, rhs_of(A, xs), {"nx": nx, "seed": seed})


def poisson3d_problem(nx: int = 256, seed: int = 2) -> Problem:
    A = poisson3d(nx)
    xs = uniform_vector(A.n, [seed, 1])
    return Problem(f"poisson3d_{nx}^3", A, xs, rhs_of(A, xs), {"nx": nx, "seed": seed})


def random_spd_problem(n: int = 2_000_000, seed: int = 3, max_degree: int = 2000) -> Problem:
    A = random_spd_lognormal(n, seed, max_degree=max_degree)
    xs = uniform_vector(A.n, [seed, 1])
    return Problem(f"random_spd_lognormal_n{n}", A, xs, rhs_of(A, xs),
                   {"n": n, "seed": seed, "max_degree": max_degree})


def diffusion_problem(nx: int = 1024, seed: int = 10_000) -> Problem:
    k = log_normal_field(nx, nx, [seed, 0])
    A = diffusion2d(k)
    xs = uniform_vector(A.n, [seed, 1])
    return Problem(f"diffusion2d_{nx}x{nx}", A, xs, rhs_of(A, xs),
                   {"nx": nx, "seed": seed, "k_min": float(k.min()), "k_max": float(k.max())})


def training_field(index: int, nx: int = 128) -> CSR:
    """Training system ``index`` (seeds 0..1999 at 128x128)."""
    return diffusion2d(log_normal_field(nx, nx, [index, 0]))


def batch_sides(nsys: int = 256, seed: int = 5, smin: int = 32, smax: int = 512) -> np.ndarray:
    rng = np.random.default_rng([seed, 0])
    return rng.integers(smin, smax + 1, size=nsys)


def batch_problem(nsys: int = 256, nrhs: int = 16, seed: int = 5, smin: int = 32,
                  smax: int = 512, sides=None) -> list:
    """Uneven batch of diffusion systems, each with ``nrhs`` right-hand sides.

    Returns a list of Problem whose xstar/b have shape (n, nrhs).
    """
    sides = batch_sides(nsys, seed, smin, smax) if sides is None else np.asarray(sides)
    out = []
    for s_idx, s in enumerate(sides):
        s = int(s)
        A = diffusion2d(log_normal_field(s, s, [seed, 1, s_idx]))
        xs = uniform_vector(A.n, [seed, 2, s_idx], nrhs=nrhs)
        out.append(Problem(f"batch{s_idx}_{s}x{s}", A, xs, rhs_of(A, xs), {"side": s}))
    return out
