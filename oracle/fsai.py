"""Learned factored sparse-approximate-inverse (FSAI) preconditioner oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy / scipy in
float64, with bfloat16 round-to-nearest-even applied explicitly at the points
where the GPU kernels round (network inputs, weights, hidden activations and
back-propagated signals), so the two can be compared element by element.

The preconditioner is M^-1 = G^T G with G lower triangular on the pattern of
tril(A).  For the 5-point operators used here a row i of G has the slots
C (i), W (i-1) and S (i-nx).  A small MLP 12 -> 64 -> 64 -> 5 maps per-row
features of the Jacobi-scaled operator A_hat = D^-1/2 A D^-1/2 to the outputs
[C, W, E, S, N]; the E and N outputs have no slot in tril(A) and are unused.

  G~_ii = softplus(o_C) + 1e-3,  G~_iW = o_W,  G~_iS = o_S,   G = G~ D^-1/2,

so G A G^T = G~ A_hat G~^T.  Training minimises, on a sample S of rows,

  L = (1/|S|) sum_{i in S} sum_j ((G~ A_hat G~^T)_ij - delta_ij)^2,

whose gradient is dL/dG~ = (2/|S|) (E + E^T) G~ A_hat restricted to the
pattern, E being G~ A_hat G~^T - I with the rows outside S zeroed.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

N_FEAT = 12
HIDDEN = 64
N_OUT = 5
SLOTS = ("C", "W", "E", "S", "N")
EPS_DIAG = 1e-3
SHAPES = [("W1", (HIDDEN, N_FEAT)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)),
          ("b2", (HIDDEN,)), ("W3", (N_OUT, HIDDEN)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)   # 5317


# ----------------------------------------------------------------------------- helpers

def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    """Flat parameter vector (W1, b1, W2, b2, W3, b3; row-major) -> dict."""
    theta = np.asarray(theta, dtype=np.float64)
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[k:k + size].reshape(shape)
        k += size
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def glorot_init(rng) -> np.ndarray:
    """Glorot-uniform weights, zero biases (the random numbers are the caller's)."""
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            p[name] = rng.uniform(-lim, lim, size=shape)
        else:
            p[name] = np.zeros(shape)
    return pack(p)


def softplus(x):
    return np.logaddexp(0.0, x)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


# ----------------------------------------------------------------------------- stencil slots and features

def slot_index(A) -> np.ndarray:
    """(n, 5) CSR positions of the C, W, E, S, N entries of each row (-1 if absent).

    For a row i of a 5-point operator in x-fastest order: column i is C, i-1 is
    W, i+1 is E, below i-1 is S, above i+1 is N."""
    n = A.n
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    c = A.col.astype(np.int64)
    slot = np.where(c == rows, 0, np.where(c == rows - 1, 1, np.where(c == rows + 1, 2,
                    np.where(c < rows, 3, 4))))
    idx = np.full((n, 5), -1, dtype=np.int64)
    pos = np.arange(c.size)
    key = rows * 5 + slot
    if np.unique(key).size != key.size:
        raise ValueError("matrix is not a 5-point operator: two entries share a stencil slot")
    idx.reshape(-1)[key] = pos
    return idx


def features(A) -> np.ndarray:
    """(n, 12) features of each row of A_hat = D^-1/2 A D^-1/2:
    [a_ij / sqrt(d_i d_j) for W, E, S, N;  log(d_j / d_i) for W, E, S, N;
     1 if the neighbour is absent for W, E, S, N]  (0 for absent neighbours)."""
    idx = slot_index(A)
    d = A.val[idx[:, 0]]
    F = np.zeros((A.n, N_FEAT))
    for s in range(4):
        k = idx[:, s + 1]
        have = k >= 0
        j = A.col[np.where(have, k, 0)]
        dj = d[j]
        F[:, s] = np.where(have, A.val[np.where(have, k, 0)] / np.sqrt(d * dj), 0.0)
        F[:, 4 + s] = np.where(have, np.log(dj / d), 0.0)
        F[:, 8 + s] = np.where(have, 0.0, 1.0)
    return F


# ----------------------------------------------------------------------------- network

def mlp_forward(theta, F, round_bf16: bool = True):
    """Outputs (n, 5) of the MLP; with round_bf16 the inputs, weights and hidden
    activations are rounded to bfloat16 (products and sums stay float64, biases
    are not rounded).  Returns (o, cache)."""
    p = unpack(theta)
    r = bf16 if round_bf16 else (lambda x: np.asarray(x, dtype=np.float64))
    f = r(F)
    z1 = f @ r(p["W1"]).T + p["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ r(p["W2"]).T + p["b2"]
    h2 = r(np.maximum(z2, 0.0))
    o = h2 @ r(p["W3"]).T + p["b3"]
    return o, {"f": f, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def mlp_backward(theta, F, dO, round_bf16: bool = True) -> np.ndarray:
    """Gradient of sum(dO * o) with respect to the flat parameters.

    The back-propagated signals entering a weight product (dO, dz2, dz1) are
    rounded to bfloat16 like the forward operands; bias gradients use the
    unrounded signals; ReLU passes gradient where its input was > 0."""
    p = unpack(theta)
    r = bf16 if round_bf16 else (lambda x: np.asarray(x, dtype=np.float64))
    _, c = mlp_forward(theta, F, round_bf16)
    dz3 = np.asarray(dO, dtype=np.float64)
    dz3r = r(dz3)
    g = {"W3": dz3r.T @ c["h2"], "b3": dz3.sum(axis=0)}
    dz2 = (dz3r @ r(p["W3"])) * (c["z2"] > 0)
    dz2r = r(dz2)
    g["W2"] = dz2r.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2r @ r(p["W2"])) * (c["z1"] > 0)
    dz1r = r(dz1)
    g["W1"] = dz1r.T @ c["f"]
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


# ----------------------------------------------------------------------------- factor and loss

def scaled_operator(A):
    """A_hat = D^-1/2 A D^-1/2 as scipy CSR, and d = diag(A)."""
    S = A.scipy()
    d = S.diagonal()
    s = 1.0 / np.sqrt(d)
    return sp.csr_matrix(sp.diags(s) @ S @ sp.diags(s)), d


def g_tilde(A, o) -> sp.csr_matrix:
    """G~ on the pattern of tril(A) from the network outputs o (n, 5)."""
    idx = slot_index(A)
    n = A.n
    rows, cols, vals = [], [], []
    i = np.arange(n)
    for s, value in ((3, o[:, 3]), (1, o[:, 1]), (0, softplus(o[:, 0]) + EPS_DIAG)):
        have = idx[:, s] >= 0
        rows.append(i[have])
        cols.append(A.col[idx[have, s]])
        vals.append(value[have])
    G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    G.sort_indices()
    return G


def g_unscaled(Gt: sp.csr_matrix, d) -> sp.csr_matrix:
    """G = G~ D^-1/2."""
    return sp.csr_matrix(Gt @ sp.diags(1.0 / np.sqrt(d)))


def loss_and_grad(Gt: sp.csr_matrix, Ahat: sp.csr_matrix, rows):
    """L and dL/dG~ (on G~'s pattern, as a CSR with G~'s structure)."""
    rows = np.asarray(rows)
    n = Gt.shape[0]
    M = (Gt @ Ahat @ Gt.T).tocsr()
    I = sp.identity(n, format="csr")
    sub = (M[rows] - I[rows]).tocsr()
    E = sp.csr_matrix((sub.data, sub.indices, sub.indptr), shape=(rows.size, n))
    P = sp.csr_matrix((np.ones(rows.size), (rows, np.arange(rows.size))), shape=(n, rows.size))
    Ebar = (P @ E).tocsr()
    L = float(E.multiply(E).sum()) / rows.size
    full = ((2.0 / rows.size) * ((Ebar + Ebar.T) @ Gt @ Ahat)).tocsr()
    G = Gt.tocsr()
    G.sort_indices()
    r = np.repeat(np.arange(n), np.diff(G.indptr))
    vals = np.asarray(full[r, G.indices]).reshape(-1)
    return L, sp.csr_matrix((vals, G.indices.copy(), G.indptr.copy()), shape=G.shape)


def grad_outputs(A, o, dG: sp.csr_matrix) -> np.ndarray:
    """dL/do (n, 5) from dL/dG~ through the slot map and the softplus."""
    idx = slot_index(A)
    n = A.n
    dO = np.zeros((n, N_OUT))
    dGd = dG.tocsr()
    for s in (0, 1, 3):
        have = idx[:, s] >= 0
        i = np.arange(n)[have]
        j = A.col[idx[have, s]]
        vals = np.asarray(dGd[i, j]).reshape(-1)
        dO[have, s] = vals * (sigmoid(o[have, 0]) if s == 0 else 1.0)
    return dO


def network_loss(theta, A, rows, round_bf16: bool = True):
    """Whole chain: features -> MLP -> G~ -> L.  Returns L and dL/dtheta."""
    F = features(A)
    o, _ = mlp_forward(theta, F, round_bf16)
    Ahat, _ = scaled_operator(A)
    Gt = g_tilde(A, o)
    L, dG = loss_and_grad(Gt, Ahat, rows)
    dO = grad_outputs(A, o, dG)
    return L, mlp_backward(theta, F, dO, round_bf16)


def network_loss_multi(theta, systems, rows_list, round_bf16: bool = True):
    """The training loss over several systems: the mean over every sampled
    row of all systems together, (1/|S|) sum over S = S_1 + ... + S_k.  The
    signal dL/do of each row therefore carries the factor 1/|S|, and the
    backward pass runs once over all rows, so its bfloat16 rounding points see
    that signal (rounding each system's own mean and averaging would round
    differently).  Returns L and dL/dtheta."""
    total = sum(np.asarray(r).size for r in rows_list)
    F_all, dO_all, L = [], [], 0.0
    for A, rows in zip(systems, rows_list):
        rows = np.asarray(rows)
        F = features(A)
        o, _ = mlp_forward(theta, F, round_bf16)
        Ahat, _ = scaled_operator(A)
        Gt = g_tilde(A, o)
        Lk, dG = loss_and_grad(Gt, Ahat, rows)          # mean over this system's rows
        w = rows.size / total
        L += w * Lk
        F_all.append(F)
        dO_all.append(w * grad_outputs(A, o, dG))
    return L, mlp_backward(theta, np.concatenate(F_all), np.concatenate(dO_all), round_bf16)


def adam_step(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------- reference factors

def classic_fsai(A) -> sp.csr_matrix:
    """Non-learned FSAI on the tril(A) pattern (Kolotilina-Yeremin): row i
    solves A[P_i, P_i] g = e_i over its pattern P_i and is scaled by
    1/sqrt(g_i), so G A G^T has a unit diagonal.  Returns G (unscaled)."""
    S = A.scipy().tocsr()
    L = sp.tril(S).tocsr()
    rows, cols, vals = [], [], []
    for i in range(A.n):
        P = L.indices[L.indptr[i]:L.indptr[i + 1]]
        sub = S[P][:, P].toarray()
        e = np.zeros(P.size)
        e[-1] = 1.0                    # i is the last (largest) column of tril row i
        g = np.linalg.solve(sub, e)
        g = g / np.sqrt(g[-1])
        rows += [i] * P.size
        cols += list(P)
        vals += list(g)
    G = sp.csr_matrix((vals, (rows, cols)), shape=(A.n, A.n))
    G.sort_indices()
    return G


def csr_parts(M: sp.csr_matrix):
    """(row_ptr int32, col int32, val float64) of a scipy CSR, sorted."""
    M = M.tocsr()
    M.sort_indices()
    return M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64)
